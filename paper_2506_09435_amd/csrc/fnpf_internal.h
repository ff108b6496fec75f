// Internal declarations shared by the host driver and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fnpf.h"
#include "partials.h"

namespace fnpf {

constexpr int kMaxP = 8;
constexpr int kMaxN1 = kMaxP + 1;
constexpr int kDStride = kMaxN1 * kMaxN1;  // per-degree stride of the D tables
constexpr uint8_t kFirst = 1;              // column is the first writer of this horizontal node
constexpr uint8_t kLast = 2;               // column is the last writer (sees the final sum)
constexpr uint8_t kOwned = 4;              // column owns this horizontal node (owner-computes apply)
constexpr uint8_t kShared = 8;             // the node belongs to more than one column
// tile assembly of the owner-computes apply (a tile = the columns of one workgroup)
constexpr uint8_t kTRep = 16;              // the column sums this node's contributions in its tile
constexpr uint8_t kTOwn = 32;              // ... and its tile owns the node (stores y there)
constexpr uint8_t kTShared = 64;           // the node also receives face slots of other tiles

// Horizontal metric components stored per (column, local horizontal node).
// 3D: A = J_h^{-1} (A00, A01, A10, A11), det J_h, J_h (x_xi, x_eta, y_xi, y_eta).
// 2D: 1/x_xi, x_xi.
constexpr int kHm3 = 9;
constexpr int kHm2 = 2;

// Device-side PCG scalars (FP64 even for the FP32 inner solve).
struct PcgScalars {
  double rz;       // r^T z of the current iterate
  double rr;       // r^T r of the current iterate
  double pq;       // p^T A p
  double alpha;
  double beta;
  double tol2;     // squared absolute stopping threshold
  double bnorm2;   // ||b||^2
  double rr0;      // r^T r at the start of this (inner) solve
  int32_t done;
  int32_t iters;
  int32_t breakdown;
  int32_t pad;
};

// Launch helpers for one colour of the column colouring.
struct ColourRange {
  int32_t offset;
  int32_t count;
};

template <typename T>
struct DevBuf {
  T *ptr = nullptr;
  size_t n = 0;
};

struct Ctx;

// Kernel launchers (kernels_*.hip). All return hipSuccess or the launch error.
hipError_t upload_constants(int device);
// The allocation-free apply's face-slot scratch: a file-scope device array of
// noalloc_scratch_bytes(); init_noalloc_scratch looks up its address on the current device (once
// per device, at context creation) and noalloc_scratch returns it (nullptr before).
hipError_t init_noalloc_scratch(int device);
void *noalloc_scratch(int device);
size_t noalloc_scratch_bytes();
// full_diag: store the assembled diagonal at every node (it is also stored when store_G or
// c.keep_diag); otherwise the owner-computes path keeps only what its inverses need
hipError_t launch_geom(Ctx &c, const double *eta, const double *h, bool store_G, bool h_is_total,
                       hipStream_t s, bool full_diag = false);
// the assembled diagonal d_diag at every node, recomputed from the saved column data if the last
// geometry update did not store it
hipError_t ensure_diag(Ctx &c, hipStream_t s);
hipError_t launch_apply(Ctx &c, fnpf_dtype dt, const void *x, void *y, bool mask, double *partial,
                        const int32_t *skip, hipStream_t s, void *face_scratch = nullptr);
hipError_t launch_neumann(Ctx &c, const double *q, double *f, hipStream_t s);
hipError_t launch_wsurf(Ctx &c, const double *phi, double *w, hipStream_t s);
struct RkStageArgs {
  const double *eta0;   // state at the start of the step
  const double *phi0;
  double *acc_e;        // stage accumulators
  double *acc_p;
  double *out_e;        // next stage state (stage < 3) or the final state (stage 3, may alias eta0)
  double *out_p;
  double bdt;           // b_s dt
  double cdt;           // c_{s+1} dt (stage < 3)
  int stage;            // 0..3, or -1: plain RHS into out_e/out_p
  // relaxation (stage 3 only): f <- (1-cr) f + cr (rc f_c + rs f_s)
  const double *cr, *ec, *es, *pc, *ps;
  double rc, rs;
  int linear;           // linear potential flow: d eta/dt = w, d phi_s/dt = -g eta
};
hipError_t launch_rhs(Ctx &c, const double *eta, const double *phi_s, const double *w, const RkStageArgs &a,
                      hipStream_t s);

// adjoint kernels (adjoint_kernels.inc); outputs are accumulated
hipError_t launch_rhs_vjp(Ctx &c, const double *eta, const double *phs, const double *w, const double *kbe,
                          const double *kbp, double *eta_bar, double *phs_bar, double *w_bar, hipStream_t s);
hipError_t launch_wsurf_vjp(Ctx &c, const double *wbar, const double *w, double *phi_bar, double *eta_bar,
                            double *h_bar, hipStream_t s);
hipError_t launch_geom_vjp(Ctx &c, const double *lam, const double *phi, double *eta_bar, double *h_bar,
                           hipStream_t s);

// vector kernels (kernels_vec.hip)
// consistent over-integrated free-surface form
constexpr int kMaxSurfaceNq = 24;
const char *sq_setup(Ctx &c, int nq);
void sq_free(Ctx &c);
hipError_t launch_sq_rhs(Ctx &c, const double *eta, const double *phs, const double *w, double *b, hipStream_t s);
hipError_t launch_sq_rhs_vjp(Ctx &c, const double *eta, const double *phs, const double *w, const double *bbar,
                             double *eta_bar, double *phi_bar, double *w_bar, hipStream_t s);
hipError_t sq_solve(Ctx &c, const double *b, double *x, hipStream_t s);
hipError_t launch_sq_stage(const RkStageArgs &a, const double *k2, int64_t n_s, hipStream_t s);
hipError_t launch_sq_pack(const double *a, const double *b, double *out, int64_t n_s, hipStream_t s);
// modal filter (forward: out = W (M x M) in, out != in; transpose: in_bar += (M x M)^T W out_bar)
hipError_t launch_modal_filter(Ctx &c, const double *in, double *out, bool transpose, hipStream_t s);
void modal_filter_matrix(int p, int cutoff, double alpha, int order, double *M);
hipError_t launch_rhs_vjp_linear(const double *kbe, const double *kbp, double *eta_bar, double *w_bar, double g,
                                 int64_t n, hipStream_t s);
hipError_t launch_lincomb(double *out, double a, const double *x, double b, const double *y, int64_t n,
                          hipStream_t s);
hipError_t launch_relax_vjp(double *v, const double *cr, int64_t n, hipStream_t s);
hipError_t launch_surface_adj(double *phis_bar, const double *phibar, const double *Alam, int64_t n_v, int64_t n_s,
                              hipStream_t s);
hipError_t launch_set_lift(double *v, const double *phis, int64_t n_v, int64_t n_s, hipStream_t s);
hipError_t launch_copy_top(double *x, const double *phis, int64_t n_v, int64_t n_s, hipStream_t s);
hipError_t launch_bnorm(const double *f, const double *y, int64_t n_v, int64_t n_s, double *partial,
                        PcgScalars *sc, double rtol, double atol, hipStream_t s);
template <typename T>
hipError_t launch_pcg_init(const double *f, const T *Ax, T *r, T *p, const T *dinv, int64_t n_v, int64_t n_s,
                           double *partial, PcgScalars *sc, bool relative_tol, double inner_rtol, hipStream_t s);
hipError_t launch_resid_to32(const double *f, const double *Ax, float *r, float *p, float *d, const float *dinv,
                             int64_t n_v, int64_t n_s, double *partial, PcgScalars *outer, PcgScalars *inner,
                             double inner_rtol, hipStream_t s);
hipError_t launch_finalize_pq(const double *partial, int np, PcgScalars *sc, hipStream_t s);
template <typename T, typename TX>
hipError_t launch_pcg_update(TX *x, T *r, const T *p, const T *q, const T *dinv, int64_t n_v, double *partial,
                             PcgScalars *sc, hipStream_t s);
hipError_t launch_finalize_rz(const double *partial, int np, PcgScalars *sc, hipStream_t s);
template <typename T>
hipError_t launch_pcg_dir(T *p, const T *r, const T *dinv, int64_t n_v, PcgScalars *sc, hipStream_t s);
hipError_t launch_add_f32(double *x, const float *d, int64_t n_v, hipStream_t s);
hipError_t launch_cast_f32(const double *a, float *b, int64_t n, hipStream_t s);
hipError_t launch_fill(double *v, double val, int64_t n, hipStream_t s);
hipError_t launch_zero_i32(int32_t *v, int64_t n, hipStream_t s);

constexpr int kVecBlocks = kPartialVecBlocks;   // fixed grid of the grid-stride vector kernels (deterministic partials)
constexpr int kVecThreads = 256;

// one coarse level of the p-multigrid preconditioner
struct MgLevel {
  fnpf_ctx child = nullptr;               // context of the same mesh at the coarse degree (owned)
  struct Ctx *c = nullptr;                // its state
  double *Hc = nullptr, *hc = nullptr;    // eta + h and h at its surface nodes
  double *v64[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // b, x, r, d, q
  float *v32[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double *ev64 = nullptr;                 // its eigenvector estimate (power-iteration warm start)
  float *ev32 = nullptr;
  bool ev_ok64 = false, ev_ok32 = false;
};

struct Ctx {
  // mesh
  int dim = 3, p = 1, nz = 1, n_eh = 0;
  int64_t n_s = 0, n_v = 0, n_e = 0;
  int nh = 1, np = 1, ng = 6;
  double g = 9.81;
  std::vector<int32_t> h_eh_nodes;
  std::vector<double> h_corner;           // [n_eh][2^(dim-1)][dim-1]
  std::vector<double> h_arc;              // [n_eh][4][3] or empty
  std::vector<int32_t> h_tags;            // [n_eh][2(dim-1)]
  std::vector<double> h_node_xy;          // [n_s][dim-1]
  std::vector<double> h_xh;               // [n_eh][nh][dim-1] unwrapped element node coordinates
  std::vector<double> h_layer_s;          // [nz+1]
  std::vector<double> h_sigma;            // [p nz + 1]
  std::vector<ColourRange> colours;
  std::vector<double> h_hm;               // horizontal metrics (host copy)
  std::vector<double> h_half_ds;          // [nz]
  int ncg = 5;                            // column-data components (5 in 3D, 3 in 2D)
  int max_colour_blocks = 0;              // sum over colours of apply blocks
  // device mesh data
  int32_t *d_eh_nodes = nullptr;
  int32_t *d_cols = nullptr;              // columns grouped by colour
  uint8_t *d_flags = nullptr;             // [n_eh][nh] first/last writer flags
  int32_t *d_face_tag = nullptr;          // [n_eh][2(dim-1)]
  double *d_hm = nullptr;                 // [ncomp][n_eh*nh]
  double *d_sigma = nullptr;              // [p nz + 1]
  double *d_layer_s = nullptr;            // [nz + 1]
  double *d_mlump_w = nullptr;            // [n_s] sum_e w_i w_j w_p det J_h (w recovery denominator)
  double *d_mlump_s = nullptr;            // [n_s] sum_e w_i w_j det J_h (surface mass)
  // apply variant: 0 fused geometry (factors recomputed in registers), 1 stored factors,
  // 2 fused geometry, unrolled schedule; the schedule of 0 is refined by the fields below
  int apply_variant = 0;
  bool apply_lines = false;               // 3D fused apply with the xi/eta line schedule
  bool apply_owner = false;               // 3D line schedule with owner-computes assembly (two passes)
  // owner-computes assembly: contributions of a column at nodes it does not own go to face
  // slots (column-major numbering); the second pass adds them at the owner
  std::vector<int32_t> h_slot;            // [n_eh][nh] slot id, -1 where owned
  std::vector<int32_t> h_ps_node, h_ps_ptr, h_ps_slot;  // shared nodes, CSR of their slots
  int64_t n_slots = 0;
  int n_ps = 0;
  int32_t *d_slot = nullptr, *d_ps_node = nullptr, *d_ps_ptr = nullptr, *d_ps_slot = nullptr;
  // tile assembly of the owner-computes apply: a tile is tile_cols consecutive columns (one
  // workgroup); contributions of a tile's columns at a node are summed in LDS by the tile's
  // representative column of the node (exchange entries h_xch: [n_eh][nh][4] int16, the entry this
  // column writes and up to three its representative reads, -1 none), and only the tile sums of
  // non-owning tiles (and exchange overflow) go through face slots h_tslot
  int tile_cols = 0;
  int tile_xmax = 0;                      // exchange entries per tile (LDS)
  std::vector<int32_t> h_tslot;           // [n_eh][nh] face slot, -1 none
  std::vector<int16_t> h_xch;             // [n_eh][nh][4]
  std::vector<int32_t> h_tps_node, h_tps_ptr, h_tps_slot;  // nodes with face slots, CSR of the slots
  int64_t n_tslots = 0;
  int n_tps = 0;
  int32_t *d_tslot = nullptr, *d_tps_node = nullptr, *d_tps_ptr = nullptr, *d_tps_slot = nullptr;
  int16_t *d_xch = nullptr;
  // the geometry's face layout (k_geom, k_diag_faces): per column node its place in a level row
  // of n_gslots entries (-1 none): the owner tile's value at a node with slots at k (its position
  // among h_tps_node), the node's first slot at n_tps + k, further slots from 2 n_tps on, listed
  // per node (CSR h_gx_ptr, h_gx_slot)
  std::vector<int32_t> h_gslot, h_gx_ptr, h_gx_slot;
  int64_t n_gslots = 0;
  int32_t *d_gslot = nullptr, *d_gx_ptr = nullptr, *d_gx_slot = nullptr;
  double *d_F64 = nullptr;                // [p nz + 1][largest of n_slots, n_tslots, n_gslots]
  float *d_F32 = nullptr;
  double *d_cg64 = nullptr;               // [5|3][n_eh*nh] H, H_xi, h_xi, (H_eta, h_eta) per column node
  float *d_cg32 = nullptr;
  float *d_hm32 = nullptr;                // FP32 copy of d_hm
  double *d_half_ds = nullptr;            // [nz] (s_{l+1} - s_l) / 2
  float *d_half_ds32 = nullptr;
  float *d_sigma32 = nullptr;
  bool have_G = false;                    // stored factors are current
  // geometry state
  double *d_G64 = nullptr;
  float *d_G32 = nullptr;
  double *d_diag = nullptr;
  bool have_diag = false;                 // d_diag holds the assembled diagonal at every node
  bool keep_diag = false;                 // store it at every geometry update (line smoothing reads it)
  double *d_dinv = nullptr;
  float *d_dinv32 = nullptr;
  const double *geom_eta = nullptr;       // eta/h of the last fnpf_geom (caller-owned, used by w recovery)
  const double *geom_h = nullptr;
  bool have_geom = false;
  bool have_geom32 = false;
  bool want32 = false;
  int32_t *d_err = nullptr;               // device error flag (GEOM)
  // workspaces
  double *d_r = nullptr, *d_p = nullptr, *d_q = nullptr, *d_phi = nullptr;
  float *d_r32 = nullptr, *d_p32 = nullptr, *d_q32 = nullptr, *d_d32 = nullptr;
  double *d_sa[2] = {nullptr, nullptr};   // stage states (eta) ping-pong
  double *d_sp[2] = {nullptr, nullptr};   // stage states (phi_s)
  double *d_acc_e = nullptr, *d_acc_p = nullptr;
  double *d_w = nullptr;                  // recovered w at the surface
  double *d_geoH = nullptr, *d_geoh = nullptr;    // eta + h and h of the last fnpf_geom
  double *d_wnum = nullptr, *d_nk = nullptr, *d_nd = nullptr;  // surface scatter scratch
  double *d_partial = nullptr;
  int n_partial = 0;                       // capacity: partial_capacity(partial_uses(...))
  double *d_mg_scal = nullptr;             // [4] power-iteration scalars of the p-multigrid refresh
  PcgScalars *d_sc = nullptr;             // [2]: outer/plain, inner
  PcgScalars *h_sc = nullptr;             // pinned host mirror
  // per stage, the solutions of the last steps of a sequence (initial-guess extrapolation)
  static constexpr int kHistMax = 5;      // extrapolation orders 1 .. kHistMax - 1
  struct History {
    double *v[4][kHistMax] = {};          // a ring of `slots` vectors [n_v] per stage
    int slots = 0;                        // ring length in use (allocated slots per stage)
    int head = 0;                         // slot of the newest step
    int count = 0;                        // steps recorded in the current sequence
    double dt = 0.0, t = 0.0;             // step size of the sequence, time of its newest step
  };
  History hist;                           // forward potentials of fnpf_rk4_step
  History ahist;                          // adjoint solutions of fnpf_rk4_step_vjp (steps run backwards)
  // adjoint workspaces (allocated on first use)
  double *d_lam = nullptr, *d_phibar = nullptr;
  double *d_kbe = nullptr, *d_kbp = nullptr, *d_ybe = nullptr, *d_ybp = nullptr;
  double *d_acce = nullptr, *d_accp = nullptr, *d_wbar = nullptr, *d_zero_s = nullptr;
  bool have_adjoint = false;
  // p-multigrid preconditioner (built on first use; the fine level is this context)
  std::vector<MgLevel> mg;
  bool mg_built = false;
  bool mg_stale64 = true, mg_stale32 = true;   // geometry changed since the last refresh
  bool mg_line = false;                   // smoothing with the vertical line blocks instead of D
  // Cholesky factors of this level's vertical line blocks, [p+1][p nz+1][n_s] (line_smoother.hip)
  double *d_lb64 = nullptr;
  float *d_lb32 = nullptr;
  double *mg_f64[4] = {nullptr, nullptr, nullptr, nullptr};  // fine-level z, r, d, q
  float *mg_f32[4] = {nullptr, nullptr, nullptr, nullptr};
  double *d_mgc = nullptr;                // Chebyshev coefficient table [precision][level][32]
  double *d_mg_lam = nullptr;             // eigenvalue estimates behind it [precision][level]
  double *d_mg_lz = nullptr;              // Lanczos coefficients and scalars of the eigenvalue estimate
  double *mg_ev64 = nullptr;              // fine-level eigenvector estimate
  float *mg_ev32 = nullptr;
  bool mg_ev_ok64 = false, mg_ev_ok32 = false;
  // captured PCG iteration chunks, replayed with hipGraphLaunch: [0] FP64 solve, [1] FP32 inner
  struct GraphKey {
    const void *x = nullptr;
    int precond = -1, check_every = 0, cheb = 0, variant = -1, nb = 0;
    bool lines = false, owner = false, line = false;
    bool operator==(const GraphKey &o) const {
      return x == o.x && precond == o.precond && check_every == o.check_every && cheb == o.cheb &&
             variant == o.variant && nb == o.nb && lines == o.lines && owner == o.owner && line == o.line;
    }
  };
  hipGraph_t g_graph[2] = {nullptr, nullptr};
  hipGraphExec_t g_exec[2] = {nullptr, nullptr};
  GraphKey g_key[2];
  hipStream_t cap_stream = nullptr;       // capture-only stream (default priority)
  double *d_mask = nullptr;               // 1 below the surface level, 0 on it (no preconditioner)
  float *d_mask32 = nullptr;
  // consistent over-integrated free-surface form (sq_nq = 0: lumped GLL collocation)
  int sq_nq = 0, sq_iters = 0;
  double sq_lo = 0.0, sq_hi = 0.0;        // Chebyshev interval of M_L^{-1} M
  double *d_sq_B = nullptr, *d_sq_Bd = nullptr;   // [nq][p+1] Lagrange values / derivatives at Gauss points
  double *d_sq_met = nullptr;             // [5 | 2][n_eh * nq^(dim-1)]: J^{-1} entries, W det J
  double *d_sq_b = nullptr, *d_sq_x = nullptr, *d_sq_r = nullptr, *d_sq_d = nullptr, *d_sq_ad = nullptr;  // [2][n_s]
  double *d_sq_scr = nullptr;             // [3][n_s] VJP accumulation
  // modal filter of the surface fields (cutoff < 0: off)
  int filter_cutoff = -1, filter_order = 0;
  double filter_alpha = 0.0;
  double *d_filt_M = nullptr;             // [(p+1)^2] nodal 1D filter matrix M[i*(p+1)+k]
  double *d_filt_inv_mult = nullptr;      // [n_s] 1 / number of surface elements at the node
  double *d_filt_acc = nullptr;           // [n_s] colour-ordered accumulation
  double *d_filt_tmp = nullptr;           // [n_s] filtered copy before write-back
  // linear potential flow (flat geometry at eta = 0, linear free-surface conditions)
  bool linear = false;
  double *d_flat = nullptr;               // [n_s] zeros: the LPF surface
  const double *flat_h = nullptr;         // depth pointer of the current flat geometry
  bool flat_valid = false;                // the current geometry is the flat one for flat_h
  double *d_scr_s = nullptr;              // [n_s] scratch (discarded eta adjoint of the LPF geometry)
  // relaxation
  double *d_cr = nullptr, *d_rec = nullptr, *d_res = nullptr, *d_rpc = nullptr, *d_rps = nullptr;
  double relax_omega = 0.0, relax_tramp = 0.0;
  bool have_relax = false;
  std::string err;
  int device = 0;
};

// owner-computes apply (3D line schedule): active for the current settings, and its block count
// (pass 1 + pass 2 partials of the fused dot product)
bool owner_apply_active(const Ctx &c);
int owner_apply_blocks(const Ctx &c);

// p-multigrid (multigrid.hip)
fnpf_status mg_build(Ctx &c);
void mg_free(Ctx &c);
template <typename T>
fnpf_status mg_refresh(Ctx &c, hipStream_t s);
template <typename T>
hipError_t mg_vcycle(Ctx &c, const T *r, T *z, const int32_t *skip, int smooth, hipStream_t s,
                     double *dot_partial = nullptr, bool *dot_done = nullptr, bool pre_scaled = false);
// x += alpha p, r -= alpha q with the partials of r.r; with the degree-2 V-cycle (smooth == 2 and a
// hierarchy) it also writes the cycle's first smoothing step, and the mg_vcycle call on this r that
// follows must pass pre_scaled = true.
hipError_t launch_mg_update(Ctx &c, fnpf_dtype dt, void *x, void *r, const void *p, const void *q, double *partial,
                            PcgScalars *sc, hipStream_t s, int smooth);
hipError_t launch_mg_dot_dir(Ctx &c, fnpf_dtype dt, const void *r, const void *z, void *p, double *partial,
                             PcgScalars *sc, int first, hipStream_t s, bool have_partials = false);
Ctx &ctx_of(fnpf_ctx h);
fnpf_status ctx_ensure32(Ctx &c);
fnpf_status geom_impl_total(Ctx &c, const double *H, const double *h, hipStream_t s);
hipError_t launch_faces(Ctx &c, fnpf_dtype dt, void *y, bool mask, hipStream_t s, const int32_t *skip);
// vertical line smoother (line_smoother.hip): band[d][v][n] of B assembled from the geometry,
// the level's Cholesky factors (FP64, and FP32 when the level keeps FP32 data), and the smoothing
// steps with them
hipError_t launch_line_band(Ctx &c, double *band, hipStream_t s);
void mg_set_line(Ctx &c, bool line);
hipError_t line_setup(Ctx &c, hipStream_t s);
template <typename T>
hipError_t line_apply(const Ctx &c, const T *w, T *z, hipStream_t s);
template <typename T>
hipError_t line_cheb0(const Ctx &c, const T *b, T *r, T *d, T *x, const double *cf, const int32_t *skip,
                      hipStream_t s);
template <typename T>
hipError_t line_cheb1(const Ctx &c, const T *b, T *q, T *r, T *d, T *x, const double *cf, const int32_t *skip,
                      hipStream_t s);
template <typename T>
hipError_t line_chebk(const Ctx &c, T *q, T *r, T *d, T *x, const double *cf, int k, const int32_t *skip,
                      hipStream_t s);
template <typename T>
hipError_t line_lanczos_w(const Ctx &c, T *q, const T *v, T *vp, const double *al, const double *be, hipStream_t s);
template <typename T>
hipError_t line_bnorm_partials(const Ctx &c, const T *w, double *partial, int nblocks, hipStream_t s);

// host setup (setup.cpp)
void gll_host(int p, double *x, double *w, double *D);
std::string coarse_numbering(const Ctx &f, int pc, std::vector<int32_t> &nodes, int64_t &n_s);
std::string surface_interp_weights(const Ctx &c, int32_t n_pts, const double *pts, int32_t *node, double *w);
std::string build_host_mesh(const fnpf_mesh_desc &m, Ctx &c, std::vector<double> &hm, std::vector<uint8_t> &flags,
                            std::vector<int32_t> &cols, std::vector<double> &mlump_w, std::vector<double> &mlump_s);

}  // namespace fnpf
