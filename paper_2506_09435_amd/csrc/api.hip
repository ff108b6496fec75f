// C ABI of the FNPF-SEM Laplace-solve library: context management, argument validation and
// the host drivers of the PCG solve and the ERK4 step.  Kernels live in kernels_*.hip.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fnpf_internal.h"

using namespace fnpf;

struct fnpf_ctx_s {
  Ctx c;
};

static thread_local std::string g_create_error;

namespace {

const double kRkB[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
const double kRkC[4] = {0.0, 0.5, 0.5, 1.0};

fnpf_status fail(Ctx *c, fnpf_status st, const std::string &msg) {
  if (c) c->err = msg;
  return st;
}

fnpf_status hipfail(Ctx *c, hipError_t e, const char *where) {
  if (c) c->err = std::string(where) + ": " + hipGetErrorString(e);
  return FNPF_ERR_HIP;
}

#define HIPCHK(expr)                                 \
  do {                                               \
    hipError_t e__ = (expr);                         \
    if (e__ != hipSuccess) return hipfail(&c, e__, #expr); \
  } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc((void **)p, n * sizeof(T));
}

template <typename T>
void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

void free_graphs(Ctx &c) {
  for (int k = 0; k < 2; ++k) {
    if (c.g_exec[k]) (void)hipGraphExecDestroy(c.g_exec[k]);
    if (c.g_graph[k]) (void)hipGraphDestroy(c.g_graph[k]);
    c.g_exec[k] = nullptr;
    c.g_graph[k] = nullptr;
    c.g_key[k] = Ctx::GraphKey();
  }
}

void free_all(Ctx &c) {
  free_graphs(c);
  dfree(c.d_flat);
  dfree(c.d_scr_s);
  sq_free(c);
  dfree(c.d_filt_M);
  dfree(c.d_filt_inv_mult);
  dfree(c.d_filt_acc);
  dfree(c.d_filt_tmp);
  if (c.cap_stream) (void)hipStreamDestroy(c.cap_stream);
  c.cap_stream = nullptr;
  mg_free(c);
  dfree(c.d_mask);
  dfree(c.d_mask32);
  dfree(c.d_eh_nodes);
  dfree(c.d_cols);
  dfree(c.d_slot);
  dfree(c.d_ps_node);
  dfree(c.d_ps_ptr);
  dfree(c.d_ps_slot);
  dfree(c.d_F64);
  dfree(c.d_F32);
  dfree(c.d_tslot);
  dfree(c.d_xch);
  dfree(c.d_tps_node);
  dfree(c.d_tps_ptr);
  dfree(c.d_tps_slot);
  dfree(c.d_gslot);
  dfree(c.d_gx_ptr);
  dfree(c.d_gx_slot);
  dfree(c.d_flags);
  dfree(c.d_face_tag);
  dfree(c.d_hm);
  dfree(c.d_sigma);
  dfree(c.d_layer_s);
  dfree(c.d_mlump_w);
  dfree(c.d_mlump_s);
  dfree(c.d_G64);
  dfree(c.d_G32);
  dfree(c.d_cg64);
  dfree(c.d_cg32);
  dfree(c.d_hm32);
  dfree(c.d_half_ds);
  dfree(c.d_half_ds32);
  dfree(c.d_sigma32);
  dfree(c.d_diag);
  dfree(c.d_dinv);
  dfree(c.d_dinv32);
  dfree(c.d_err);
  dfree(c.d_r);
  dfree(c.d_p);
  dfree(c.d_q);
  dfree(c.d_phi);
  dfree(c.d_r32);
  dfree(c.d_p32);
  dfree(c.d_q32);
  dfree(c.d_d32);
  for (int k = 0; k < 2; ++k) {
    dfree(c.d_sa[k]);
    dfree(c.d_sp[k]);
  }
  dfree(c.d_acc_e);
  dfree(c.d_acc_p);
  dfree(c.d_w);
  dfree(c.d_geoH);
  dfree(c.d_geoh);
  dfree(c.d_wnum);
  dfree(c.d_nk);
  dfree(c.d_nd);
  dfree(c.d_partial);
  dfree(c.d_mg_scal);
  dfree(c.d_lb64);
  dfree(c.d_lb32);
  dfree(c.d_sc);
  if (c.h_sc) (void)hipHostFree(c.h_sc);
  c.h_sc = nullptr;
  for (int s = 0; s < 4; ++s)
    for (int k = 0; k < Ctx::kHistMax; ++k) {
      dfree(c.hist.v[s][k]);
      dfree(c.ahist.v[s][k]);
    }
  dfree(c.d_lam);
  dfree(c.d_phibar);
  dfree(c.d_kbe);
  dfree(c.d_kbp);
  dfree(c.d_ybe);
  dfree(c.d_ybp);
  dfree(c.d_acce);
  dfree(c.d_accp);
  dfree(c.d_wbar);
  dfree(c.d_zero_s);
  dfree(c.d_cr);
  dfree(c.d_rec);
  dfree(c.d_res);
  dfree(c.d_rpc);
  dfree(c.d_rps);
}

template <typename T>
hipError_t upload(T **d, const T *h, size_t n) {
  hipError_t e = dalloc(d, n);
  if (e != hipSuccess) return e;
  return hipMemcpy(*d, h, n * sizeof(T), hipMemcpyHostToDevice);
}

// Enable the FP32 path (allocates FP32 factors and inner PCG vectors on first use).
fnpf_status ensure_G(Ctx &c) {
  if (!c.d_G64) HIPCHK(dalloc(&c.d_G64, (size_t)c.n_e * c.ng * c.np));
  if (c.want32 && !c.d_G32) HIPCHK(dalloc(&c.d_G32, (size_t)c.n_e * c.ng * c.np));
  return FNPF_OK;
}

template <typename T>
hipError_t upload_cast(float **d, const std::vector<T> &h) {
  std::vector<float> f(h.begin(), h.end());
  return upload(d, f.data(), f.size());
}

fnpf_status ensure32(Ctx &c) {
  if (c.want32) return FNPF_OK;
  HIPCHK(dalloc(&c.d_cg32, (size_t)c.ncg * c.n_eh * c.nh));
  HIPCHK(upload_cast(&c.d_hm32, c.h_hm));
  HIPCHK(upload_cast(&c.d_sigma32, c.h_sigma));
  HIPCHK(upload_cast(&c.d_half_ds32, c.h_half_ds));
  if (c.apply_variant == 1) HIPCHK(dalloc(&c.d_G32, (size_t)c.n_e * c.ng * c.np));
  HIPCHK(dalloc(&c.d_dinv32, c.n_v));
  HIPCHK(dalloc(&c.d_r32, c.n_v));
  HIPCHK(dalloc(&c.d_p32, c.n_v));
  HIPCHK(dalloc(&c.d_q32, c.n_v));
  HIPCHK(dalloc(&c.d_d32, c.n_v));
  HIPCHK(dalloc(&c.d_F32, (size_t)(c.p * c.nz + 1) * std::max<int64_t>(std::max(c.n_slots, c.n_tslots), 1)));
  c.want32 = true;
  c.have_geom32 = false;
  return FNPF_OK;
}

fnpf_status ensure_adjoint(Ctx &c, hipStream_t s) {
  if (c.have_adjoint) return FNPF_OK;
  HIPCHK(dalloc(&c.d_lam, c.n_v));
  HIPCHK(dalloc(&c.d_phibar, c.n_v));
  double **surf[8] = {&c.d_kbe, &c.d_kbp, &c.d_ybe, &c.d_ybp, &c.d_acce, &c.d_accp, &c.d_wbar, &c.d_zero_s};
  for (auto p : surf) HIPCHK(dalloc(p, c.n_s));
  HIPCHK(launch_fill(c.d_lam, 0.0, c.n_v, s));
  HIPCHK(launch_fill(c.d_zero_s, 0.0, c.n_s, s));
  c.have_adjoint = true;
  return FNPF_OK;
}

// A ring of `slots` past solutions per stage; a new length starts an empty history.
fnpf_status ensure_history(Ctx &c, Ctx::History &H, int slots) {
  if (slots == H.slots) return FNPF_OK;
  for (int s = 0; s < 4; ++s)
    for (int k = 0; k < Ctx::kHistMax; ++k) {
      if (k >= slots) dfree(H.v[s][k]);
      else if (!H.v[s][k]) HIPCHK(dalloc(&H.v[s][k], c.n_v));
    }
  H.slots = slots;
  H.head = 0;
  H.count = 0;
  return FNPF_OK;
}

// out = the polynomial extrapolation of stage stg's history to the next step of the sequence:
// out = sum_{j=1}^{k+1} (-1)^(j+1) binom(k+1, j) v(n-j), k = min(order, steps recorded - 1).
// Returns false (out untouched) when fewer than two steps are recorded.
bool history_extrapolate(const Ctx::History &H, int stg, int order, double *out, int64_t n, hipStream_t s,
                         hipError_t &err) {
  err = hipSuccess;
  const int k = std::min(order, H.count - 1);
  if (k < 1) return false;
  const int K = H.slots;
  auto past = [&](int j) { return H.v[stg][(H.head - (j - 1) + K) % K]; };   // j = 1: newest
  double cj[Ctx::kHistMax + 1];
  for (int j = 1, b = 1; j <= k + 1; ++j) {
    b = b * (k + 2 - j) / j;   // binom(k+1, j)
    cj[j] = (j % 2 ? 1.0 : -1.0) * b;
  }
  if ((err = launch_lincomb(out, cj[1], past(1), cj[2], past(2), n, s)) != hipSuccess) return false;
  for (int j = 3; j <= k + 1; ++j)
    if ((err = launch_lincomb(out, 1.0, out, cj[j], past(j), n, s)) != hipSuccess) return false;
  return true;
}

// stage stg's solution of the current step goes over the oldest slot
hipError_t history_record(const Ctx::History &H, int stg, const double *x, int64_t n, hipStream_t s) {
  return hipMemcpyAsync(H.v[stg][(H.head + 1) % H.slots], x, n * sizeof(double), hipMemcpyDeviceToDevice, s);
}

// after the step at time t: its slot becomes the newest
void history_advance(Ctx::History &H, double t, double dt, bool continues) {
  H.head = (H.head + 1) % H.slots;
  H.count = continues ? std::min(H.count + 1, H.slots) : 1;
  H.dt = dt;
  H.t = t;
}

fnpf_status ensure_flat(Ctx &c, hipStream_t s) {
  if (c.d_flat) return FNPF_OK;
  HIPCHK(dalloc(&c.d_flat, c.n_s));
  HIPCHK(dalloc(&c.d_scr_s, c.n_s));
  HIPCHK(launch_fill(c.d_flat, 0.0, c.n_s, s));
  return FNPF_OK;
}

bool consistent_surface(const Ctx &c) { return c.sq_nq > 0 && !c.linear; }

// Free-surface RHS of one stage (lumped: fused kernel; consistent: quadrature, mass solve, stage update)
hipError_t stage_rhs(Ctx &c, const double *eta, const double *phs, const double *w, const RkStageArgs &a,
                     hipStream_t s) {
  if (!consistent_surface(c)) return launch_rhs(c, eta, phs, w, a, s);
  hipError_t e = launch_sq_rhs(c, eta, phs, w, c.d_sq_b, s);
  if (e != hipSuccess) return e;
  e = sq_solve(c, c.d_sq_b, c.d_sq_x, s);
  if (e != hipSuccess) return e;
  return launch_sq_stage(a, c.d_sq_x, c.n_s, s);
}

// VJP of the free-surface RHS: adds to eta_bar, phis_bar, w_bar from kbar_e, kbar_p
hipError_t stage_rhs_vjp(Ctx &c, const double *eta, const double *phs, const double *w, const double *kbe,
                         const double *kbp, double *eta_bar, double *phis_bar, double *w_bar, hipStream_t s) {
  if (c.linear) return launch_rhs_vjp_linear(kbe, kbp, eta_bar, w_bar, c.g, c.n_s, s);
  if (!consistent_surface(c)) return launch_rhs_vjp(c, eta, phs, w, kbe, kbp, eta_bar, phis_bar, w_bar, s);
  // the fixed-length Chebyshev solve is a symmetric map, so bbar = S kbar
  hipError_t e = launch_sq_pack(kbe, kbp, c.d_sq_b, c.n_s, s);
  if (e != hipSuccess) return e;
  e = sq_solve(c, c.d_sq_b, c.d_sq_x, s);
  if (e != hipSuccess) return e;
  return launch_sq_rhs_vjp(c, eta, phs, w, c.d_sq_x, eta_bar, phis_bar, w_bar, s);
}

fnpf_status check_err_flag(Ctx &c, hipStream_t s) {
  int32_t flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, c.d_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (flag) {
    HIPCHK(launch_zero_i32(c.d_err, 1, s));
    return fail(&c, FNPF_ERR_GEOM, "eta + h <= 0 (or non-finite) at a surface node: the column collapsed");
  }
  return FNPF_OK;
}

int apply_blocks(const Ctx &c) {
  if (owner_apply_active(c)) return owner_apply_blocks(c);
  return c.max_colour_blocks;
}

// Diagonal scaling of the preconditioner choice: the Jacobi inverse (1), or the mask of the
// non-surface unknowns (0: none; 2: the first direction before the multigrid one replaces it).
fnpf_status ensure_mask(Ctx &c, hipStream_t s) {
  if (c.d_mask) return FNPF_OK;
  HIPCHK(dalloc(&c.d_mask, c.n_v));
  HIPCHK(launch_fill(c.d_mask, 1.0, c.n_v, s));
  HIPCHK(launch_fill(c.d_mask + (c.n_v - c.n_s), 0.0, c.n_s, s));
  if (c.want32) {
    HIPCHK(dalloc(&c.d_mask32, c.n_v));
    HIPCHK(launch_cast_f32(c.d_mask, c.d_mask32, c.n_v, s));
  }
  return FNPF_OK;
}

// Runs body (check_every PCG iterations enqueued on a stream): directly, or as a HIP graph captured
// on the context's capture stream and replayed on s.  A graph is reused while its key (solution
// pointer, preconditioner and schedule settings) is unchanged; every kernel in it reads its
// scalars (alpha, beta, Chebyshev coefficients, the done flag) from device memory.
template <typename Body>
fnpf_status run_chunk(Ctx &c, int slot, const Ctx::GraphKey &key, bool use_graph, hipStream_t s, Body body) {
  if (!use_graph) return body(s);
  if (!c.g_exec[slot] || !(c.g_key[slot] == key)) {
    if (c.g_exec[slot]) (void)hipGraphExecDestroy(c.g_exec[slot]);
    if (c.g_graph[slot]) (void)hipGraphDestroy(c.g_graph[slot]);
    c.g_exec[slot] = nullptr;
    c.g_graph[slot] = nullptr;
    if (!c.cap_stream) HIPCHK(hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeThreadLocal));
    fnpf_status st = body(c.cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c.cap_stream, &g);
    if (st != FNPF_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hipfail(&c, e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hipfail(&c, e, "hipGraphInstantiate");
    }
    c.g_graph[slot] = g;
    c.g_exec[slot] = x;
    c.g_key[slot] = key;
  }
  HIPCHK(hipGraphLaunch(c.g_exec[slot], s));
  return FNPF_OK;
}

Ctx::GraphKey graph_key(const Ctx &c, const void *x, const fnpf_solve_opts &o, int nb) {
  Ctx::GraphKey k;
  k.x = x;
  k.precond = o.precond;
  k.check_every = o.check_every;
  k.cheb = o.cheb_degree;
  k.variant = c.apply_variant;
  k.lines = c.apply_lines;
  k.owner = c.apply_owner;
  k.line = c.mg_line;
  k.nb = nb;
  return k;
}

// PCG on A_II (FP64), x = phi holds the guess with its surface level set.
fnpf_status pcg64(Ctx &c, const double *f, double *x, const fnpf_solve_opts &o, int &iters, hipStream_t s) {
  PcgScalars *sc = c.d_sc;
  const bool mg = o.precond == 2;
  if (o.precond != 1) {
    fnpf_status st = ensure_mask(c, s);
    if (st != FNPF_OK) return st;
  }
  if (mg) {
    mg_set_line(c, o.line_smoother != 0);
    fnpf_status st = mg_refresh<double>(c, s);
    if (st != FNPF_OK) return fail(&c, st, c.err.empty() ? "p-multigrid setup failed" : c.err);
  }
  const double *dinv = o.precond == 1 ? c.d_dinv : c.d_mask;
  double *z = mg ? c.mg_f64[0] : nullptr;
  HIPCHK(launch_apply(c, FNPF_F64, x, c.d_q, true, nullptr, nullptr, s));
  HIPCHK(launch_pcg_init<double>(f, c.d_q, c.d_r, c.d_p, dinv, c.n_v, c.n_s, c.d_partial, sc, false, 0.0, s));
  if (mg) {
    bool fused = false;
    HIPCHK(mg_vcycle<double>(c, c.d_r, z, &sc->done, o.cheb_degree, s, c.d_partial, &fused));
    HIPCHK(launch_mg_dot_dir(c, FNPF_F64, c.d_r, z, c.d_p, c.d_partial, sc, 1, s, fused));
  }
  const int nb = apply_blocks(c);
  auto body = [&](hipStream_t st) -> fnpf_status {
    for (int k = 0; k < o.check_every; ++k) {
      HIPCHK(launch_apply(c, FNPF_F64, c.d_p, c.d_q, true, c.d_partial, &sc->done, st));
      HIPCHK(launch_finalize_pq(c.d_partial, nb, sc, st));
      if (mg) {
        HIPCHK(launch_mg_update(c, FNPF_F64, x, c.d_r, c.d_p, c.d_q, c.d_partial, sc, st, o.cheb_degree));
        bool fused = false;
        HIPCHK(mg_vcycle<double>(c, c.d_r, z, &sc->done, o.cheb_degree, st, c.d_partial, &fused, true));
        HIPCHK(launch_mg_dot_dir(c, FNPF_F64, c.d_r, z, c.d_p, c.d_partial, sc, 0, st, fused));
      } else {
        HIPCHK((launch_pcg_update<double, double>(x, c.d_r, c.d_p, c.d_q, dinv, c.n_v, c.d_partial, sc, st)));
        HIPCHK(launch_pcg_dir<double>(c.d_p, c.d_r, dinv, c.n_v, sc, st));
      }
    }
    return FNPF_OK;
  };
  const Ctx::GraphKey key = graph_key(c, x, o, nb);
  iters = 0;
  for (;;) {
    fnpf_status st = run_chunk(c, 0, key, o.use_graph != 0, s, body);
    if (st != FNPF_OK) return st;
    HIPCHK(hipMemcpyAsync(c.h_sc, c.d_sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    iters = c.h_sc[0].iters;
    if (c.h_sc[0].done || iters >= o.max_iter) break;
  }
  if (c.h_sc[0].breakdown == 2) return fail(&c, FNPF_ERR_NAN, "non-finite residual in PCG");
  if (c.h_sc[0].breakdown == 1)
    return fail(&c, FNPF_ERR_BREAKDOWN, "PCG breakdown: p^T A p <= 0 or r^T z <= 0");
  if (!c.h_sc[0].done) return fail(&c, FNPF_ERR_NOCONV, "PCG did not reach the tolerance within max_iter");
  return FNPF_OK;
}

// Mixed precision: FP64 residual and update around FP32 PCG (defect correction).
fnpf_status pcg_mixed(Ctx &c, const double *f, double *x, const fnpf_solve_opts &o, int &iters, int &outer,
                      hipStream_t s) {
  PcgScalars *so = c.d_sc, *si = c.d_sc + 1;
  const bool mg = o.precond == 2;
  if (o.precond != 1) {
    fnpf_status st = ensure_mask(c, s);
    if (st != FNPF_OK) return st;
  }
  if (mg) {
    mg_set_line(c, o.line_smoother != 0);
    fnpf_status st = mg_refresh<float>(c, s);
    if (st != FNPF_OK) return fail(&c, st, c.err.empty() ? "p-multigrid setup failed" : c.err);
  }
  const float *dinv = o.precond == 1 ? c.d_dinv32 : c.d_mask32;
  float *z = mg ? c.mg_f32[0] : nullptr;
  const int nb = apply_blocks(c);
  auto body = [&](hipStream_t st) -> fnpf_status {
    for (int k = 0; k < o.check_every; ++k) {
      HIPCHK(launch_apply(c, FNPF_F32, c.d_p32, c.d_q32, true, c.d_partial, &si->done, st));
      HIPCHK(launch_finalize_pq(c.d_partial, nb, si, st));
      if (mg) {
        HIPCHK(launch_mg_update(c, FNPF_F32, c.d_d32, c.d_r32, c.d_p32, c.d_q32, c.d_partial, si, st,
                                o.cheb_degree));
        bool fused = false;
        HIPCHK(mg_vcycle<float>(c, c.d_r32, z, &si->done, o.cheb_degree, st, c.d_partial, &fused, true));
        HIPCHK(launch_mg_dot_dir(c, FNPF_F32, c.d_r32, z, c.d_p32, c.d_partial, si, 0, st, fused));
      } else {
        HIPCHK((launch_pcg_update<float, float>(c.d_d32, c.d_r32, c.d_p32, c.d_q32, dinv, c.n_v, c.d_partial, si,
                                                st)));
        HIPCHK(launch_pcg_dir<float>(c.d_p32, c.d_r32, dinv, c.n_v, si, st));
      }
    }
    return FNPF_OK;
  };
  const Ctx::GraphKey key = graph_key(c, c.d_d32, o, nb);
  iters = 0;
  outer = 0;
  for (;;) {
    HIPCHK(launch_apply(c, FNPF_F64, x, c.d_q, true, nullptr, nullptr, s));
    HIPCHK(launch_resid_to32(f, c.d_q, c.d_r32, c.d_p32, c.d_d32, dinv, c.n_v, c.n_s, c.d_partial, so, si,
                             o.inner_rtol, s));
    if (mg) {
      bool fused = false;
      HIPCHK(mg_vcycle<float>(c, c.d_r32, z, &si->done, o.cheb_degree, s, c.d_partial, &fused));
      HIPCHK(launch_mg_dot_dir(c, FNPF_F32, c.d_r32, z, c.d_p32, c.d_partial, si, 1, s, fused));
    }
    ++outer;
    HIPCHK(hipMemcpyAsync(c.h_sc, c.d_sc, 2 * sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (c.h_sc[0].breakdown == 2) return fail(&c, FNPF_ERR_NAN, "non-finite residual in the FP64 defect correction");
    if (c.h_sc[0].done) break;
    if (outer > o.max_outer || iters >= o.max_iter)
      return fail(&c, FNPF_ERR_NOCONV, "mixed-precision solve did not reach the tolerance");
    for (;;) {
      fnpf_status st = run_chunk(c, 1, key, o.use_graph != 0, s, body);
      if (st != FNPF_OK) return st;
      HIPCHK(hipMemcpyAsync(c.h_sc + 1, si, sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (c.h_sc[1].done || iters + c.h_sc[1].iters >= o.max_iter) break;
    }
    iters += c.h_sc[1].iters;
    if (c.h_sc[1].breakdown == 2) return fail(&c, FNPF_ERR_NAN, "non-finite residual in the FP32 inner PCG");
    // a breakdown of the inner solve still leaves a usable correction; the outer loop decides
    HIPCHK(launch_add_f32(x, c.d_d32, c.n_v, s));
  }
  return FNPF_OK;
}

fnpf_status validate_opts(Ctx &c, const fnpf_solve_opts &o) {
  if (o.precision != 0 && o.precision != 1) return fail(&c, FNPF_ERR_ARG, "opts.precision must be 0 or 1");
  if (o.precond < 0 || o.precond > 2)
    return fail(&c, FNPF_ERR_ARG, "opts.precond must be 0 (none), 1 (Jacobi) or 2 (p-multigrid)");
  if (o.precond == 2 && (o.cheb_degree < 1 || o.cheb_degree > 8))
    return fail(&c, FNPF_ERR_ARG, "opts.cheb_degree must be in 1..8 for the p-multigrid preconditioner");
  if (!(o.rtol >= 0.0) || !(o.atol >= 0.0) || (o.rtol == 0.0 && o.atol == 0.0))
    return fail(&c, FNPF_ERR_ARG, "opts.rtol/atol must be >= 0 and not both 0");
  if (o.max_iter < 1 || o.check_every < 1) return fail(&c, FNPF_ERR_ARG, "opts.max_iter and check_every must be >= 1");
  if (o.extrapolate < 0 || o.extrapolate >= Ctx::kHistMax)
    return fail(&c, FNPF_ERR_ARG, "opts.extrapolate must be in 0..4");
  if (o.use_graph != 0 && o.use_graph != 1) return fail(&c, FNPF_ERR_ARG, "opts.use_graph must be 0 or 1");
  if (o.line_smoother != 0 && o.line_smoother != 1)
    return fail(&c, FNPF_ERR_ARG, "opts.line_smoother must be 0 (point) or 1 (vertical lines)");
  if (o.precision == 1 && (!(o.inner_rtol > 0.0) || !(o.inner_rtol < 1.0) || o.max_outer < 1))
    return fail(&c, FNPF_ERR_ARG, "opts.inner_rtol must be in (0,1) and max_outer >= 1 for the mixed path");
  return FNPF_OK;
}

// Solve with the current geometry: phi (guess in, solution out), surface data phis.
fnpf_status solve_impl(Ctx &c, const double *phis, const double *f, double *phi, const fnpf_solve_opts &o,
                       fnpf_solve_info *info, hipStream_t s) {
  if (info) std::memset(info, 0, sizeof(*info));
  // ||b|| with b = f - A [0; phi_s]
  HIPCHK(launch_set_lift(c.d_p, phis, c.n_v, c.n_s, s));
  HIPCHK(launch_apply(c, FNPF_F64, c.d_p, c.d_q, true, nullptr, nullptr, s));
  HIPCHK(launch_bnorm(f, c.d_q, c.n_v, c.n_s, c.d_partial, c.d_sc, o.rtol, o.atol, s));
  HIPCHK(launch_copy_top(phi, phis, c.n_v, c.n_s, s));
  fnpf_status st = check_err_flag(c, s);
  if (st != FNPF_OK) return st;
  int iters = 0, outer = 0;
  if (o.precision == 0)
    st = pcg64(c, f, phi, o, iters, s);
  else
    st = pcg_mixed(c, f, phi, o, iters, outer, s);
  if (info) {
    info->iters = iters;
    info->outer_iters = outer;
    info->bnorm = std::sqrt(c.h_sc[0].bnorm2);
    info->rel_res = c.h_sc[0].bnorm2 > 0 ? std::sqrt(c.h_sc[0].rr / c.h_sc[0].bnorm2) : std::sqrt(c.h_sc[0].rr);
  }
  return st;
}

fnpf_status geom_impl(Ctx &c, const double *eta, const double *h, hipStream_t s) {
  c.flat_valid = false;
  const bool store = c.apply_variant == 1;
  if (store) {
    fnpf_status st = ensure_G(c);
    if (st != FNPF_OK) return st;
  }
  HIPCHK(launch_geom(c, eta, h, store, false, s));
  c.have_geom = true;
  c.have_geom32 = c.want32;
  c.have_G = store;
  c.mg_stale64 = c.mg_stale32 = true;
  return FNPF_OK;
}

// Linear potential flow: the flat geometry (eta = 0) for depth h, computed once and kept while no
// other call replaces the geometry and h is the same array (fnpf_set_linear drops it).
fnpf_status flat_geometry(Ctx &c, const double *h, hipStream_t s) {
  if (c.flat_valid && c.flat_h == h && c.have_geom && c.have_geom32 == c.want32 &&
      (c.apply_variant != 1 || c.have_G))
    return FNPF_OK;
  fnpf_status st = ensure_flat(c, s);
  if (st != FNPF_OK) return st;
  st = geom_impl(c, c.d_flat, h, s);
  if (st != FNPF_OK) return st;
  c.flat_valid = true;
  c.flat_h = h;
  return FNPF_OK;
}

}  // namespace

namespace fnpf {

Ctx &ctx_of(fnpf_ctx h) { return h->c; }

fnpf_status ctx_ensure32(Ctx &c) { return ensure32(c); }

// geometry from eta + h (H) and h, as the coarse levels of the p-multigrid get it
fnpf_status geom_impl_total(Ctx &c, const double *H, const double *h, hipStream_t s) {
  HIPCHK(launch_geom(c, H, h, false, true, s));
  c.have_geom = true;
  c.have_geom32 = c.want32;
  c.have_G = false;
  return FNPF_OK;
}

}  // namespace fnpf

extern "C" {

void fnpf_default_opts(fnpf_solve_opts *o) {
  if (!o) return;
  o->precision = 0;
  o->precond = 2;
  o->rtol = 1e-8;
  o->atol = 0.0;
  o->max_iter = 20000;
  o->check_every = 8;
  o->inner_rtol = 1e-6;
  o->max_outer = 30;
  o->extrapolate = 4;
  o->cheb_degree = 2;
  o->use_graph = 1;
  o->line_smoother = 0;
}

const char *fnpf_status_string(fnpf_status s) {
  switch (s) {
    case FNPF_OK: return "ok";
    case FNPF_ERR_ARG: return "invalid argument";
    case FNPF_ERR_ALLOC: return "allocation failed";
    case FNPF_ERR_HIP: return "HIP runtime error";
    case FNPF_ERR_GEOM: return "geometry error (eta + h <= 0)";
    case FNPF_ERR_NOCONV: return "PCG did not converge";
    case FNPF_ERR_BREAKDOWN: return "PCG breakdown";
    case FNPF_ERR_NAN: return "non-finite values";
    case FNPF_ERR_STATE: return "invalid call sequence";
  }
  return "unknown status";
}

const char *fnpf_last_error(fnpf_ctx ctx) { return ctx ? ctx->c.err.c_str() : g_create_error.c_str(); }

fnpf_status fnpf_gll(int32_t p, double *nodes, double *weights, double *D) {
  if (p < 1 || p > kMaxP) return FNPF_ERR_ARG;
  gll_host(p, nodes, weights, D);
  return FNPF_OK;
}

fnpf_status fnpf_create(const fnpf_mesh_desc *m, fnpf_ctx *out) {
  g_create_error.clear();
  if (!out) {
    g_create_error = "out is NULL";
    return FNPF_ERR_ARG;
  }
  *out = nullptr;
  if (!m) {
    g_create_error = "mesh is NULL";
    return FNPF_ERR_ARG;
  }
  if ((m->dim != 2 && m->dim != 3) || m->p < 1 || m->p > kMaxP || m->nz < 1 || m->n_eh < 1 || m->n_s < 1 ||
      !m->eh_nodes || !m->eh_corner || !(m->g > 0.0)) {
    g_create_error = "invalid mesh header (dim 2|3, 1 <= p <= 8, nz >= 1, n_eh >= 1, n_s >= 1, g > 0, "
                     "eh_nodes and eh_corner required)";
    return FNPF_ERR_ARG;
  }
  if (m->dim == 2 && m->eh_arc) {
    g_create_error = "eh_arc is only meaningful for dim 3";
    return FNPF_ERR_ARG;
  }
  fnpf_ctx_s *h = new (std::nothrow) fnpf_ctx_s();
  if (!h) return FNPF_ERR_ALLOC;
  Ctx &c = h->c;
  std::vector<double> hm, mw, ms;
  std::vector<uint8_t> flags;
  std::vector<int32_t> cols;
  std::string e = build_host_mesh(*m, c, hm, flags, cols, mw, ms);
  if (!e.empty()) {
    g_create_error = e;
    delete h;
    return FNPF_ERR_ARG;
  }
  c.h_hm = hm;
  c.ncg = c.dim == 3 ? 5 : 3;
  c.apply_lines = c.apply_owner = c.dim == 3;   // default schedule of the 3D apply
  c.h_half_ds.resize(c.nz);
  for (int l = 0; l < c.nz; ++l) c.h_half_ds[l] = 0.5 * (c.h_layer_s[l + 1] - c.h_layer_s[l]);
  // total apply blocks over colours (partials of the fused dot product)
  {
    const int cpb = 256 / c.nh;
    int tot = 0;
    for (const auto &cr : c.colours) tot += (cr.count + cpb - 1) / cpb;
    c.max_colour_blocks = tot;
  }
  hipError_t he = hipGetDevice(&c.device);
  auto bad = [&](hipError_t err) {
    g_create_error = std::string("HIP error during create: ") + hipGetErrorString(err);
    free_all(c);
    delete h;
    return err == hipErrorOutOfMemory ? FNPF_ERR_ALLOC : FNPF_ERR_HIP;
  };
  if (he != hipSuccess) return bad(he);
  static bool uploaded[64] = {false};
  if (c.device >= 0 && c.device < 64 && !uploaded[c.device]) {
    he = upload_constants(c.device);
    if (he != hipSuccess) return bad(he);
    he = init_noalloc_scratch(c.device);
    if (he != hipSuccess) return bad(he);
    uploaded[c.device] = true;
  }
  const int nsides = 2 * (c.dim - 1);
  std::vector<int32_t> tags((size_t)c.n_eh * nsides, 0);
  if (m->eh_face_tag)
    for (size_t k = 0; k < tags.size(); ++k) tags[k] = m->eh_face_tag[k];
#define UP(dst, src, n)                       \
  do {                                        \
    he = upload(&dst, src, n);                \
    if (he != hipSuccess) return bad(he);     \
  } while (0)
#define AL(dst, n)                            \
  do {                                        \
    he = dalloc(&dst, n);                     \
    if (he != hipSuccess) return bad(he);     \
  } while (0)
  UP(c.d_eh_nodes, c.h_eh_nodes.data(), c.h_eh_nodes.size());
  UP(c.d_cols, cols.data(), cols.size());
  {
    UP(c.d_slot, c.h_slot.data(), c.h_slot.size());
    if (c.h_ps_node.empty()) c.h_ps_node.push_back(0);   // a mesh without shared nodes: one unused entry
    if (c.h_ps_slot.empty()) c.h_ps_slot.push_back(0);
    UP(c.d_ps_node, c.h_ps_node.data(), c.h_ps_node.size());
    UP(c.d_ps_ptr, c.h_ps_ptr.data(), c.h_ps_ptr.size());
    UP(c.d_ps_slot, c.h_ps_slot.data(), c.h_ps_slot.size());
    AL(c.d_F64, (size_t)(c.p * c.nz + 1) * std::max<int64_t>(std::max({c.n_slots, c.n_tslots, c.n_gslots}), 1));
    if (c.dim == 3) {
      // the lists may be empty (a mesh within one tile): upload one unused entry then
      if (c.h_tps_node.empty()) c.h_tps_node.push_back(0);
      if (c.h_tps_slot.empty()) c.h_tps_slot.push_back(0);
      UP(c.d_tslot, c.h_tslot.data(), c.h_tslot.size());
      UP(c.d_xch, c.h_xch.data(), c.h_xch.size());
      UP(c.d_tps_node, c.h_tps_node.data(), c.h_tps_node.size());
      UP(c.d_tps_ptr, c.h_tps_ptr.data(), c.h_tps_ptr.size());
      UP(c.d_tps_slot, c.h_tps_slot.data(), c.h_tps_slot.size());
      if (c.h_gx_slot.empty()) c.h_gx_slot.push_back(0);
      UP(c.d_gslot, c.h_gslot.data(), c.h_gslot.size());
      UP(c.d_gx_ptr, c.h_gx_ptr.data(), c.h_gx_ptr.size());
      UP(c.d_gx_slot, c.h_gx_slot.data(), c.h_gx_slot.size());
    }
  }
  UP(c.d_flags, flags.data(), flags.size());
  UP(c.d_face_tag, tags.data(), tags.size());
  UP(c.d_hm, hm.data(), hm.size());
  UP(c.d_sigma, c.h_sigma.data(), c.h_sigma.size());
  UP(c.d_layer_s, c.h_layer_s.data(), c.h_layer_s.size());
  UP(c.d_mlump_w, mw.data(), mw.size());
  UP(c.d_mlump_s, ms.data(), ms.size());
  AL(c.d_cg64, (size_t)c.ncg * c.n_eh * c.nh);
  UP(c.d_half_ds, c.h_half_ds.data(), c.h_half_ds.size());
  AL(c.d_diag, c.n_v);
  AL(c.d_dinv, c.n_v);
  AL(c.d_err, 1);
  AL(c.d_r, c.n_v);
  AL(c.d_p, c.n_v);
  AL(c.d_q, c.n_v);
  AL(c.d_phi, c.n_v);
  for (int k = 0; k < 2; ++k) {
    AL(c.d_sa[k], c.n_s);
    AL(c.d_sp[k], c.n_s);
  }
  AL(c.d_acc_e, c.n_s);
  AL(c.d_acc_p, c.n_s);
  AL(c.d_w, c.n_s);
  AL(c.d_geoH, c.n_s);
  AL(c.d_geoh, c.n_s);
  AL(c.d_wnum, c.n_s);
  AL(c.d_nk, c.n_s);
  AL(c.d_nd, c.n_s);
  {
    const auto uses = partial_uses(c.max_colour_blocks, owner_apply_blocks(c));
    c.n_partial = (int)partial_capacity(uses);
    const std::string le = partial_layout_error(uses, c.n_partial);
    if (!le.empty()) {
      g_create_error = le;
      free_all(c);
      delete h;
      return FNPF_ERR_ARG;
    }
  }
  AL(c.d_partial, c.n_partial);
  AL(c.d_mg_scal, 4);
  AL(c.d_sc, 2);
#undef UP
#undef AL
  he = hipHostMalloc((void **)&c.h_sc, 2 * sizeof(PcgScalars), hipHostMallocDefault);
  if (he != hipSuccess) return bad(he);
  std::memset(c.h_sc, 0, 2 * sizeof(PcgScalars));
  if ((he = hipMemset(c.d_err, 0, sizeof(int32_t))) != hipSuccess) return bad(he);
  if ((he = hipMemset(c.d_phi, 0, c.n_v * sizeof(double))) != hipSuccess) return bad(he);
  if ((he = hipMemset(c.d_sc, 0, 2 * sizeof(PcgScalars))) != hipSuccess) return bad(he);
  if ((he = hipDeviceSynchronize()) != hipSuccess) return bad(he);
  *out = h;
  return FNPF_OK;
}

fnpf_status fnpf_destroy(fnpf_ctx ctx) {
  if (!ctx) return FNPF_ERR_ARG;
  (void)hipDeviceSynchronize();
  free_all(ctx->c);
  delete ctx;
  return FNPF_OK;
}

fnpf_status fnpf_sizes(fnpf_ctx ctx, int64_t *n_v, int64_t *n_s, int64_t *n_e, int32_t *n_colours) {
  if (!ctx) return FNPF_ERR_ARG;
  if (n_v) *n_v = ctx->c.n_v;
  if (n_s) *n_s = ctx->c.n_s;
  if (n_e) *n_e = ctx->c.n_e;
  if (n_colours) *n_colours = (int32_t)ctx->c.colours.size();
  return FNPF_OK;
}

fnpf_status fnpf_surface_interp_weights(fnpf_ctx ctx, int32_t n_pts, const double *pts, int32_t *node, double *w) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (n_pts < 0) return fail(&c, FNPF_ERR_ARG, "n_pts must be >= 0");
  if (n_pts > 0 && (!pts || !node || !w)) return fail(&c, FNPF_ERR_ARG, "pts, node and w must be host arrays");
  const std::string e = surface_interp_weights(c, n_pts, pts, node, w);
  if (!e.empty()) return fail(&c, FNPF_ERR_ARG, e);
  return FNPF_OK;
}

fnpf_status fnpf_node_coords(fnpf_ctx ctx, double *xy) {
  if (!ctx || !xy) return ctx ? fail(&ctx->c, FNPF_ERR_ARG, "xy is NULL") : FNPF_ERR_ARG;
  std::memcpy(xy, ctx->c.h_node_xy.data(), ctx->c.h_node_xy.size() * sizeof(double));
  return FNPF_OK;
}

fnpf_status fnpf_set_apply_variant(fnpf_ctx ctx, int32_t variant) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (variant != 0 && variant != 1 && variant != 6 && variant != 7)
    return fail(&c, FNPF_ERR_ARG, "apply variant must be 0, 1, 6 or 7");
  c.apply_lines = c.dim == 3 && (variant == 0 || variant == 6);
  c.apply_owner = c.dim == 3 && variant == 0;
  if (variant >= 6) variant = 0;   // 6 and 7 are schedules of the fused apply (apply_lines, apply_owner)
  if (variant == c.apply_variant) return FNPF_OK;
  c.apply_variant = variant;
  if (variant == 1) {
    fnpf_status st = ensure_G(c);
    if (st != FNPF_OK) return st;
    c.have_geom = c.have_geom32 = false;   // factors must be (re)computed by fnpf_geom
  }
  return FNPF_OK;
}

fnpf_status fnpf_enable_fp32(fnpf_ctx ctx) {
  if (!ctx) return FNPF_ERR_ARG;
  return ensure32(ctx->c);
}

fnpf_status fnpf_geom(fnpf_ctx ctx, const double *eta, const double *h, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!eta || !h) return fail(&c, FNPF_ERR_ARG, "fnpf_geom: eta and h must be device pointers");
  return geom_impl(c, eta, h, (hipStream_t)stream);
}

fnpf_status fnpf_export_geometry(fnpf_ctx ctx, fnpf_dtype dtype, void *G, double *diag, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  hipStream_t s = (hipStream_t)stream;
  if (dtype != FNPF_F64 && dtype != FNPF_F32) return fail(&c, FNPF_ERR_ARG, "bad dtype");
  if (!c.have_geom) return fail(&c, FNPF_ERR_STATE, "fnpf_export_geometry before fnpf_geom");
  if (dtype == FNPF_F32 && !c.have_geom32) return fail(&c, FNPF_ERR_STATE, "no FP32 factors (enable the mixed path)");
  if (!c.have_G) {
    // factors are not stored by the fused-geometry variant: evaluate them from the saved column data
    fnpf_status st = ensure_G(c);
    if (st != FNPF_OK) return st;
    HIPCHK(launch_geom(c, c.d_geoH, c.d_geoh, true, true, s));
    c.have_G = true;
  }
  const size_t ng = (size_t)c.n_e * c.ng * c.np;
  if (G) {
    if (dtype == FNPF_F64)
      HIPCHK(hipMemcpyAsync(G, c.d_G64, ng * sizeof(double), hipMemcpyDeviceToDevice, s));
    else
      HIPCHK(hipMemcpyAsync(G, c.d_G32, ng * sizeof(float), hipMemcpyDeviceToDevice, s));
  }
  if (diag) {
    HIPCHK(ensure_diag(c, s));
    HIPCHK(hipMemcpyAsync(diag, c.d_diag, c.n_v * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  return FNPF_OK;
}

fnpf_status fnpf_laplace_apply(fnpf_ctx ctx, fnpf_dtype dtype, const void *x, void *y, int32_t mask, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!x || !y) return fail(&c, FNPF_ERR_ARG, "fnpf_laplace_apply: x and y must be device pointers");
  if (x == y) return fail(&c, FNPF_ERR_ARG, "fnpf_laplace_apply: x and y must not alias");
  if (dtype != FNPF_F64 && dtype != FNPF_F32) return fail(&c, FNPF_ERR_ARG, "bad dtype");
  if (!c.have_geom) return fail(&c, FNPF_ERR_STATE, "fnpf_laplace_apply before fnpf_geom");
  if (dtype == FNPF_F32 && !c.have_geom32)
    return fail(&c, FNPF_ERR_STATE, "no FP32 factors: call fnpf_enable_fp32, then fnpf_geom");
  HIPCHK(launch_apply(c, dtype, x, y, mask != 0, nullptr, nullptr, (hipStream_t)stream));
  return FNPF_OK;
}

fnpf_status fnpf_laplace_apply_noalloc(fnpf_ctx ctx, fnpf_dtype dtype, const void *x, void *y, int32_t mask,
                                       void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!x || !y) return fail(&c, FNPF_ERR_ARG, "fnpf_laplace_apply_noalloc: x and y must be device pointers");
  if (x == y) return fail(&c, FNPF_ERR_ARG, "fnpf_laplace_apply_noalloc: x and y must not alias");
  if (dtype != FNPF_F64 && dtype != FNPF_F32) return fail(&c, FNPF_ERR_ARG, "bad dtype");
  if (!c.have_geom) return fail(&c, FNPF_ERR_STATE, "fnpf_laplace_apply_noalloc before fnpf_geom");
  if (dtype == FNPF_F32 && !c.have_geom32)
    return fail(&c, FNPF_ERR_STATE, "no FP32 factors: call fnpf_enable_fp32, then fnpf_geom");
  // only the owner-computes schedule uses face slots; the others need no scratch
  const size_t word = dtype == FNPF_F64 ? sizeof(double) : sizeof(float);
  const size_t need = owner_apply_active(c) ? (size_t)(c.p * c.nz + 1) * (size_t)c.n_tslots * word : 0;
  if (need > noalloc_scratch_bytes()) {
    char buf[200];
    std::snprintf(buf, sizeof buf,
                  "fnpf_laplace_apply_noalloc: the face slots need %zu bytes, the scratch holds %zu; use "
                  "fnpf_laplace_apply", need, noalloc_scratch_bytes());
    return fail(&c, FNPF_ERR_ARG, buf);
  }
  void *scr = noalloc_scratch(c.device);
  if (scr == nullptr) return fail(&c, FNPF_ERR_STATE, "scratch address unknown on this device");
  HIPCHK(launch_apply(c, dtype, x, y, mask != 0, nullptr, nullptr, (hipStream_t)stream, scr));
  return FNPF_OK;
}

fnpf_status fnpf_line_smoother_apply(fnpf_ctx ctx, fnpf_dtype dtype, const void *r, void *z, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!r || !z) return fail(&c, FNPF_ERR_ARG, "fnpf_line_smoother_apply: r and z must be device pointers");
  if (r == z) return fail(&c, FNPF_ERR_ARG, "fnpf_line_smoother_apply: r and z must not alias");
  if (dtype != FNPF_F64 && dtype != FNPF_F32) return fail(&c, FNPF_ERR_ARG, "bad dtype");
  if (!c.have_geom) return fail(&c, FNPF_ERR_STATE, "fnpf_line_smoother_apply before fnpf_geom");
  if (dtype == FNPF_F32 && !c.have_geom32)
    return fail(&c, FNPF_ERR_STATE, "no FP32 data: call fnpf_enable_fp32, then fnpf_geom");
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(line_setup(c, s));
  if (dtype == FNPF_F64)
    HIPCHK(line_apply<double>(c, (const double *)r, (double *)z, s));
  else
    HIPCHK(line_apply<float>(c, (const float *)r, (float *)z, s));
  return check_err_flag(c, s);
}

fnpf_status fnpf_neumann_load(fnpf_ctx ctx, const double *q, double *f, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!q || !f) return fail(&c, FNPF_ERR_ARG, "fnpf_neumann_load: q and f must be device pointers");
  if (!c.have_geom) return fail(&c, FNPF_ERR_STATE, "fnpf_neumann_load before fnpf_geom");
  HIPCHK(launch_neumann(c, q, f, (hipStream_t)stream));
  return FNPF_OK;
}

fnpf_status fnpf_solve(fnpf_ctx ctx, const double *phis, const double *f, double *phi, const fnpf_solve_opts *opts,
                       fnpf_solve_info *info, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!phis || !phi) return fail(&c, FNPF_ERR_ARG, "fnpf_solve: phi_surface and phi must be device pointers");
  fnpf_solve_opts o;
  fnpf_default_opts(&o);
  if (opts) o = *opts;
  fnpf_status st = validate_opts(c, o);
  if (st != FNPF_OK) return st;
  if (!c.have_geom) return fail(&c, FNPF_ERR_STATE, "fnpf_solve before fnpf_geom");
  if (o.precision == 1 && !c.have_geom32)
    return fail(&c, FNPF_ERR_STATE, "mixed solve needs FP32 factors: call fnpf_enable_fp32, then fnpf_geom");
  return solve_impl(c, phis, f, phi, o, info, (hipStream_t)stream);
}

fnpf_status fnpf_w_surface(fnpf_ctx ctx, const double *phi, double *w, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!phi || !w) return fail(&c, FNPF_ERR_ARG, "fnpf_w_surface: phi and w_s must be device pointers");
  if (!c.have_geom) return fail(&c, FNPF_ERR_STATE, "fnpf_w_surface before fnpf_geom");
  HIPCHK(launch_wsurf(c, phi, w, (hipStream_t)stream));
  return FNPF_OK;
}

fnpf_status fnpf_rhs(fnpf_ctx ctx, const double *eta, const double *phis, const double *w, double *deta,
                     double *dphi, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!eta || !phis || !w || !deta || !dphi) return fail(&c, FNPF_ERR_ARG, "fnpf_rhs: null device pointer");
  if (deta == eta || deta == phis || dphi == eta || dphi == phis)
    return fail(&c, FNPF_ERR_ARG, "fnpf_rhs: outputs must not alias the inputs");
  RkStageArgs a{};
  a.linear = c.linear ? 1 : 0;
  a.stage = -1;
  a.out_e = deta;
  a.out_p = dphi;
  HIPCHK(stage_rhs(c, eta, phis, w, a, (hipStream_t)stream));
  return FNPF_OK;
}

fnpf_status fnpf_set_linear(fnpf_ctx ctx, int32_t linear) {
  if (!ctx) return FNPF_ERR_ARG;
  ctx->c.linear = linear != 0;
  ctx->c.flat_valid = false;
  return FNPF_OK;
}

fnpf_status fnpf_set_surface_quadrature(fnpf_ctx ctx, int32_t nq) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (nq == 0) {
    sq_free(c);
    return FNPF_OK;
  }
  if (nq < c.p + 1 || nq > kMaxSurfaceNq)
    return fail(&c, FNPF_ERR_ARG, "surface quadrature: nq must be 0 or in [p + 1, 24]");
  HIPCHK(hipDeviceSynchronize());   // tables may be in use by queued work
  const char *err = sq_setup(c, nq);
  if (err) {
    sq_free(c);
    return fail(&c, std::strstr(err, "Jacobian") ? FNPF_ERR_GEOM : FNPF_ERR_ALLOC, err);
  }
  return FNPF_OK;
}

fnpf_status fnpf_surface_quadrature_info(fnpf_ctx ctx, int32_t *nq, int32_t *iters, double *lam_lo,
                                         double *lam_hi) {
  if (!ctx) return FNPF_ERR_ARG;
  const Ctx &c = ctx->c;
  if (nq) *nq = c.sq_nq;
  if (iters) *iters = c.sq_iters;
  if (lam_lo) *lam_lo = c.sq_lo;
  if (lam_hi) *lam_hi = c.sq_hi;
  return FNPF_OK;
}

fnpf_status fnpf_multigrid_info(fnpf_ctx ctx, int32_t *levels, double *lam64, double *lam32, int32_t cap) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (cap < 0) return fail(&c, FNPF_ERR_ARG, "cap must be >= 0");
  const int nl = c.mg_built ? (int)c.mg.size() + 1 : 0;
  if (levels) *levels = nl;
  if (nl == 0 || cap == 0 || (!lam64 && !lam32)) return FNPF_OK;
  std::vector<double> h((size_t)2 * nl);
  HIPCHK(hipDeviceSynchronize());   // the estimates are written on the device by the solves' streams
  HIPCHK(hipMemcpy(h.data(), c.d_mg_lam, sizeof(double) * 2 * nl, hipMemcpyDeviceToHost));
  for (int l = 0; l < nl && l < cap; ++l) {
    if (lam64) lam64[l] = h[l];
    if (lam32) lam32[l] = h[nl + l];
  }
  return FNPF_OK;
}

fnpf_status fnpf_set_modal_filter(fnpf_ctx ctx, int32_t cutoff, double alpha, int32_t order) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (cutoff < 0) {
    c.filter_cutoff = -1;
    return FNPF_OK;
  }
  if (cutoff >= c.p) return fail(&c, FNPF_ERR_ARG, "modal filter cutoff must satisfy 0 <= cutoff < p");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(&c, FNPF_ERR_ARG, "modal filter alpha must be >= 0");
  if (order < 1) return fail(&c, FNPF_ERR_ARG, "modal filter order must be >= 1");
  const int n1 = c.p + 1;
  if (!c.d_filt_M) {
    std::vector<double> inv(c.n_s, 0.0);
    for (int32_t v : c.h_eh_nodes) inv[v] += 1.0;
    for (auto &x : inv) x = 1.0 / x;
    HIPCHK(upload(&c.d_filt_inv_mult, inv.data(), inv.size()));
    HIPCHK(dalloc(&c.d_filt_M, (size_t)n1 * n1));
    HIPCHK(dalloc(&c.d_filt_acc, c.n_s));
    HIPCHK(dalloc(&c.d_filt_tmp, c.n_s));
  }
  std::vector<double> M((size_t)n1 * n1);
  modal_filter_matrix(c.p, cutoff, alpha, order, M.data());
  HIPCHK(hipMemcpy(c.d_filt_M, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice));
  c.filter_cutoff = cutoff;
  c.filter_alpha = alpha;
  c.filter_order = order;
  return FNPF_OK;
}

fnpf_status fnpf_modal_filter(fnpf_ctx ctx, const double *f, double *out, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!f || !out) return fail(&c, FNPF_ERR_ARG, "fnpf_modal_filter: null device pointer");
  if (f == out) return fail(&c, FNPF_ERR_ARG, "fnpf_modal_filter: out must not alias f");
  if (c.filter_cutoff < 0) return fail(&c, FNPF_ERR_STATE, "fnpf_modal_filter: no filter set");
  HIPCHK(launch_modal_filter(c, f, out, false, (hipStream_t)stream));
  return FNPF_OK;
}

fnpf_status fnpf_modal_filter_vjp(fnpf_ctx ctx, const double *out_bar, double *f_bar, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!out_bar || !f_bar) return fail(&c, FNPF_ERR_ARG, "fnpf_modal_filter_vjp: null device pointer");
  if (out_bar == f_bar) return fail(&c, FNPF_ERR_ARG, "fnpf_modal_filter_vjp: f_bar must not alias out_bar");
  if (c.filter_cutoff < 0) return fail(&c, FNPF_ERR_STATE, "fnpf_modal_filter_vjp: no filter set");
  HIPCHK(launch_modal_filter(c, out_bar, f_bar, true, (hipStream_t)stream));
  return FNPF_OK;
}

fnpf_status fnpf_set_relaxation(fnpf_ctx ctx, const double *cr, const double *ec, const double *es, const double *pc,
                                const double *ps, double omega, double t_ramp) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!cr) {
    c.have_relax = false;
    return FNPF_OK;
  }
  if (!ec || !es || !pc || !ps) return fail(&c, FNPF_ERR_ARG, "fnpf_set_relaxation: null host array");
  for (int64_t n = 0; n < c.n_s; ++n)
    if (!(cr[n] >= 0.0 && cr[n] <= 1.0)) return fail(&c, FNPF_ERR_ARG, "relaxation weights must lie in [0, 1]");
  const double *src[5] = {cr, ec, es, pc, ps};
  double **dst[5] = {&c.d_cr, &c.d_rec, &c.d_res, &c.d_rpc, &c.d_rps};
  for (int k = 0; k < 5; ++k) {
    if (!*dst[k]) HIPCHK(dalloc(dst[k], c.n_s));
    HIPCHK(hipMemcpy(*dst[k], src[k], c.n_s * sizeof(double), hipMemcpyHostToDevice));
  }
  c.relax_omega = omega;
  c.relax_tramp = t_ramp;
  c.have_relax = true;
  return FNPF_OK;
}

fnpf_status fnpf_rk4_step(fnpf_ctx ctx, double *eta, double *phis, const double *h, double t, double dt,
                          const fnpf_solve_opts *opts, double *tape, fnpf_solve_info *info, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  hipStream_t s = (hipStream_t)stream;
  if (!eta || !phis || !h) return fail(&c, FNPF_ERR_ARG, "fnpf_rk4_step: eta, phi_s and h must be device pointers");
  if (!(dt > 0.0)) return fail(&c, FNPF_ERR_ARG, "fnpf_rk4_step: dt must be > 0");
  fnpf_solve_opts o;
  fnpf_default_opts(&o);
  if (opts) o = *opts;
  fnpf_status st = validate_opts(c, o);
  if (st != FNPF_OK) return st;
  if (o.precision == 1) {
    st = ensure32(c);
    if (st != FNPF_OK) return st;
  }
  if (info) std::memset(info, 0, 4 * sizeof(fnpf_solve_info));
  if (o.extrapolate) {
    st = ensure_history(c, c.hist, o.extrapolate + 1);
    if (st != FNPF_OK) return st;
    if (c.hist.dt != dt) c.hist.count = 0;   // a new step size starts a new sequence
  }
  const double *ein = eta, *pin = phis;
  const size_t rec = (size_t)c.n_v + 2 * (size_t)c.n_s;
  if (c.linear) {
    // linear potential flow: one flat geometry (eta = 0) serves every stage and step
    st = flat_geometry(c, h, s);
    if (st != FNPF_OK) return st;
  }
  for (int stg = 0; stg < 4; ++stg) {
    if (tape) {
      HIPCHK(hipMemcpyAsync(tape + stg * rec + c.n_v, ein, c.n_s * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(tape + stg * rec + c.n_v + c.n_s, pin, c.n_s * sizeof(double), hipMemcpyDeviceToDevice,
                            s));
    }
    if (!c.linear) {
      st = geom_impl(c, ein, h, s);
      if (st != FNPF_OK) return st;
    }
    if (o.extrapolate) {
      hipError_t e = hipSuccess;
      history_extrapolate(c.hist, stg, o.extrapolate, c.d_phi, c.n_v, s, e);
      HIPCHK(e);
    }
    st = solve_impl(c, pin, nullptr, c.d_phi, o, info ? info + stg : nullptr, s);
    if (st != FNPF_OK) return st;
    if (o.extrapolate) HIPCHK(history_record(c.hist, stg, c.d_phi, c.n_v, s));
    if (tape) HIPCHK(hipMemcpyAsync(tape + stg * rec, c.d_phi, c.n_v * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIPCHK(launch_wsurf(c, c.d_phi, c.d_w, s));
    RkStageArgs a{};
    a.linear = c.linear ? 1 : 0;
    a.eta0 = eta;
    a.phi0 = phis;
    a.acc_e = c.d_acc_e;
    a.acc_p = c.d_acc_p;
    a.stage = stg;
    a.bdt = kRkB[stg] * dt;
    if (stg < 3) {
      a.cdt = kRkC[stg + 1] * dt;
      a.out_e = c.d_sa[stg & 1];
      a.out_p = c.d_sp[stg & 1];
    } else {
      a.out_e = eta;
      a.out_p = phis;
      if (c.have_relax) {
        const double tn = t + dt;
        double r = 1.0;
        if (c.relax_tramp > 0.0 && tn < c.relax_tramp) r = 0.5 * (1.0 - std::cos(M_PI * tn / c.relax_tramp));
        a.cr = c.d_cr;
        a.ec = c.d_rec;
        a.es = c.d_res;
        a.pc = c.d_rpc;
        a.ps = c.d_rps;
        a.rc = r * std::cos(c.relax_omega * tn);
        a.rs = r * std::sin(c.relax_omega * tn);
      }
    }
    HIPCHK(stage_rhs(c, ein, pin, c.d_w, a, s));
    ein = a.out_e;
    pin = a.out_p;
  }
  if (c.filter_cutoff >= 0) {
    // modal filter of the new surface state, after relaxation
    double *fields[2] = {eta, phis};
    for (double *f : fields) {
      HIPCHK(launch_modal_filter(c, f, c.d_filt_tmp, false, s));
      HIPCHK(hipMemcpyAsync(f, c.d_filt_tmp, c.n_s * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
  }
  if (o.extrapolate)
    history_advance(c.hist, t, dt, true);
  else
    c.hist.count = 0;  // a step taken without recording breaks the sequence
  return FNPF_OK;
}

fnpf_status fnpf_rhs_vjp(fnpf_ctx ctx, const double *eta, const double *phis, const double *w, const double *deta_bar,
                         const double *dphi_bar, double *eta_bar, double *phis_bar, double *w_bar, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!eta || !phis || !w || !deta_bar || !dphi_bar || !eta_bar || !phis_bar || !w_bar)
    return fail(&c, FNPF_ERR_ARG, "fnpf_rhs_vjp: null device pointer");
  HIPCHK(stage_rhs_vjp(c, eta, phis, w, deta_bar, dphi_bar, eta_bar, phis_bar, w_bar, (hipStream_t)stream));
  return FNPF_OK;
}

fnpf_status fnpf_w_surface_vjp(fnpf_ctx ctx, const double *w, const double *w_bar, double *phi_bar, double *eta_bar,
                               double *h_bar, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!w || !w_bar || !phi_bar || !eta_bar || !h_bar)
    return fail(&c, FNPF_ERR_ARG, "fnpf_w_surface_vjp: null device pointer");
  if (!c.have_geom) return fail(&c, FNPF_ERR_STATE, "fnpf_w_surface_vjp before fnpf_geom");
  HIPCHK(launch_wsurf_vjp(c, w_bar, w, phi_bar, eta_bar, h_bar, (hipStream_t)stream));
  return FNPF_OK;
}

fnpf_status fnpf_solve_adjoint(fnpf_ctx ctx, const double *phi_bar, double *lambda, const fnpf_solve_opts *opts,
                               fnpf_solve_info *info, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  hipStream_t s = (hipStream_t)stream;
  if (!phi_bar || !lambda) return fail(&c, FNPF_ERR_ARG, "fnpf_solve_adjoint: null device pointer");
  fnpf_solve_opts o;
  fnpf_default_opts(&o);
  if (opts) o = *opts;
  fnpf_status st = validate_opts(c, o);
  if (st != FNPF_OK) return st;
  if (!c.have_geom) return fail(&c, FNPF_ERR_STATE, "fnpf_solve_adjoint before fnpf_geom");
  if (o.precision == 1 && !c.have_geom32)
    return fail(&c, FNPF_ERR_STATE, "mixed adjoint solve needs FP32 factors: fnpf_enable_fp32, then fnpf_geom");
  st = ensure_adjoint(c, s);
  if (st != FNPF_OK) return st;
  // the operator is symmetric: A_II lambda_I = phi_bar_I with lambda_S = 0
  return solve_impl(c, c.d_zero_s, phi_bar, lambda, o, info, s);
}

fnpf_status fnpf_geom_vjp(fnpf_ctx ctx, const double *lambda, const double *phi, double *eta_bar, double *h_bar,
                          void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  if (!lambda || !phi || !eta_bar || !h_bar) return fail(&c, FNPF_ERR_ARG, "fnpf_geom_vjp: null device pointer");
  if (!c.have_geom) return fail(&c, FNPF_ERR_STATE, "fnpf_geom_vjp before fnpf_geom");
  HIPCHK(launch_geom_vjp(c, lambda, phi, eta_bar, h_bar, (hipStream_t)stream));
  return FNPF_OK;
}

fnpf_status fnpf_rk4_step_vjp(fnpf_ctx ctx, const double *h, double t, double dt, const double *tape,
                              double *eta_bar, double *phis_bar, double *h_bar, const fnpf_solve_opts *opts,
                              fnpf_solve_info *info, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  hipStream_t s = (hipStream_t)stream;
  if (!h || !tape || !eta_bar || !phis_bar || !h_bar)
    return fail(&c, FNPF_ERR_ARG, "fnpf_rk4_step_vjp: null device pointer");
  if (!(dt > 0.0)) return fail(&c, FNPF_ERR_ARG, "fnpf_rk4_step_vjp: dt must be > 0");
  fnpf_solve_opts o;
  fnpf_default_opts(&o);
  if (opts) o = *opts;
  fnpf_status st = validate_opts(c, o);
  if (st != FNPF_OK) return st;
  if (o.precision == 1) {
    st = ensure32(c);
    if (st != FNPF_OK) return st;
  }
  st = ensure_adjoint(c, s);
  if (st != FNPF_OK) return st;
  if (c.linear) {
    st = ensure_flat(c, s);
    if (st != FNPF_OK) return st;
  }
  if (info) std::memset(info, 0, 4 * sizeof(fnpf_solve_info));
  if (o.extrapolate) {
    // the adjoint solutions of consecutive step VJPs (t, t - dt, ...) form a sequence backwards
    // in time; their history extrapolates the initial guesses like the forward one
    st = ensure_history(c, c.ahist, o.extrapolate + 1);
    if (st != FNPF_OK) return st;
    const bool next = c.ahist.count > 0 && c.ahist.dt == dt &&
                      std::fabs(c.ahist.t - dt - t) <= 1e-9 * std::max(dt, std::fabs(t));
    if (!next) c.ahist.count = 0;
  } else {
    c.ahist.count = 0;
  }
  const size_t rec = (size_t)c.n_v + 2 * (size_t)c.n_s;
  const int64_t ns = c.n_s;
  if (c.filter_cutoff >= 0) {
    // the modal filter acted last: ybar <- F^T ybar
    double *bars[2] = {eta_bar, phis_bar};
    for (double *b : bars) {
      HIPCHK(launch_fill(c.d_filt_tmp, 0.0, ns, s));
      HIPCHK(launch_modal_filter(c, b, c.d_filt_tmp, true, s));
      HIPCHK(hipMemcpyAsync(b, c.d_filt_tmp, ns * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
  }
  // relaxation acted before: y_{n+1} = (1 - C_r) (y_n + sum b dt k) + C_r f_true(t + dt)
  if (c.have_relax) {
    HIPCHK(launch_relax_vjp(eta_bar, c.d_cr, ns, s));
    HIPCHK(launch_relax_vjp(phis_bar, c.d_cr, ns, s));
  }
  // accumulators of y_n bar start with the direct path
  HIPCHK(hipMemcpyAsync(c.d_acce, eta_bar, ns * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(c.d_accp, phis_bar, ns * sizeof(double), hipMemcpyDeviceToDevice, s));
  for (int stg = 3; stg >= 0; --stg) {
    const double *phi_s = tape + stg * rec;
    const double *eta_s = phi_s + c.n_v;
    const double *pin_s = eta_s + ns;
    // k bar of this stage: b_s dt ybar' + c_{s+1} dt Ybar_{s+1}
    if (stg == 3) {
      HIPCHK(launch_lincomb(c.d_kbe, kRkB[stg] * dt, eta_bar, 0.0, nullptr, ns, s));
      HIPCHK(launch_lincomb(c.d_kbp, kRkB[stg] * dt, phis_bar, 0.0, nullptr, ns, s));
    } else {
      HIPCHK(launch_lincomb(c.d_kbe, kRkB[stg] * dt, eta_bar, kRkC[stg + 1] * dt, c.d_ybe, ns, s));
      HIPCHK(launch_lincomb(c.d_kbp, kRkB[stg] * dt, phis_bar, kRkC[stg + 1] * dt, c.d_ybp, ns, s));
    }
    // stage VJP at Y_s (linear potential flow: the geometry is the flat one, so its adjoint
    // reaches h only; the eta adjoint of the geometry goes to a discarded scratch vector)
    st = c.linear ? flat_geometry(c, h, s) : geom_impl(c, eta_s, h, s);
    if (st != FNPF_OK) return st;
    double *geo_eta_bar = c.linear ? c.d_scr_s : c.d_ybe;
    HIPCHK(launch_wsurf(c, phi_s, c.d_w, s));
    HIPCHK(launch_fill(c.d_ybe, 0.0, ns, s));
    HIPCHK(launch_fill(c.d_ybp, 0.0, ns, s));
    HIPCHK(launch_fill(c.d_wbar, 0.0, ns, s));
    HIPCHK(stage_rhs_vjp(c, eta_s, pin_s, c.d_w, c.d_kbe, c.d_kbp, c.d_ybe, c.d_ybp, c.d_wbar, s));
    HIPCHK(launch_fill(c.d_phibar, 0.0, c.n_v, s));
    HIPCHK(launch_wsurf_vjp(c, c.d_wbar, c.d_w, c.d_phibar, geo_eta_bar, h_bar, s));
    if (o.extrapolate) {
      hipError_t e = hipSuccess;
      history_extrapolate(c.ahist, stg, o.extrapolate, c.d_lam, c.n_v, s, e);
      HIPCHK(e);
    }
    st = solve_impl(c, c.d_zero_s, c.d_phibar, c.d_lam, o, info ? info + stg : nullptr, s);
    if (st != FNPF_OK) return st;
    if (o.extrapolate) HIPCHK(history_record(c.ahist, stg, c.d_lam, c.n_v, s));
    HIPCHK(launch_apply(c, FNPF_F64, c.d_lam, c.d_q, false, nullptr, nullptr, s));
    HIPCHK(launch_surface_adj(c.d_ybp, c.d_phibar, c.d_q, c.n_v, ns, s));
    HIPCHK(launch_geom_vjp(c, c.d_lam, phi_s, geo_eta_bar, h_bar, s));
    HIPCHK(launch_lincomb(c.d_acce, 1.0, c.d_acce, 1.0, c.d_ybe, ns, s));
    HIPCHK(launch_lincomb(c.d_accp, 1.0, c.d_accp, 1.0, c.d_ybp, ns, s));
  }
  HIPCHK(hipMemcpyAsync(eta_bar, c.d_acce, ns * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(phis_bar, c.d_accp, ns * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (o.extrapolate) history_advance(c.ahist, t, dt, c.ahist.count > 0);
  return FNPF_OK;
}

fnpf_status fnpf_get_warm_start(fnpf_ctx ctx, double *phi, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  c.hist.count = 0;
  if (!phi) return fail(&c, FNPF_ERR_ARG, "phi is NULL");
  HIPCHK(hipMemcpyAsync(phi, c.d_phi, c.n_v * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return FNPF_OK;
}

fnpf_status fnpf_set_warm_start(fnpf_ctx ctx, const double *phi, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  c.hist.count = 0;
  if (phi)
    HIPCHK(hipMemcpyAsync(c.d_phi, phi, c.n_v * sizeof(double), hipMemcpyDeviceToDevice, (hipStream_t)stream));
  else
    HIPCHK(launch_fill(c.d_phi, 0.0, c.n_v, (hipStream_t)stream));
  return FNPF_OK;
}

fnpf_status fnpf_sync(fnpf_ctx ctx, void *stream) {
  if (!ctx) return FNPF_ERR_ARG;
  Ctx &c = ctx->c;
  return check_err_flag(c, (hipStream_t)stream);
}

}  // extern "C"
