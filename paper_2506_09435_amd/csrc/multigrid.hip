// p-multigrid preconditioner for the Laplace system on A_II.
//
// The paper solves the Laplace system with CG preconditioned by algebraic multigrid (Sec. 4
// solver settings).  Here the preconditioner is a V-cycle over polynomial degrees of the same
// extruded mesh, p -> p/2 -> ... -> 1: every level is a full context of the library at its
// degree (same columns, layers and corners; geometry from eta + h and h interpolated to its
// surface nodes), with Chebyshev smoothing of the Jacobi-scaled operator D^-1 A.  The transfer
// between a level of degree pf and the next of degree pc = pf/2 is the tensor-product Lagrange
// interpolation P of the coarse element polynomial at the fine GLL nodes, element by element;
// the restriction is its exact transpose.  With the same polynomial before and after the coarse
// correction, the V-cycle is a fixed symmetric positive definite operator, so the outer
// iteration stays plain CG.
//
// Deterministic: each fine node takes its interpolated value from the column that owns it, the
// restriction counts each fine node once (in its owner column, the shared layer level in the
// upper layer), and coarse sums are assembled with the owner-computes face slots of the coarse
// level; every reduction has a fixed order.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <utility>
#include <vector>

#include "fnpf_internal.h"

namespace fnpf {

namespace {

constexpr int kMgCoarseSteps = 10;      // Chebyshev steps on the coarsest level
constexpr double kMgSafety = 1.1;       // upper end of the smoothing interval over the estimate
constexpr double kMgSmoothRatio = 24.0; // smoothing interval [lmax / 24, lmax]
constexpr double kMgCoarseRatio = 30.0;
constexpr int kLanczosSteps = 20;             // first estimate of the largest eigenvalue
constexpr int kPowNext = 1;                   // power iterations per geometry update after that
constexpr int kLzScalars = 2 * kLanczosSteps + 8;
constexpr int kMgCoef = 32;                   // coefficient-table entries per level
// Grid of the streaming vector kernels of the cycle: FP32 passes move half the bytes per element
// and need twice the blocks in flight to keep HBM busy (FP64 passes are slower with the larger
// grid).  Their reductions use the same grid, so partial counts follow it; the context's partial
// buffer is sized from the table of partials.h, which lists both grids (up to two sums per block).
template <typename T>
constexpr int kVB = sizeof(T) == 4 ? 2 * kVecBlocks : kVecBlocks;
static_assert(kVB<float> == 2 * kPartialVecBlocks && kVB<double> == kPartialVecBlocks,
              "vector grids must match the partial-sum table (partials.h)");

// Interpolation tables for a fine degree pf (2..8) and pc = pf / 2:
//   c_IP[pf][r (pc+1) + a] = l^c_a(x^f_r)   coarse Lagrange basis at the fine GLL nodes
//   c_IS[pf][a (pf+1) + i] = l^f_i(x^c_a)   fine Lagrange basis at the coarse GLL nodes
__constant__ double c_IP64[kMaxN1][kMaxN1 * kMaxN1];
__constant__ float c_IP32[kMaxN1][kMaxN1 * kMaxN1];
__constant__ double c_IS64[kMaxN1][kMaxN1 * kMaxN1];

template <typename T>
__device__ __forceinline__ T ip(int pf, int k);
template <>
__device__ __forceinline__ double ip<double>(int pf, int k) { return c_IP64[pf][k]; }
template <>
__device__ __forceinline__ float ip<float>(int pf, int k) { return c_IP32[pf][k]; }

double lagrange(const double *X, int n1, int j, double x) {
  double v = 1.0;
  for (int m = 0; m < n1; ++m)
    if (m != j) v *= (x - X[m]) / (X[j] - X[m]);
  return v;
}

hipError_t upload_tables() {
  static double IP[kMaxN1][kMaxN1 * kMaxN1];
  static float IP32[kMaxN1][kMaxN1 * kMaxN1];
  static double IS[kMaxN1][kMaxN1 * kMaxN1];
  std::memset(IP, 0, sizeof IP);
  std::memset(IP32, 0, sizeof IP32);
  std::memset(IS, 0, sizeof IS);
  for (int pf = 2; pf <= kMaxP; ++pf) {
    const int pc = pf / 2;
    double xf[kMaxN1], xc[kMaxN1];
    gll_host(pf, xf, nullptr, nullptr);
    gll_host(pc, xc, nullptr, nullptr);
    for (int r = 0; r <= pf; ++r)
      for (int a = 0; a <= pc; ++a) {
        IP[pf][r * (pc + 1) + a] = lagrange(xc, pc + 1, a, xf[r]);
        IP32[pf][r * (pc + 1) + a] = (float)IP[pf][r * (pc + 1) + a];
      }
    for (int a = 0; a <= pc; ++a)
      for (int i = 0; i <= pf; ++i) IS[pf][a * (pf + 1) + i] = lagrange(xf, pf + 1, i, xc[a]);
  }
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_IP64), IP, sizeof IP);
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_IP32), IP32, sizeof IP32);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_IS64), IS, sizeof IS);
}

template <int P, int DIM>
struct Lay {
  static constexpr int N1 = P + 1;
  static constexpr int NH = DIM == 3 ? N1 * N1 : N1;
  static constexpr int CPB = 256 / NH;
  static constexpr int NT = CPB * NH;
};

// ---- transfer kernels ------------------------------------------------------------------------

// Coarse surface data (eta + h and h) at the coarse nodes from the fine nodal values.
template <int PF, int DIM>
__global__ __launch_bounds__(256) void k_mg_surf(const double *__restrict__ Hf, const double *__restrict__ hf,
                                                 const int32_t *__restrict__ nodes_f,
                                                 const int32_t *__restrict__ nodes_c,
                                                 const uint8_t *__restrict__ flags_c, int ncols,
                                                 double *__restrict__ Hc, double *__restrict__ hc) {
  constexpr int PC = PF / 2, N1F = PF + 1, N1C = PC + 1;
  constexpr int NHC = Lay<PC, DIM>::NH, NHF = Lay<PF, DIM>::NH;
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t col = g / NHC;
  const int t = (int)(g - col * NHC);
  if (col >= ncols) return;
  if (!(flags_c[col * NHC + t] & kOwned)) return;
  const int a = t % N1C, b = DIM == 3 ? t / N1C : 0;
  double sH = 0.0, sh = 0.0;
  for (int j = 0; j < (DIM == 3 ? N1F : 1); ++j) {
    const double wj = DIM == 3 ? c_IS64[PF][b * N1F + j] : 1.0;
    for (int i = 0; i < N1F; ++i) {
      const double w = wj * c_IS64[PF][a * N1F + i];
      const int n = nodes_f[col * NHF + j * N1F + i];
      sH += w * Hf[n];
      sh += w * hf[n];
    }
  }
  const int n = nodes_c[col * NHC + t];
  Hc[n] = sH;
  hc[n] = sh;
}

// Restriction b_c = P^T (r_f - q_f) (q_f = NULL: P^T r_f).  One thread per (column, fine
// horizontal node) loads its fine line (owner columns only; the shared layer level counts in the
// upper layer) and contracts it vertically in registers; the horizontal contraction is split in
// two LDS stages over all threads of the column: (a, j, c) sums over i, then (a, b, c) over j.
// Coarse nodes owned by the column go to b_c, the others to the coarse face slots (summed by the
// coarse level's face pass); the coarse surface level is set to zero.  The vertical carry of the
// shared layer level passes through a double-buffered LDS slot per coarse horizontal node.
// waves per SIMD the restriction is compiled for: six for the FP64 p = 6 -> 3 transfer (at most 80
// VGPRs; the compiler's own choice lands just above and leaves five), else the compiler's choice
template <int PF, typename T>
struct RestrictWaves {
  static constexpr int v = (PF == 6 && sizeof(T) == 8) ? 6 : 1;
};

template <int PF, int DIM, typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RestrictWaves<PF, T>::v))) void k_restrict(const T *__restrict__ rf, const T *__restrict__ qf,
                                                  T *__restrict__ bc, T *__restrict__ Fc,
                                                  const int32_t *__restrict__ nodes_f,
                                                  const uint8_t *__restrict__ flags_f,
                                                  const int32_t *__restrict__ nodes_c,
                                                  const uint8_t *__restrict__ flags_c,
                                                  const int32_t *__restrict__ slot_c, int ncols, int nz,
                                                  int64_t ns_f, int64_t ns_c, int64_t nslots_c,
                                                  const int32_t *__restrict__ skip) {
  using LF = Lay<PF, DIM>;
  constexpr int PC = PF / 2, N1F = PF + 1, N1C = PC + 1;
  constexpr int NHF = LF::NH, CPB = LF::CPB, NHC = Lay<PC, DIM>::NH;
  constexpr int NJ = DIM == 3 ? N1F : 1;               // fine rows left after stage A
  constexpr int NA = N1C * NJ * N1C;                   // stage A items (a, j, c)
  constexpr int NB = NHC * N1C;                        // stage B items (a, b, c)
  __shared__ T sW[CPB * N1C * NHF];
  __shared__ T sA[CPB * NA];
  __shared__ T sC[CPB * 2 * NHC];
  if (skip != nullptr && *skip) return;
  const int lc = threadIdx.x / NHF;
  const int t = threadIdx.x - lc * NHF;
  const int ci = blockIdx.x * CPB + lc;
  const bool active = ci < ncols;
  const int col = active ? ci : 0;
  const int hn = active ? nodes_f[col * NHF + t] : 0;
  const bool own = active && (flags_f[col * NHF + t] & kOwned);
  T *W = sW + lc * N1C * NHF;
  T *A = sA + lc * NA;
  T *Cr = sC + lc * 2 * NHC;
  const int vtop = PC * nz;
  // stage B items of this thread (it = t + m NHF, the same coarse horizontal node in every layer),
  // loaded once: the coarse node where the column owns it, else -1 - its face slot
  constexpr int MI = (NB + NHF - 1) / NHF;
  int dst[MI];
#pragma unroll
  for (int m = 0; m < MI; ++m) {
    const int it = t + m * NHF;
    const int h = it % NHC;
    dst[m] = 0;
    if (active && it < NB)
      dst[m] = (flags_c[col * NHC + h] & kOwned) ? nodes_c[col * NHC + h] : -1 - slot_c[col * NHC + h];
  }
  // the fine line of layer l + 1 is loaded while layer l is contracted (raw values of both
  // operands, so that nothing waits for them before their use)
  T nr[N1F], nq[N1F];
  auto load_layer = [&](int l) {
    const int kmax = (l == nz - 1) ? N1F : PF;
#pragma unroll
    for (int k = 0; k < N1F; ++k) {
      const int64_t idx = (int64_t)(l * PF + k) * ns_f + hn;
      const bool ld = own && k < kmax;
      nr[k] = ld ? rf[idx] : T(0);
      nq[k] = (ld && qf) ? qf[idx] : T(0);
    }
  };
  load_layer(0);
  for (int l = 0; l < nz; ++l) {
    T rv[N1F];
#pragma unroll
    for (int k = 0; k < N1F; ++k) rv[k] = nr[k] - nq[k];
    if (l + 1 < nz) load_layer(l + 1);
    T w[N1C];
#pragma unroll
    for (int c = 0; c < N1C; ++c) w[c] = T(0);
    if (own) {
#pragma unroll
      for (int k = 0; k < N1F; ++k)
#pragma unroll
        for (int c = 0; c < N1C; ++c) w[c] += ip<T>(PF, k * N1C + c) * rv[k];
    }
#pragma unroll
    for (int c = 0; c < N1C; ++c) W[c * NHF + t] = w[c];
    __syncthreads();
    if constexpr (DIM == 3) {
      // stage A: A[(c NJ + j) N1C + a] = sum_i IP[i][a] W[c][j][i]
      for (int it = t; it < NA; it += NHF) {
        const int a = it % N1C, j = (it / N1C) % NJ, c = it / (N1C * NJ);
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < N1F; ++i) acc += ip<T>(PF, i * N1C + a) * W[c * NHF + j * N1F + i];
        A[it] = acc;
      }
      __syncthreads();
    }
    // stage B: coarse value (a, b, c) of this layer's element, assembled
#pragma unroll 1
    for (int m = 0; m < MI; ++m) {
      const int it = t + m * NHF;
      if (!active || it >= NB) continue;
      const int h = it % NHC, c = it / NHC;            // h = b N1C + a
      const int a = h % N1C, b = h / N1C;
      T acc = T(0);
      if constexpr (DIM == 3) {
#pragma unroll
        for (int j = 0; j < N1F; ++j) acc += ip<T>(PF, j * N1C + b) * A[(c * NJ + j) * N1C + a];
      } else {
#pragma unroll
        for (int i = 0; i < N1F; ++i) acc += ip<T>(PF, i * N1C + a) * W[c * NHF + i];
      }
      if (c == 0 && l > 0) acc += Cr[((l - 1) & 1) * NHC + h];
      if (c == PC && l < nz - 1) {
        Cr[(l & 1) * NHC + h] = acc;                   // the shared layer level, finished above
        continue;
      }
      const int v = l * PC + c;
      int d = dst[0];   // dst[m] by selects (constant indices keep dst in registers)
#pragma unroll
      for (int q = 1; q < MI; ++q)
        if (m == q) d = dst[q];
      if (d >= 0)
        bc[(int64_t)v * ns_c + d] = (v == vtop) ? T(0) : acc;
      else if (v != vtop)
        Fc[(int64_t)v * nslots_c + (-1 - d)] = acc;
    }
    __syncthreads();
  }
}

// Prolongation x_f += P x_c, written by the owner column of each fine node.
template <int PF, int DIM, typename T>
__global__ __launch_bounds__(256) void k_prolong_add(const T *__restrict__ xc, T *__restrict__ xf,
                                                     const int32_t *__restrict__ nodes_f,
                                                     const uint8_t *__restrict__ flags_f,
                                                     const int32_t *__restrict__ nodes_c, int ncols, int nz,
                                                     int64_t ns_f, int64_t ns_c, const int32_t *__restrict__ skip) {
  using LF = Lay<PF, DIM>;
  constexpr int PC = PF / 2, N1F = PF + 1, N1C = PC + 1;
  constexpr int NHF = LF::NH, CPB = LF::CPB, NHC = Lay<PC, DIM>::NH;
  __shared__ T sX[CPB * N1C * NHC];
  if (skip != nullptr && *skip) return;
  const int lc = threadIdx.x / NHF;
  const int t = threadIdx.x - lc * NHF;
  const int ci = blockIdx.x * CPB + lc;
  const bool active = ci < ncols;
  const int col = active ? ci : 0;
  const int hn = active ? nodes_f[col * NHF + t] : 0;
  const bool own = active && (flags_f[col * NHF + t] & kOwned);
  const bool cthr = active && t < NHC;
  const int hnc = cthr ? nodes_c[col * NHC + t] : 0;
  const int i = t % N1F, j = DIM == 3 ? t / N1F : 0;
  T *X = sX + lc * N1C * NHC;
  // the coarse values of layer l + 1 and the fine values of layer l are loaded before they are
  // needed, so the loads overlap the barrier and the contractions
  T xn[N1C];
  auto load_coarse = [&](int l) {
#pragma unroll
    for (int c = 0; c < N1C; ++c) xn[c] = cthr ? xc[(int64_t)(l * PC + c) * ns_c + hnc] : T(0);
  };
  load_coarse(0);
  for (int l = 0; l < nz; ++l) {
    const int kend = (l == nz - 1) ? N1F : PF;
    T old[N1F];
#pragma unroll
    for (int k = 0; k < N1F; ++k) old[k] = (own && k < kend) ? xf[(int64_t)(l * PF + k) * ns_f + hn] : T(0);
    if (cthr) {
#pragma unroll
      for (int c = 0; c < N1C; ++c) X[c * NHC + t] = xn[c];
    }
    if (l + 1 < nz) load_coarse(l + 1);
    __syncthreads();
    if (own) {
      T w[N1C];
#pragma unroll
      for (int c = 0; c < N1C; ++c) {
        T acc = T(0);
#pragma unroll
        for (int b = 0; b < (DIM == 3 ? N1C : 1); ++b) {
          T inner = T(0);
#pragma unroll
          for (int a = 0; a < N1C; ++a) inner += ip<T>(PF, i * N1C + a) * X[c * NHC + b * N1C + a];
          acc += (DIM == 3 ? ip<T>(PF, j * N1C + b) : T(1)) * inner;
        }
        w[c] = acc;
      }
#pragma unroll
      for (int k = 0; k < N1F; ++k) {
        if (k < kend) {
          T u = T(0);
#pragma unroll
          for (int c = 0; c < N1C; ++c) u += ip<T>(PF, k * N1C + c) * w[c];
          xf[(int64_t)(l * PF + k) * ns_f + hn] = old[k] + u;
        }
      }
    }
    __syncthreads();
  }
}

// ---- vector kernels (grid-stride, fixed grid, deterministic partials) -----------------------

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int NS>
__device__ __forceinline__ void block_partials(double (&v)[NS], double *partial) {
  constexpr int NW = kVecThreads / 64;
  __shared__ double s[NS][NW];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    double r = wsum(v[k]);
    if (lane == 0) s[k][wv] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      double a = 0.0;
      for (int w = 0; w < NW; ++w) a += s[k][w];
      partial[blockIdx.x * NS + k] = a;
    }
  }
}

template <int NS>
__device__ __forceinline__ void final_sums(const double *partial, int np, double (&out)[NS]) {
  __shared__ double s[NS][kVecThreads];
  double a[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) a[k] = 0.0;
  for (int b = threadIdx.x; b < np; b += kVecThreads)
#pragma unroll
    for (int k = 0; k < NS; ++k) a[k] += partial[b * NS + k];
#pragma unroll
  for (int k = 0; k < NS; ++k) s[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int w = kVecThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < NS; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) out[k] = s[k][0];
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// first Chebyshev step from x = 0: r = b, d = c dinv b, x = d
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_cheb0(const T *b, T *r, T *d, T *x, const T *dinv,
                                                       const double *cf, int64_t n, const int32_t *skip) {
  if (skip != nullptr && *skip) return;
  const T c = (T)cf[0];
  GRID_STRIDE(i, n) {
    const T bi = b[i];
    const T di = c * dinv[i] * bi;
    r[i] = bi;
    d[i] = di;
    x[i] = di;
  }
}

// first Chebyshev step from x: r = b - q (q = A x), d = c dinv r, x += d
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_cheb1(const T *b, const T *q, T *r, T *d, T *x, const T *dinv,
                                                       const double *cf, int64_t n, const int32_t *skip) {
  if (skip != nullptr && *skip) return;
  const T c = (T)cf[0];
  GRID_STRIDE(i, n) {
    const T ri = b[i] - q[i];
    const T di = c * dinv[i] * ri;
    r[i] = ri;
    d[i] = di;
    x[i] += di;
  }
}

// later steps: r -= q (q = A d), d = c1 d + c2 dinv r, x += d
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_cheb_step(T *r, const T *q, T *d, T *x, const T *dinv,
                                                           const double *cf, int k, int64_t n,
                                                           const int32_t *skip) {
  if (skip != nullptr && *skip) return;
  const T c1 = (T)cf[3 + 2 * (k - 2)], c2 = (T)cf[4 + 2 * (k - 2)];
  GRID_STRIDE(i, n) {
    const T ri = r[i] - q[i];
    const T di = c1 * d[i] + c2 * dinv[i] * ri;
    r[i] = ri;
    d[i] = di;
    x[i] += di;
  }
}

// Two-step smoothing written out (the default degree): with d1 = c0 D^-1 r0 and
// d2 = c1 d1 + c2 D^-1 (r0 - A d1), x2 = x0 + a1 d1 + a2 D^-1 (r0 - A d1) (a1 = 1 + c1, a2 = c2)
// = x0 + D^-1 ((a1 c0 + a2) r0 - a2 A d1): d1 is needed only as the input of its product, and
// no residual or step vector survives it.
//   y = c dinv b
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_scale(T *y, const T *b, const T *dinv, const double *cf, int64_t n,
                                                       const int32_t *skip) {
  if (skip != nullptr && *skip) return;
  const T c = (T)cf[0];
  GRID_STRIDE(i, n) y[i] = c * dinv[i] * b[i];
}

//   from zero: x = dinv ((a1 c0 + a2) b - a2 q), q = A d1
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_pre2(T *x, const T *b, const T *q, const T *dinv,
                                                      const double *cf, int64_t n, const int32_t *skip) {
  if (skip != nullptr && *skip) return;
  const T e = (T)(cf[1] * cf[0] + cf[2]), a2 = (T)cf[2];
  GRID_STRIDE(i, n) x[i] = dinv[i] * (e * b[i] - a2 * q[i]);
}

//   from x: d1 = c dinv (b - q1), q1 = A x
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_post2a(T *d, const T *b, const T *q1, const T *dinv,
                                                        const double *cf, int64_t n, const int32_t *skip) {
  if (skip != nullptr && *skip) return;
  const T c = (T)cf[0];
  GRID_STRIDE(i, n) d[i] = c * dinv[i] * (b[i] - q1[i]);
}

//   x += dinv ((a1 c0 + a2) (b - q1) - a2 q2), q1 = A x, q2 = A d1
// DOT: also the block partials of b.x (the CG's r.z when b is the residual and x the V-cycle's
// result), in the order k_dot takes them, so the sum is the same bit for bit
template <typename T, bool DOT>
__global__ __launch_bounds__(kVecThreads) void k_post2b(T *x, const T *b, const T *q1, const T *q2,
                                                        const T *dinv, const double *cf, int64_t n,
                                                        const int32_t *skip, double *partial) {
  if (skip != nullptr && *skip) return;
  const T e = (T)(cf[1] * cf[0] + cf[2]), a2 = (T)cf[2];
  double v[1] = {0.0};
  GRID_STRIDE(i, n) {
    const T xi = x[i] + dinv[i] * (e * (b[i] - q1[i]) - a2 * q2[i]);
    x[i] = xi;
    if constexpr (DOT) v[0] += (double)b[i] * (double)xi;
  }
  if constexpr (DOT) block_partials<1>(v, partial);
}

// PCG with a general preconditioner: x += alpha p, r -= alpha q; partial r.r.  SCALE: also the
// first step of the degree-2 V-cycle that follows on the new residual, d = c0 dinv r.
template <typename T, bool SCALE>
__global__ __launch_bounds__(kVecThreads) void k_mg_update(T *x, T *r, const T *p, const T *q, int64_t n,
                                                           double *partial, const PcgScalars *sc, T *d,
                                                           const T *dinv, const double *cf) {
  if (sc->done) return;
  const T a = (T)sc->alpha;
  const T c0 = SCALE ? (T)cf[0] : T(0);
  double v[1] = {0.0};
  GRID_STRIDE(i, n) {
    x[i] += a * p[i];
    const T ri = r[i] - a * q[i];
    r[i] = ri;
    if constexpr (SCALE) d[i] = c0 * dinv[i] * ri;
    v[0] += (double)ri * (double)ri;
  }
  block_partials<1>(v, partial);
}

__global__ __launch_bounds__(kVecThreads) void k_mg_fin_rr(const double *partial, int np, PcgScalars *sc) {
  if (sc->done) return;
  double s[1];
  final_sums<1>(partial, np, s);
  if (threadIdx.x == 0) {
    sc->rr = s[0];
    sc->iters += 1;
    if (!(s[0] == s[0]) || !(s[0] <= 1e300)) {
      sc->breakdown = 2;
      sc->done = 1;
    } else if (s[0] <= sc->tol2) {
      sc->done = 1;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_dot(const T *a, const T *b, int64_t n, double *partial,
                                                     const PcgScalars *sc) {
  if (sc->done) return;
  double v[1] = {0.0};
  GRID_STRIDE(i, n) v[0] += (double)a[i] * (double)b[i];
  block_partials<1>(v, partial);
}

// beta = (r.z)_new / (r.z)_old (first: beta = 0); a non-positive r.z means the preconditioner
// is not positive definite on this residual
__global__ __launch_bounds__(kVecThreads) void k_mg_fin_rz(const double *partial, int np, PcgScalars *sc,
                                                           int first) {
  if (sc->done) return;
  double s[1];
  final_sums<1>(partial, np, s);
  if (threadIdx.x == 0) {
    sc->beta = first ? 0.0 : s[0] / sc->rz;
    sc->rz = s[0];
    if (!(s[0] > 0.0) || !(s[0] <= 1e300)) {
      sc->breakdown = (s[0] == s[0]) ? 1 : 2;
      sc->done = 1;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_mg_dir(T *p, const T *z, int64_t n, const PcgScalars *sc,
                                                        int first) {
  if (sc->done) return;
  const T b = (T)sc->beta;
  GRID_STRIDE(i, n) p[i] = first ? z[i] : z[i] + b * p[i];
}

// Largest eigenvalue of D^-1 A.  D^-1 A is self-adjoint in <u, v>_D = sum u_i v_i / dinv_i over
// the unknowns (dinv = 0 on the Dirichlet rows, which take no part), so Lanczos in that inner
// product gives a symmetric tridiagonal matrix whose largest eigenvalue approaches lambda_max
// from below.  The top of this spectrum is clustered (element-local modes), where Lanczos needs
// far fewer products than the power iteration's Rayleigh quotient.

// v = fixed start vector on the unknowns, vp = 0; partials of <v, v>_D
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_lz_start(T *v, T *vp, const T *dinv, int64_t n, double *partial) {
  double s[1] = {0.0};
  GRID_STRIDE(i, n) {
    const T d = dinv[i];
    const T vi = d != T(0) ? T(1.0 + 0.5 * sin(0.7 * (double)i) + 0.25 * cos(0.013 * (double)i)) : T(0);
    v[i] = vi;
    vp[i] = T(0);
    if (d != T(0)) s[0] += (double)vi * (double)vi / (double)d;
  }
  block_partials<1>(s, partial);
}

// out = sum (mode 0) or its square root (mode 1), set to 0 when it is below rel^2 * ref^2
// (an invariant subspace: the recurrence then produces zeros, which add zero Ritz values only)
__global__ __launch_bounds__(kVecThreads) void k_lz_fin(const double *partial, int np, double *out, int mode,
                                                        const double *ref, double rel) {
  double s[1];
  final_sums<1>(partial, np, s);
  if (threadIdx.x == 0) {
    double v = s[0];
    if (mode == 1) {
      const double r = ref != nullptr ? fabs(*ref) : 0.0;
      v = (v > 0.0 && v > rel * rel * r * r) ? sqrt(v) : 0.0;
    }
    *out = v;
  }
}

// w = dinv q - alpha v - beta_prev vp, stored in vp; partials of <w, w>_D
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_lz_w(T *vp, const T *v, const T *q, const T *dinv, int64_t n,
                                                      const double *alpha, const double *beta_prev,
                                                      double *partial) {
  const T a = (T)*alpha, b = beta_prev != nullptr ? (T)*beta_prev : T(0);
  double s[1] = {0.0};
  GRID_STRIDE(i, n) {
    const T d = dinv[i];
    const T w = d * q[i] - a * v[i] - b * vp[i];
    vp[i] = w;
    if (d != T(0)) s[0] += (double)w * (double)w / (double)d;
  }
  block_partials<1>(s, partial);
}

// partials of a.b
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_lz_dot(const T *a, const T *b, int64_t n, double *partial) {
  double s[1] = {0.0};
  GRID_STRIDE(i, n) s[0] += (double)a[i] * (double)b[i];
  block_partials<1>(s, partial);
}

// v /= beta (0 when beta is 0)
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_lz_scale(T *v, int64_t n, const double *beta) {
  const T f = *beta > 0.0 ? (T)(1.0 / *beta) : T(0);
  GRID_STRIDE(i, n) v[i] *= f;
}

// u = y_j v (first) or u += y_j v
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_lz_acc(T *u, const T *v, int64_t n, double y, int first) {
  const T c = (T)y;
  GRID_STRIDE(i, n) u[i] = first ? c * v[i] : u[i] + c * v[i];
}

// power iteration on D^-1 A: pw[0] = (v.Av)/(v.Dv) (Rayleigh quotient), pw[1] = 1/sqrt(v.Dv)

template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_pow_dots(const T *v, const T *q, const T *dinv, int64_t n,
                                                          double *partial) {
  double s[2] = {0.0, 0.0};
  GRID_STRIDE(i, n) {
    const double vi = (double)v[i];
    s[0] += vi * (double)q[i];
    if (dinv[i] != T(0)) s[1] += vi * vi / (double)dinv[i];
  }
  block_partials<2>(s, partial);
}

__global__ __launch_bounds__(kVecThreads) void k_pow_fin(const double *partial, int np, double *pw) {
  double s[2];
  final_sums<2>(partial, np, s);
  if (threadIdx.x == 0) {
    pw[0] = s[1] > 0.0 ? s[0] / s[1] : 0.0;
    pw[1] = s[1] > 0.0 ? 1.0 / sqrt(s[1]) : 1.0;
  }
}

template <typename T>
__global__ void k_pow_next(T *v, const T *q, const T *dinv, int64_t n, const double *pw) {
  const T sc = (T)pw[1];
  GRID_STRIDE(i, n) v[i] = dinv[i] * q[i] * sc;
}

// ---- host side --------------------------------------------------------------------------------

template <typename T>
struct Prec;
template <>
struct Prec<double> {
  static constexpr fnpf_dtype dt = FNPF_F64;
  static double *const *lv(MgLevel &L) { return L.v64; }
  static double *const *fv(Ctx &c) { return c.mg_f64; }
  static const double *dinv(Ctx &c) { return c.d_dinv; }
  static bool &stale(Ctx &c) { return c.mg_stale64; }
  static double *&ev(MgLevel &L) { return L.ev64; }
  static double *&evf(Ctx &c) { return c.mg_ev64; }
  static bool &evok(MgLevel &L) { return L.ev_ok64; }
  static bool &evokf(Ctx &c) { return c.mg_ev_ok64; }
};
template <>
struct Prec<float> {
  static constexpr fnpf_dtype dt = FNPF_F32;
  static float *const *lv(MgLevel &L) { return L.v32; }
  static float *const *fv(Ctx &c) { return c.mg_f32; }
  static const float *dinv(Ctx &c) { return c.d_dinv32; }
  static bool &stale(Ctx &c) { return c.mg_stale32; }
  static float *&ev(MgLevel &L) { return L.ev32; }
  static float *&evf(Ctx &c) { return c.mg_ev32; }
  static bool &evok(MgLevel &L) { return L.ev_ok32; }
  static bool &evokf(Ctx &c) { return c.mg_ev_ok32; }
};

template <typename T>
hipError_t dalloc_t(T **p, size_t n) {
  return hipMalloc((void **)p, n * sizeof(T));
}

#define MG_DISPATCH(DIMV, PV, CALL)                    \
  switch (PV) {                                        \
    case 2: { constexpr int PF_ = 2; CALL; } break;    \
    case 3: { constexpr int PF_ = 3; CALL; } break;    \
    case 4: { constexpr int PF_ = 4; CALL; } break;    \
    case 5: { constexpr int PF_ = 5; CALL; } break;    \
    case 6: { constexpr int PF_ = 6; CALL; } break;    \
    case 7: { constexpr int PF_ = 7; CALL; } break;    \
    case 8: { constexpr int PF_ = 8; CALL; } break;    \
    default: return hipErrorInvalidValue;              \
  }

template <int PF, int DIM, typename T>
hipError_t restrict_impl(Ctx &F, Ctx &C, const T *rf, const T *qf, T *bc, T *Fc, const int32_t *skip,
                         hipStream_t s) {
  using LF = Lay<PF, DIM>;
  const int nb = (F.n_eh + LF::CPB - 1) / LF::CPB;
  k_restrict<PF, DIM, T><<<nb, LF::NT, 0, s>>>(rf, qf, bc, Fc, F.d_eh_nodes, F.d_flags, C.d_eh_nodes, C.d_flags,
                                               C.d_slot, F.n_eh, F.nz, F.n_s, C.n_s, C.n_slots, skip);
  return hipGetLastError();
}

template <int PF, int DIM, typename T>
hipError_t prolong_impl(Ctx &F, Ctx &C, const T *xc, T *xf, const int32_t *skip, hipStream_t s) {
  using LF = Lay<PF, DIM>;
  const int nb = (F.n_eh + LF::CPB - 1) / LF::CPB;
  k_prolong_add<PF, DIM, T><<<nb, LF::NT, 0, s>>>(xc, xf, F.d_eh_nodes, F.d_flags, C.d_eh_nodes, F.n_eh, F.nz,
                                                  F.n_s, C.n_s, skip);
  return hipGetLastError();
}

template <int PF, int DIM>
hipError_t surf_impl(Ctx &F, Ctx &C, double *Hc, double *hc, hipStream_t s) {
  constexpr int NHC = Lay<PF / 2, DIM>::NH;
  const int64_t nthr = (int64_t)F.n_eh * NHC;
  k_mg_surf<PF, DIM><<<(unsigned)((nthr + 255) / 256), 256, 0, s>>>(F.d_geoH, F.d_geoh, F.d_eh_nodes, C.d_eh_nodes,
                                                                     C.d_flags, F.n_eh, Hc, hc);
  return hipGetLastError();
}

template <typename T>
hipError_t restrict_to(Ctx &F, Ctx &C, const T *rf, const T *qf, T *bc, const int32_t *skip, hipStream_t s) {
  T *Fc = nullptr;
  if constexpr (sizeof(T) == 8) Fc = (T *)C.d_F64; else Fc = (T *)C.d_F32;
  if (F.dim == 3) {
    MG_DISPATCH(3, F.p, { hipError_t e = (restrict_impl<PF_, 3, T>(F, C, rf, qf, bc, Fc, skip, s)); if (e != hipSuccess) return e; });
  } else {
    MG_DISPATCH(2, F.p, { hipError_t e = (restrict_impl<PF_, 2, T>(F, C, rf, qf, bc, Fc, skip, s)); if (e != hipSuccess) return e; });
  }
  return launch_faces(C, Prec<T>::dt, bc, true, s, skip);
}

template <typename T>
hipError_t prolong_to(Ctx &F, Ctx &C, const T *xc, T *xf, const int32_t *skip, hipStream_t s) {
  if (F.dim == 3) {
    MG_DISPATCH(3, F.p, return (prolong_impl<PF_, 3, T>(F, C, xc, xf, skip, s)));
  } else {
    MG_DISPATCH(2, F.p, return (prolong_impl<PF_, 2, T>(F, C, xc, xf, skip, s)));
  }
  return hipSuccess;
}

hipError_t surf_to(Ctx &F, Ctx &C, double *Hc, double *hc, hipStream_t s) {
  if (F.dim == 3) {
    MG_DISPATCH(3, F.p, return (surf_impl<PF_, 3>(F, C, Hc, hc, s)));
  } else {
    MG_DISPATCH(2, F.p, return (surf_impl<PF_, 2>(F, C, Hc, hc, s)));
  }
  return hipSuccess;
}

// Device table of the Chebyshev coefficients, kMgCoef doubles per (precision, level): [0] 1/theta,
// [1] 1 + c1_2 and [2] c2_2 (closed-form degree 2), then (c1_k, c2_k) for steps k = 2 .. 10 of the
// three-term recurrence on [lmax / ratio, lmax], lmax = 1.1 lam.  Kernels read it from device
// memory, so captured iteration graphs stay valid when the estimates change.
template <typename T>
const double *coef_table(Ctx &c, int l) {
  return c.d_mgc + ((sizeof(T) == 8 ? 0 : 1) * (int)(c.mg.size() + 1) + l) * kMgCoef;
}

__host__ __device__ void chebyshev_coefficients(double lam, double ratio, double *cf) {
  const double lmax = kMgSafety * lam, lmin = lmax / ratio;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  for (int k = 0; k < kMgCoef; ++k) cf[k] = 0.0;
  cf[0] = 1.0 / theta;
  double rho0 = 1.0 / sigma;
  for (int k = 2; k <= kMgCoarseSteps; ++k) {
    const double rho1 = 1.0 / (2.0 * sigma - rho0);
    cf[3 + 2 * (k - 2)] = rho1 * rho0;
    cf[4 + 2 * (k - 2)] = 2.0 * rho1 / delta;
    if (k == 2) {
      cf[1] = 1.0 + rho1 * rho0;
      cf[2] = 2.0 * rho1 / delta;
    }
    rho0 = rho1;
  }
}

// The table of one level from its eigenvalue estimate *lam on the device, so that a geometry update
// needs no host round trip; lam_out keeps the estimate.  A non-positive or non-finite estimate
// gives a NaN table, which the solve then reports as a non-finite residual.
__global__ void k_cheb_coef(const double *lam, double ratio, double *cf, double *lam_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double l = *lam;
  *lam_out = l;
  if (l > 0.0 && l <= 1e300) {
    chebyshev_coefficients(l, ratio, cf);
  } else {
    for (int k = 0; k < kMgCoef; ++k) cf[k] = __builtin_nan("");
  }
}

__global__ void k_set_scalar(double *p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Chebyshev smoothing of A x = b on level L (D^-1 A spectrum estimate lam), m steps.  From zero:
// x = p(D^-1 A) D^-1 b; otherwise x += p(D^-1 A) D^-1 (b - A x).  On return r = b - A x_{m-1}
// and d = x_m - x_{m-1}.
// line: B^-1 (the level's vertical line blocks, line_smoother.hip) in place of D^-1.
template <typename T>
hipError_t smooth(Ctx &L, const T *b, T *x, T *r, T *d, T *q, const double *cf, int m, bool from_zero,
                  const int32_t *skip, hipStream_t s, bool line = false) {
  if (line) {
    hipError_t e = hipSuccess;
    if (from_zero) {
      e = line_cheb0<T>(L, b, r, d, x, cf, skip, s);
    } else {
      if ((e = launch_apply(L, Prec<T>::dt, x, q, true, nullptr, skip, s)) != hipSuccess) return e;
      e = line_cheb1<T>(L, b, q, r, d, x, cf, skip, s);
    }
    for (int k = 2; k <= m && e == hipSuccess; ++k) {
      if ((e = launch_apply(L, Prec<T>::dt, d, q, true, nullptr, skip, s)) != hipSuccess) return e;
      e = line_chebk<T>(L, q, r, d, x, cf, k, skip, s);
    }
    return e;
  }
  const T *dinv = Prec<T>::dinv(L);
  const int64_t n = L.n_v;
  if (from_zero) {
    k_cheb0<T><<<kVB<T>, kVecThreads, 0, s>>>(b, r, d, x, dinv, cf, n, skip);
  } else {
    hipError_t e = launch_apply(L, Prec<T>::dt, x, q, true, nullptr, skip, s);
    if (e != hipSuccess) return e;
    k_cheb1<T><<<kVB<T>, kVecThreads, 0, s>>>(b, q, r, d, x, dinv, cf, n, skip);
  }
  for (int k = 2; k <= m; ++k) {
    hipError_t e = launch_apply(L, Prec<T>::dt, d, q, true, nullptr, skip, s);
    if (e != hipSuccess) return e;
    k_cheb_step<T><<<kVB<T>, kVecThreads, 0, s>>>(r, q, d, x, dinv, cf, k, n, skip);
  }
  return hipGetLastError();
}

// V-cycle on level l (0 = this context) for the right-hand side b, result in x.
// pre_scaled (level 0, degree 2): d = c0 dinv b is already in place (k_mg_update<T, true>).
template <typename T>
hipError_t vcycle(Ctx &c, int l, const T *b, T *x, const int32_t *skip, int m, hipStream_t s,
                  double *dot_partial = nullptr, bool *dot_done = nullptr, bool pre_scaled = false) {
  Ctx &L = l == 0 ? c : *c.mg[l - 1].c;
  T *r, *d, *q;
  if (l == 0) {
    r = Prec<T>::fv(c)[1];
    d = Prec<T>::fv(c)[2];
    q = Prec<T>::fv(c)[3];
  } else {
    r = Prec<T>::lv(c.mg[l - 1])[2];
    d = Prec<T>::lv(c.mg[l - 1])[3];
    q = Prec<T>::lv(c.mg[l - 1])[4];
  }
  const double *cf = coef_table<T>(c, l);
  const int last = (int)c.mg.size();
  const bool line = c.mg_line;
  if (l == last) return smooth<T>(L, b, x, r, d, q, cf, kMgCoarseSteps, true, skip, s, line);
  MgLevel &C = c.mg[l];
  T *bc = Prec<T>::lv(C)[0], *xc = Prec<T>::lv(C)[1];
  const int64_t n = L.n_v;
  const T *dinv = Prec<T>::dinv(L);
  hipError_t e = hipSuccess;
  if (m == 2 && !line) {
    if (!(l == 0 && pre_scaled)) k_scale<T><<<kVB<T>, kVecThreads, 0, s>>>(d, b, dinv, cf, n, skip);
    if ((e = launch_apply(L, Prec<T>::dt, d, q, true, nullptr, skip, s)) != hipSuccess) return e;
    k_pre2<T><<<kVB<T>, kVecThreads, 0, s>>>(x, b, q, dinv, cf, n, skip);
    if ((e = launch_apply(L, Prec<T>::dt, x, q, true, nullptr, skip, s)) != hipSuccess) return e;
    if ((e = restrict_to<T>(L, *C.c, b, q, bc, skip, s)) != hipSuccess) return e;   // P^T (b - A x)
    if ((e = vcycle<T>(c, l + 1, bc, xc, skip, m, s)) != hipSuccess) return e;
    if ((e = prolong_to<T>(L, *C.c, xc, x, skip, s)) != hipSuccess) return e;
    if ((e = launch_apply(L, Prec<T>::dt, x, r, true, nullptr, skip, s)) != hipSuccess) return e;
    k_post2a<T><<<kVB<T>, kVecThreads, 0, s>>>(d, b, r, dinv, cf, n, skip);
    if ((e = launch_apply(L, Prec<T>::dt, d, q, true, nullptr, skip, s)) != hipSuccess) return e;
    if (dot_partial != nullptr) {
      k_post2b<T, true><<<kVB<T>, kVecThreads, 0, s>>>(x, b, r, q, dinv, cf, n, skip, dot_partial);
      if (dot_done) *dot_done = true;
    } else {
      k_post2b<T, false><<<kVB<T>, kVecThreads, 0, s>>>(x, b, r, q, dinv, cf, n, skip, nullptr);
    }
    return hipGetLastError();
  }
  e = smooth<T>(L, b, x, r, d, q, cf, m, true, skip, s, line);
  if (e != hipSuccess) return e;
  // residual of the smoothed x, r - A d, restricted directly
  e = launch_apply(L, Prec<T>::dt, d, q, true, nullptr, skip, s);
  if (e != hipSuccess) return e;
  e = restrict_to<T>(L, *C.c, r, q, bc, skip, s);
  if (e != hipSuccess) return e;
  e = vcycle<T>(c, l + 1, bc, xc, skip, m, s);
  if (e != hipSuccess) return e;
  e = prolong_to<T>(L, *C.c, xc, x, skip, s);
  if (e != hipSuccess) return e;
  return smooth<T>(L, b, x, r, d, q, cf, m, false, skip, s, line);
}

// Eigenvalues and eigenvectors of a small symmetric matrix a[n][n] (row-major, destroyed) by
// cyclic Jacobi rotations: w[k] and column k of z[n][n].
void symmetric_eigen(int n, std::vector<double> &a, std::vector<double> &w, std::vector<double> &z) {
  z.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) z[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double x = a[(size_t)i * n + j] * a[(size_t)i * n + j];
        tot += x;
        if (i != j) off += x;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (apq == 0.0) continue;
        const double theta = (a[(size_t)q * n + q] - a[(size_t)p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
          a[(size_t)k * n + p] = c * akp - sn * akq;
          a[(size_t)k * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
          a[(size_t)p * n + k] = c * apk - sn * aqk;
          a[(size_t)q * n + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double zkp = z[(size_t)k * n + p], zkq = z[(size_t)k * n + q];
          z[(size_t)k * n + p] = c * zkp - sn * zkq;
          z[(size_t)k * n + q] = sn * zkp + c * zkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
}

// kLanczosSteps Lanczos steps on D^-1 A of level L from the fixed start vector (vectors v, vp, q);
// the largest Ritz value is the estimate, and a second pass over the same recurrence (its
// coefficients kept from the first) forms the Ritz vector in u for the later warm updates.
template <typename T>
hipError_t lanczos_lambda(Ctx &c, Ctx &L, T *u, T *v, T *vp, T *q, double &lam, hipStream_t s) {
  const T *dinv = Prec<T>::dinv(L);
  const int64_t n = L.n_v;
  constexpr int K = kLanczosSteps;
  double *al = c.d_mg_lz, *be = c.d_mg_lz + K, *nrm = c.d_mg_lz + 2 * K;
  const double rel = 1e-12;
  std::vector<double> y(K, 0.0);
  for (int pass = 0; pass < 2; ++pass) {
    T *a = v, *b = vp;
    k_lz_start<T><<<kVB<T>, kVecThreads, 0, s>>>(a, b, dinv, n, c.d_partial);
    k_lz_fin<<<1, kVecThreads, 0, s>>>(c.d_partial, kVB<T>, nrm, 1, nullptr, 0.0);
    k_lz_scale<T><<<kVB<T>, kVecThreads, 0, s>>>(a, n, nrm);
    for (int j = 0; j < K; ++j) {
      if (pass == 1) k_lz_acc<T><<<kVB<T>, kVecThreads, 0, s>>>(u, a, n, y[j], j == 0);
      if (pass == 1 && j == K - 1) break;
      hipError_t e = launch_apply(L, Prec<T>::dt, a, q, true, nullptr, nullptr, s);
      if (e != hipSuccess) return e;
      if (pass == 0) {
        k_lz_dot<T><<<kVB<T>, kVecThreads, 0, s>>>(a, q, n, c.d_partial);
        k_lz_fin<<<1, kVecThreads, 0, s>>>(c.d_partial, kVB<T>, al + j, 0, nullptr, 0.0);
      }
      k_lz_w<T><<<kVB<T>, kVecThreads, 0, s>>>(b, a, q, dinv, n, al + j, j > 0 ? be + j - 1 : nullptr,
                                                   c.d_partial);
      if (pass == 0) k_lz_fin<<<1, kVecThreads, 0, s>>>(c.d_partial, kVB<T>, be + j, 1, al + j, rel);
      k_lz_scale<T><<<kVB<T>, kVecThreads, 0, s>>>(b, n, be + j);
      std::swap(a, b);
    }
    if (pass == 0) {
      std::vector<double> h(2 * K);
      hipError_t e = hipMemcpyAsync(h.data(), c.d_mg_lz, sizeof(double) * 2 * K, hipMemcpyDeviceToHost, s);
      if (e != hipSuccess) return e;
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
      std::vector<double> t((size_t)K * K, 0.0), w, z;
      for (int j = 0; j < K; ++j) {
        t[(size_t)j * K + j] = h[j];
        if (j + 1 < K) t[(size_t)j * K + j + 1] = t[(size_t)(j + 1) * K + j] = h[K + j];
      }
      symmetric_eigen(K, t, w, z);
      int top = 0;
      for (int k = 1; k < K; ++k)
        if (w[k] > w[top]) top = k;
      lam = w[top];
      for (int j = 0; j < K; ++j) y[j] = z[(size_t)j * K + top];
    }
  }
  return hipGetLastError();
}

// The same Lanczos recurrence for B^-1 A (B: the level's vertical line blocks), self-adjoint in
// <u, v>_B = u^T B v = (L^T u).(L^T v): w = B^-1 q - alpha v - beta vp (one line solve), its B-norm
// from the factor, alpha = v.A v as before.
template <typename T>
hipError_t lanczos_lambda_line(Ctx &c, Ctx &L, T *u, T *v, T *vp, T *q, double &lam, hipStream_t s) {
  const T *dinv = Prec<T>::dinv(L);   // only places the start vector on the unknowns
  const int64_t n = L.n_v;
  constexpr int K = kLanczosSteps;
  double *al = c.d_mg_lz, *be = c.d_mg_lz + K, *nrm = c.d_mg_lz + 2 * K;
  const double rel = 1e-12;
  std::vector<double> y(K, 0.0);
  hipError_t e = hipSuccess;
  for (int pass = 0; pass < 2; ++pass) {
    T *a = v, *b = vp;
    k_lz_start<T><<<kVB<T>, kVecThreads, 0, s>>>(a, b, dinv, n, c.d_partial);
    if ((e = line_bnorm_partials<T>(L, a, c.d_partial, kVB<T>, s)) != hipSuccess) return e;
    k_lz_fin<<<1, kVecThreads, 0, s>>>(c.d_partial, kVB<T>, nrm, 1, nullptr, 0.0);
    k_lz_scale<T><<<kVB<T>, kVecThreads, 0, s>>>(a, n, nrm);
    for (int j = 0; j < K; ++j) {
      if (pass == 1) k_lz_acc<T><<<kVB<T>, kVecThreads, 0, s>>>(u, a, n, y[j], j == 0);
      if (pass == 1 && j == K - 1) break;
      if ((e = launch_apply(L, Prec<T>::dt, a, q, true, nullptr, nullptr, s)) != hipSuccess) return e;
      if (pass == 0) {
        k_lz_dot<T><<<kVB<T>, kVecThreads, 0, s>>>(a, q, n, c.d_partial);
        k_lz_fin<<<1, kVecThreads, 0, s>>>(c.d_partial, kVB<T>, al + j, 0, nullptr, 0.0);
      }
      if ((e = line_lanczos_w<T>(L, q, a, b, al + j, j > 0 ? be + j - 1 : nullptr, s)) != hipSuccess) return e;
      if (pass == 0) {
        if ((e = line_bnorm_partials<T>(L, b, c.d_partial, kVB<T>, s)) != hipSuccess) return e;
        k_lz_fin<<<1, kVecThreads, 0, s>>>(c.d_partial, kVB<T>, be + j, 1, al + j, rel);
      }
      k_lz_scale<T><<<kVB<T>, kVecThreads, 0, s>>>(b, n, be + j);
      std::swap(a, b);
    }
    if (pass == 0) {
      std::vector<double> h(2 * K);
      if ((e = hipMemcpyAsync(h.data(), c.d_mg_lz, sizeof(double) * 2 * K, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return e;
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
      std::vector<double> t((size_t)K * K, 0.0), w, z;
      for (int j = 0; j < K; ++j) {
        t[(size_t)j * K + j] = h[j];
        if (j + 1 < K) t[(size_t)j * K + j + 1] = t[(size_t)(j + 1) * K + j] = h[K + j];
      }
      symmetric_eigen(K, t, w, z);
      int top = 0;
      for (int k = 1; k < K; ++k)
        if (w[k] > w[top]) top = k;
      lam = w[top];
      for (int j = 0; j < K; ++j) y[j] = z[(size_t)j * K + top];
    }
  }
  return hipGetLastError();
}

// power-iteration scalars of B^-1 A: pw[0] = (v.Av)/(v.Bv), pw[1] = sqrt(v.Bv) (pw[2], pw[3]: the sums)
__global__ void k_line_pow_fin(double *pw) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double vbv = pw[3];
  pw[0] = vbv > 0.0 ? pw[2] / vbv : 0.0;
  pw[1] = vbv > 0.0 ? sqrt(vbv) : 1.0;
}

// Largest eigenvalue of D^-1 A on level L, left in *pw on the device: Lanczos the first time
// (Ritz vector into v), then Rayleigh-quotient power iterations from the previous eigenvector
// estimate v after each geometry update (no host synchronisation).  w1, w2, q are work vectors.
// With the line smoother (c.mg_line) the same for B^-1 A.
template <typename T>
hipError_t estimate_lambda(Ctx &c, Ctx &L, T *v, T *q, T *w1, T *w2, bool warm, double *pw, hipStream_t s) {
  if (!warm) {
    double lam = 0.0;
    hipError_t e = c.mg_line ? lanczos_lambda_line<T>(c, L, v, w1, w2, q, lam, s)
                             : lanczos_lambda<T>(c, L, v, w1, w2, q, lam, s);
    if (e != hipSuccess) return e;
    k_set_scalar<<<1, 1, 0, s>>>(pw, lam);
    return hipGetLastError();
  }
  const T *dinv = Prec<T>::dinv(L);
  const int64_t n = L.n_v;
  if (c.mg_line) {
    for (int it = 0; it < kPowNext; ++it) {
      hipError_t e = launch_apply(L, Prec<T>::dt, v, q, true, nullptr, nullptr, s);
      if (e != hipSuccess) return e;
      k_lz_dot<T><<<kVB<T>, kVecThreads, 0, s>>>(v, q, n, c.d_partial);
      k_lz_fin<<<1, kVecThreads, 0, s>>>(c.d_partial, kVB<T>, pw + 2, 0, nullptr, 0.0);
      if ((e = line_bnorm_partials<T>(L, v, c.d_partial, kVB<T>, s)) != hipSuccess) return e;
      k_lz_fin<<<1, kVecThreads, 0, s>>>(c.d_partial, kVB<T>, pw + 3, 0, nullptr, 0.0);
      k_line_pow_fin<<<1, 1, 0, s>>>(pw);
      if ((e = line_apply<T>(L, q, v, s)) != hipSuccess) return e;
      k_lz_scale<T><<<kVB<T>, kVecThreads, 0, s>>>(v, n, pw + 1);
    }
    return hipGetLastError();
  }
  for (int it = 0; it < kPowNext; ++it) {
    hipError_t e = launch_apply(L, Prec<T>::dt, v, q, true, nullptr, nullptr, s);
    if (e != hipSuccess) return e;
    k_pow_dots<T><<<kVB<T>, kVecThreads, 0, s>>>(v, q, dinv, n, c.d_partial);
    k_pow_fin<<<1, kVecThreads, 0, s>>>(c.d_partial, kVB<T>, pw);
    k_pow_next<T><<<kVB<T>, kVecThreads, 0, s>>>(v, q, dinv, n, pw);
  }
  return hipGetLastError();
}

}  // namespace

// Builds the coarse levels (contexts at degrees p/2, p/4, ..., 1) and their work vectors.
fnpf_status mg_build(Ctx &c) {
  if (c.mg_built) return FNPF_OK;
  static bool uploaded[64] = {false};
  if (c.device >= 0 && c.device < 64 && !uploaded[c.device]) {
    if (upload_tables() != hipSuccess) return FNPF_ERR_HIP;
    uploaded[c.device] = true;
  }
  Ctx *F = &c;
  while (F->p > 1) {
    const int pc = F->p / 2;
    std::vector<int32_t> nodes;
    int64_t ns = 0;
    std::string err = coarse_numbering(*F, pc, nodes, ns);
    if (!err.empty()) {
      c.err = "p-multigrid: " + err;
      return FNPF_ERR_ARG;
    }
    fnpf_mesh_desc d{};
    d.dim = F->dim;
    d.p = pc;
    d.nz = F->nz;
    d.n_eh = F->n_eh;
    d.n_s = ns;
    d.eh_nodes = nodes.data();
    d.eh_corner = F->h_corner.data();
    d.eh_arc = F->h_arc.empty() ? nullptr : F->h_arc.data();
    d.eh_face_tag = F->h_tags.data();
    d.layer_s = F->h_layer_s.data();
    d.g = F->g;
    MgLevel L;
    fnpf_status st = fnpf_create(&d, &L.child);
    if (st != FNPF_OK) {
      c.err = std::string("p-multigrid: coarse level: ") + fnpf_last_error(nullptr);
      return st;
    }
    L.c = &ctx_of(L.child);
    if (dalloc_t(&L.Hc, L.c->n_s) != hipSuccess || dalloc_t(&L.hc, L.c->n_s) != hipSuccess) {
      c.mg.push_back(L);
      return FNPF_ERR_ALLOC;
    }
    c.mg.push_back(L);
    F = c.mg.back().c;
  }
  if (dalloc_t(&c.d_mgc, (size_t)2 * (c.mg.size() + 1) * kMgCoef) != hipSuccess) return FNPF_ERR_ALLOC;
  if (dalloc_t(&c.d_mg_lz, (size_t)kLzScalars) != hipSuccess) return FNPF_ERR_ALLOC;
  if (dalloc_t(&c.d_mg_lam, (size_t)2 * (c.mg.size() + 1)) != hipSuccess) return FNPF_ERR_ALLOC;
  if (hipMemset(c.d_mg_lam, 0, sizeof(double) * 2 * (c.mg.size() + 1)) != hipSuccess) return FNPF_ERR_HIP;
  c.mg_built = true;
  c.mg_stale64 = c.mg_stale32 = true;
  return FNPF_OK;
}

void mg_free(Ctx &c) {
  for (auto &L : c.mg) {
    if (L.Hc) (void)hipFree(L.Hc);
    if (L.hc) (void)hipFree(L.hc);
    for (int k = 0; k < 5; ++k) {
      if (L.v64[k]) (void)hipFree(L.v64[k]);
      if (L.v32[k]) (void)hipFree(L.v32[k]);
    }
    if (L.ev64) (void)hipFree(L.ev64);
    if (L.ev32) (void)hipFree(L.ev32);
    if (L.child) fnpf_destroy(L.child);
  }
  c.mg.clear();
  for (int k = 0; k < 4; ++k) {
    if (c.mg_f64[k]) (void)hipFree(c.mg_f64[k]);
    if (c.mg_f32[k]) (void)hipFree(c.mg_f32[k]);
    c.mg_f64[k] = nullptr;
    c.mg_f32[k] = nullptr;
  }
  if (c.mg_ev64) (void)hipFree(c.mg_ev64);
  if (c.mg_ev32) (void)hipFree(c.mg_ev32);
  c.mg_ev64 = nullptr;
  c.mg_ev32 = nullptr;
  c.mg_ev_ok64 = c.mg_ev_ok32 = false;
  if (c.d_mgc) (void)hipFree(c.d_mgc);
  c.d_mgc = nullptr;
  if (c.d_mg_lz) (void)hipFree(c.d_mg_lz);
  c.d_mg_lz = nullptr;
  if (c.d_mg_lam) (void)hipFree(c.d_mg_lam);
  c.d_mg_lam = nullptr;
  c.mg_built = false;
}

// Brings the coarse levels up to the current geometry (and FP32 data when T is float) and
// re-estimates the smoothing intervals.  The work vectors of precision T are allocated here.
template <typename T>
fnpf_status mg_refresh(Ctx &c, hipStream_t s) {
  fnpf_status st = mg_build(c);
  if (st != FNPF_OK) return st;
  const bool fresh = Prec<T>::fv(c)[0] == nullptr;
  if (fresh) {
    T **fv = const_cast<T **>(Prec<T>::fv(c));
    for (int k = 0; k < 4; ++k)
      if (dalloc_t(&fv[k], c.n_v) != hipSuccess) return FNPF_ERR_ALLOC;
    if (dalloc_t(&Prec<T>::evf(c), c.n_v) != hipSuccess) return FNPF_ERR_ALLOC;
    for (auto &L : c.mg) {
      T **lv = const_cast<T **>(Prec<T>::lv(L));
      for (int k = 0; k < 5; ++k)
        if (dalloc_t(&lv[k], L.c->n_v) != hipSuccess) return FNPF_ERR_ALLOC;
      if (dalloc_t(&Prec<T>::ev(L), L.c->n_v) != hipSuccess) return FNPF_ERR_ALLOC;
      if (sizeof(T) == 4 && ctx_ensure32(*L.c) != FNPF_OK) return FNPF_ERR_ALLOC;
    }
  }
  if (!Prec<T>::stale(c)) return FNPF_OK;
  Ctx *F = &c;
  for (auto &L : c.mg) {
    L.c->keep_diag = c.mg_line;
    if (surf_to(*F, *L.c, L.Hc, L.hc, s) != hipSuccess) return FNPF_ERR_HIP;
    st = geom_impl_total(*L.c, L.Hc, L.hc, s);
    if (st != FNPF_OK) return st;
    F = L.c;
  }
  if (c.mg_line) {
    // the vertical line blocks of every level from its current geometry, factored
    if (line_setup(c, s) != hipSuccess) return FNPF_ERR_HIP;
    for (auto &L : c.mg)
      if (line_setup(*L.c, s) != hipSuccess) return FNPF_ERR_HIP;
  }
  // eigenvalue estimates, warm-started from the previous geometry's eigenvector estimates, and the
  // coefficient table of this precision, all stream-ordered before any later use
  {
    const int nl = (int)c.mg.size() + 1;
    const int base = (sizeof(T) == 8 ? 0 : 1) * nl;
    double *pw = c.d_mg_scal;   // two scalars of the power iteration, apart from the partials
    for (int l = 0; l < nl; ++l) {
      hipError_t e;
      if (l == 0) {
        e = estimate_lambda<T>(c, c, Prec<T>::evf(c), Prec<T>::fv(c)[3], Prec<T>::fv(c)[1], Prec<T>::fv(c)[2],
                               Prec<T>::evokf(c), pw, s);
        Prec<T>::evokf(c) = true;
      } else {
        MgLevel &L = c.mg[l - 1];
        e = estimate_lambda<T>(c, *L.c, Prec<T>::ev(L), Prec<T>::lv(L)[4], Prec<T>::lv(L)[2], Prec<T>::lv(L)[3],
                               Prec<T>::evok(L), pw, s);
        Prec<T>::evok(L) = true;
      }
      if (e != hipSuccess) return FNPF_ERR_HIP;
      k_cheb_coef<<<1, 1, 0, s>>>(pw, l == nl - 1 ? kMgCoarseRatio : kMgSmoothRatio,
                                  c.d_mgc + (base + l) * kMgCoef, c.d_mg_lam + base + l);
      if (hipGetLastError() != hipSuccess) return FNPF_ERR_HIP;
    }
  }
  Prec<T>::stale(c) = false;
  return FNPF_OK;
}
template fnpf_status mg_refresh<double>(Ctx &, hipStream_t);
template fnpf_status mg_refresh<float>(Ctx &, hipStream_t);

template <typename T>
hipError_t mg_vcycle(Ctx &c, const T *r, T *z, const int32_t *skip, int smooth_deg, hipStream_t s,
                     double *dot_partial, bool *dot_done, bool pre_scaled) {
  if (dot_done) *dot_done = false;
  return vcycle<T>(c, 0, r, z, skip, smooth_deg, s, dot_partial, dot_done,
                   pre_scaled && smooth_deg == 2 && !c.mg.empty() && !c.mg_line);
}
template hipError_t mg_vcycle<double>(Ctx &, const double *, double *, const int32_t *, int, hipStream_t, double *,
                                      bool *, bool);
template hipError_t mg_vcycle<float>(Ctx &, const float *, float *, const int32_t *, int, hipStream_t, double *,
                                     bool *, bool);

static bool mg_prescale(const Ctx &c, int smooth_deg) { return smooth_deg == 2 && !c.mg.empty() && !c.mg_line; }

// Selects point (Jacobi) or vertical line smoothing; a change re-estimates every level's
// smoothing interval and rebuilds the line factors at the next refresh.
void mg_set_line(Ctx &c, bool line) {
  c.keep_diag = line;   // the line factors read every level's whole diagonal
  for (auto &L : c.mg) L.c->keep_diag = line;
  if (c.mg_line == line) return;
  c.mg_line = line;
  c.mg_stale64 = c.mg_stale32 = true;
  c.mg_ev_ok64 = c.mg_ev_ok32 = false;
  for (auto &L : c.mg) L.ev_ok64 = L.ev_ok32 = false;
}

hipError_t launch_mg_update(Ctx &c, fnpf_dtype dt, void *x, void *r, const void *p, const void *q, double *partial,
                            PcgScalars *sc, hipStream_t s, int smooth_deg) {
  const bool pre = mg_prescale(c, smooth_deg);
  if (dt == FNPF_F64) {
    if (pre)
      k_mg_update<double, true><<<kVecBlocks, kVecThreads, 0, s>>>(
          (double *)x, (double *)r, (const double *)p, (const double *)q, c.n_v, partial, sc,
          Prec<double>::fv(c)[2], Prec<double>::dinv(c), coef_table<double>(c, 0));
    else
      k_mg_update<double, false><<<kVecBlocks, kVecThreads, 0, s>>>((double *)x, (double *)r, (const double *)p,
                                                                    (const double *)q, c.n_v, partial, sc, nullptr,
                                                                    nullptr, nullptr);
  } else {
    if (pre)
      k_mg_update<float, true><<<kVB<float>, kVecThreads, 0, s>>>(
          (float *)x, (float *)r, (const float *)p, (const float *)q, c.n_v, partial, sc, Prec<float>::fv(c)[2],
          Prec<float>::dinv(c), coef_table<float>(c, 0));
    else
      k_mg_update<float, false><<<kVB<float>, kVecThreads, 0, s>>>((float *)x, (float *)r, (const float *)p,
                                                                   (const float *)q, c.n_v, partial, sc, nullptr,
                                                                   nullptr, nullptr);
  }
  k_mg_fin_rr<<<1, kVecThreads, 0, s>>>(partial, dt == FNPF_F64 ? kVB<double> : kVB<float>, sc);
  return hipGetLastError();
}

hipError_t launch_mg_dot_dir(Ctx &c, fnpf_dtype dt, const void *r, const void *z, void *p, double *partial,
                             PcgScalars *sc, int first, hipStream_t s, bool have_partials) {
  if (!have_partials) {
    if (dt == FNPF_F64)
      k_dot<double><<<kVecBlocks, kVecThreads, 0, s>>>((const double *)r, (const double *)z, c.n_v, partial, sc);
    else
      k_dot<float><<<kVB<float>, kVecThreads, 0, s>>>((const float *)r, (const float *)z, c.n_v, partial, sc);
  }
  k_mg_fin_rz<<<1, kVecThreads, 0, s>>>(partial, dt == FNPF_F64 ? kVB<double> : kVB<float>, sc, first);
  if (dt == FNPF_F64)
    k_mg_dir<double><<<kVecBlocks, kVecThreads, 0, s>>>((double *)p, (const double *)z, c.n_v, sc, first);
  else
    k_mg_dir<float><<<kVB<float>, kVecThreads, 0, s>>>((float *)p, (const float *)z, c.n_v, sc, first);
  return hipGetLastError();
}

}  // namespace fnpf
