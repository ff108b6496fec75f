// Vector kernels of the preconditioned conjugate-gradient solve (paper Sec. 4: CG for the
// Laplace system) and its FP64/FP32 defect correction.
//
// All reductions are deterministic: grid-stride kernels with a fixed grid write one FP64
// partial per block (wave64 shuffle reduction, then the block's waves in order), and a
// single-block finalize kernel sums the partials in a fixed order and updates the device
// scalars (alpha, beta, convergence flag).  Once `done` is set, every later kernel of the
// iteration returns immediately, so the host may check convergence only every few
// iterations without changing the result.
//
// Vectors hold all n_v volume nodes; the free-surface level [top*n_s, n_v) of r, p, q and
// dinv is kept at zero, so the iteration acts on the non-surface unknowns only.

#include <hip/hip_runtime.h>

#include "fnpf_internal.h"

namespace fnpf {

namespace {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block reduction of NS sums; thread 0 writes them to partial[blockIdx.x * NS + k].
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

// Fixed-order sum of np partial tuples (stride NS) by one block.
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
    if (threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < NS; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) out[k] = s[k][0];
}

__global__ void k_set_lift(double *v, const double *phis, int64_t n_v, int64_t top0) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_v; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = i >= top0 ? phis[i - top0] : 0.0;
}

__global__ void k_copy_top(double *x, const double *phis, int64_t n_s, int64_t top0) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_s; i += (int64_t)gridDim.x * blockDim.x)
    x[top0 + i] = phis[i];
}

__global__ void k_fill(double *v, double val, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = val;
}

__global__ void k_zero_i32(int32_t *v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) v[i] = 0;
}

__global__ void k_cast_f32(const double *a, float *b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

// ||b||^2 with b = f - A [0; phi_s] (y = A [0; phi_s], surface rows masked to 0).
__global__ __launch_bounds__(kVecThreads) void k_bnorm(const double *f, const double *y, int64_t n_v, int64_t top0,
                                                       double *partial) {
  double v[1] = {0.0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < top0; i += (int64_t)gridDim.x * blockDim.x) {
    double b = (f ? f[i] : 0.0) - y[i];
    v[0] += b * b;
  }
  block_partials<1>(v, partial);
}

__global__ __launch_bounds__(kVecThreads) void k_fin_bnorm(const double *partial, int np, PcgScalars *sc, double rtol,
                                                           double atol) {
  double s[1];
  final_sums<1>(partial, np, s);
  if (threadIdx.x == 0) {
    sc->bnorm2 = s[0];
    sc->tol2 = fmax(rtol * rtol * s[0], atol * atol);
  }
}

// r = f - A x (surface rows 0), z = dinv r, p = z; partial sums (r.z, r.r).
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_pcg_init(const double *f, const T *Ax, T *r, T *p, const T *dinv,
                                                          int64_t n_v, int64_t top0, double *partial) {
  double v[2] = {0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_v; i += (int64_t)gridDim.x * blockDim.x) {
    T ri = i < top0 ? (T)((f ? f[i] : 0.0) - (double)Ax[i]) : T(0);
    T zi = dinv[i] * ri;
    r[i] = ri;
    p[i] = zi;
    v[0] += (double)ri * (double)zi;
    v[1] += (double)ri * (double)ri;
  }
  block_partials<2>(v, partial);
}

__global__ __launch_bounds__(kVecThreads) void k_fin_init(const double *partial, int np, PcgScalars *sc, int relative,
                                                          double inner_rtol) {
  double s[2];
  final_sums<2>(partial, np, s);
  if (threadIdx.x == 0) {
    sc->rz = s[0];
    sc->rr = s[1];
    sc->rr0 = s[1];
    if (relative) sc->tol2 = inner_rtol * inner_rtol * s[1];
    sc->iters = 0;
    sc->breakdown = (s[1] == s[1] && s[1] <= 1e300) ? 0 : 2;
    sc->done = (sc->breakdown != 0 || s[1] <= sc->tol2) ? 1 : 0;
    sc->alpha = 0.0;
    sc->beta = 0.0;
  }
}

// Outer residual of the mixed solve: r64 = f - A64 x (surface 0); r32 = (float) r64; the
// inner FP32 PCG starts from d = 0: z = dinv32 r32, p = z.  Partials (r64.r64, r32.z, r32.r32).
__global__ __launch_bounds__(kVecThreads) void k_resid_to32(const double *f, const double *Ax, float *r, float *p,
                                                            float *d, const float *dinv, int64_t n_v, int64_t top0,
                                                            double *partial) {
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_v; i += (int64_t)gridDim.x * blockDim.x) {
    double r64 = i < top0 ? (f ? f[i] : 0.0) - Ax[i] : 0.0;
    float r32 = (float)r64;
    float z = dinv[i] * r32;
    r[i] = r32;
    p[i] = z;
    d[i] = 0.0f;
    v[0] += r64 * r64;
    v[1] += (double)r32 * (double)z;
    v[2] += (double)r32 * (double)r32;
  }
  block_partials<3>(v, partial);
}

// The inner FP32 solve stops at its relative reduction or, earlier, once its residual is below
// this fraction of the outer tolerance: the FP64 test that follows then passes unless the FP32
// rounding of the correction is larger, so iterations past that point would be wasted.
constexpr double kInnerFloor = 0.5;

__global__ __launch_bounds__(kVecThreads) void k_fin_outer(const double *partial, int np, PcgScalars *outer,
                                                           PcgScalars *inner, double inner_rtol) {
  double s[3];
  final_sums<3>(partial, np, s);
  if (threadIdx.x == 0) {
    outer->rr = s[0];
    outer->breakdown = (s[0] == s[0] && s[0] <= 1e300) ? 0 : 2;
    outer->done = (outer->breakdown != 0 || s[0] <= outer->tol2) ? 1 : 0;
    inner->rz = s[1];
    inner->rr = s[2];
    inner->rr0 = s[2];
    inner->tol2 = fmax(inner_rtol * inner_rtol * s[2], kInnerFloor * kInnerFloor * outer->tol2);
    inner->iters = 0;
    inner->breakdown = 0;
    inner->alpha = 0.0;
    inner->beta = 0.0;
    inner->done = (outer->done || s[2] <= inner->tol2) ? 1 : 0;
  }
}

__global__ __launch_bounds__(kVecThreads) void k_fin_pq(const double *partial, int np, PcgScalars *sc) {
  if (sc->done) return;
  double s[1];
  final_sums<1>(partial, np, s);
  if (threadIdx.x == 0) {
    sc->pq = s[0];
    if (!(s[0] > 0.0) || !(s[0] <= 1e300)) {
      sc->breakdown = (s[0] == s[0]) ? 1 : 2;
      sc->done = 1;
      sc->alpha = 0.0;
    } else {
      sc->alpha = sc->rz / s[0];
    }
  }
}

// x += alpha p ; r -= alpha q ; partial sums (r.z, r.r) with z = dinv r.
// Vectorised over 16-byte chunks (VW elements); the tail is handled element-wise.
template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int W = 2;
};
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int W = 4;
};

template <typename T>
__device__ __forceinline__ void upd_one(T *x, T *r, const T *p, const T *q, const T *dinv, int64_t i, T a,
                                        double (&v)[2]) {
  x[i] = x[i] + a * p[i];
  T ri = r[i] - a * q[i];
  r[i] = ri;
  T zi = dinv[i] * ri;
  v[0] += (double)ri * (double)zi;
  v[1] += (double)ri * (double)ri;
}

// element-wise fallback (operands not 16-byte aligned)
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_pcg_update_scalar(T *x, T *r, const T *p, const T *q, const T *dinv,
                                                                   int64_t n_v, double *partial,
                                                                   const PcgScalars *sc) {
  if (sc->done) return;
  const T a = (T)sc->alpha;
  double v[2] = {0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_v; i += (int64_t)gridDim.x * blockDim.x)
    upd_one(x, r, p, q, dinv, i, a, v);
  block_partials<2>(v, partial);
}

template <typename T, typename TX>
__global__ __launch_bounds__(kVecThreads) void k_pcg_update(TX *x, T *r, const T *p, const T *q, const T *dinv,
                                                            int64_t n_v, double *partial, const PcgScalars *sc) {
  static_assert(sizeof(T) == sizeof(TX), "the solution and the residual share the precision");
  if (sc->done) return;
  const T a = (T)sc->alpha;
  double v[2] = {0.0, 0.0};
  using V = typename Vec16<T>::type;
  constexpr int W = Vec16<T>::W;
  const int64_t nvec = n_v / W;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nvec; c += stride) {
    V xv = reinterpret_cast<V *>(x)[c];
    V rv = reinterpret_cast<V *>(r)[c];
    const V pv = reinterpret_cast<const V *>(p)[c];
    const V qv = reinterpret_cast<const V *>(q)[c];
    const V dv = reinterpret_cast<const V *>(dinv)[c];
    T *xs = reinterpret_cast<T *>(&xv);
    T *rs = reinterpret_cast<T *>(&rv);
    const T *ps = reinterpret_cast<const T *>(&pv);
    const T *qs = reinterpret_cast<const T *>(&qv);
    const T *ds = reinterpret_cast<const T *>(&dv);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      xs[w] = xs[w] + a * ps[w];
      const T ri = rs[w] - a * qs[w];
      rs[w] = ri;
      const T zi = ds[w] * ri;
      v[0] += (double)ri * (double)zi;
      v[1] += (double)ri * (double)ri;
    }
    reinterpret_cast<V *>(x)[c] = xv;
    reinterpret_cast<V *>(r)[c] = rv;
  }
  if (blockIdx.x == 0)
    for (int64_t i = nvec * W + threadIdx.x; i < n_v; i += blockDim.x) upd_one(x, r, p, q, dinv, i, a, v);
  block_partials<2>(v, partial);
}

__global__ __launch_bounds__(kVecThreads) void k_fin_rz(const double *partial, int np, PcgScalars *sc) {
  if (sc->done) return;
  double s[2];
  final_sums<2>(partial, np, s);
  if (threadIdx.x == 0) {
    sc->beta = s[0] / sc->rz;
    sc->rz = s[0];
    sc->rr = s[1];
    sc->iters += 1;
    if (!(s[1] == s[1]) || !(s[1] <= 1e300)) {
      sc->breakdown = 2;
      sc->done = 1;
    } else if (s[1] <= sc->tol2) {
      sc->done = 1;
    }
  }
}

// p = dinv r + beta p
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_pcg_dir(T *p, const T *r, const T *dinv, int64_t n_v,
                                                         const PcgScalars *sc) {
  if (sc->done) return;
  const T b = (T)sc->beta;
  using V = typename Vec16<T>::type;
  constexpr int W = Vec16<T>::W;
  const int64_t nvec = n_v / W;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nvec; c += stride) {
    V pv = reinterpret_cast<V *>(p)[c];
    const V rv = reinterpret_cast<const V *>(r)[c];
    const V dv = reinterpret_cast<const V *>(dinv)[c];
    T *ps = reinterpret_cast<T *>(&pv);
    const T *rs = reinterpret_cast<const T *>(&rv);
    const T *ds = reinterpret_cast<const T *>(&dv);
#pragma unroll
    for (int w = 0; w < W; ++w) ps[w] = ds[w] * rs[w] + b * ps[w];
    reinterpret_cast<V *>(p)[c] = pv;
  }
  if (blockIdx.x == 0)
    for (int64_t i = nvec * W + threadIdx.x; i < n_v; i += blockDim.x) p[i] = dinv[i] * r[i] + b * p[i];
}

__global__ void k_add_f32(double *x, const float *d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] += (double)d[i];
}

__global__ void k_lincomb(double *out, double a, const double *x, double b, const double *y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (x ? a * x[i] : 0.0) + (y ? b * y[i] : 0.0);
}

// VJP of the linear free-surface conditions (d eta/dt = w, d phi_s/dt = -g eta):
// eta_bar += -g kbar_p, w_bar += kbar_e
__global__ void k_rhs_vjp_linear(const double *kbe, const double *kbp, double *eta_bar, double *w_bar, double g,
                                 int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    eta_bar[i] -= g * kbp[i];
    w_bar[i] += kbe[i];
  }
}

__global__ void k_relax_vjp(double *v, const double *cr, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] *= (1.0 - cr[i]);
}

// phi_s bar += phi_bar(surface level) - (A lambda)(surface level)
__global__ void k_surface_adj(double *phis_bar, const double *phibar, const double *Alam, int64_t n_s,
                              int64_t top0) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_s; i += (int64_t)gridDim.x * blockDim.x)
    phis_bar[i] += phibar[top0 + i] - Alam[top0 + i];
}

}  // namespace

hipError_t launch_lincomb(double *out, double a, const double *x, double b, const double *y, int64_t n,
                          hipStream_t s) {
  k_lincomb<<<kVecBlocks, kVecThreads, 0, s>>>(out, a, x, b, y, n);
  return hipGetLastError();
}

hipError_t launch_rhs_vjp_linear(const double *kbe, const double *kbp, double *eta_bar, double *w_bar, double g,
                                 int64_t n, hipStream_t s) {
  k_rhs_vjp_linear<<<kVecBlocks, kVecThreads, 0, s>>>(kbe, kbp, eta_bar, w_bar, g, n);
  return hipGetLastError();
}

hipError_t launch_relax_vjp(double *v, const double *cr, int64_t n, hipStream_t s) {
  k_relax_vjp<<<kVecBlocks, kVecThreads, 0, s>>>(v, cr, n);
  return hipGetLastError();
}

hipError_t launch_surface_adj(double *phis_bar, const double *phibar, const double *Alam, int64_t n_v, int64_t n_s,
                              hipStream_t s) {
  k_surface_adj<<<kVecBlocks, kVecThreads, 0, s>>>(phis_bar, phibar, Alam, n_s, n_v - n_s);
  return hipGetLastError();
}

hipError_t launch_set_lift(double *v, const double *phis, int64_t n_v, int64_t n_s, hipStream_t s) {
  k_set_lift<<<kVecBlocks, kVecThreads, 0, s>>>(v, phis, n_v, n_v - n_s);
  return hipGetLastError();
}

hipError_t launch_copy_top(double *x, const double *phis, int64_t n_v, int64_t n_s, hipStream_t s) {
  k_copy_top<<<kVecBlocks, kVecThreads, 0, s>>>(x, phis, n_s, n_v - n_s);
  return hipGetLastError();
}

hipError_t launch_fill(double *v, double val, int64_t n, hipStream_t s) {
  k_fill<<<kVecBlocks, kVecThreads, 0, s>>>(v, val, n);
  return hipGetLastError();
}

hipError_t launch_zero_i32(int32_t *v, int64_t n, hipStream_t s) {
  k_zero_i32<<<1, 64, 0, s>>>(v, n);
  return hipGetLastError();
}

hipError_t launch_cast_f32(const double *a, float *b, int64_t n, hipStream_t s) {
  k_cast_f32<<<kVecBlocks, kVecThreads, 0, s>>>(a, b, n);
  return hipGetLastError();
}

hipError_t launch_bnorm(const double *f, const double *y, int64_t n_v, int64_t n_s, double *partial,
                        PcgScalars *sc, double rtol, double atol, hipStream_t s) {
  k_bnorm<<<kVecBlocks, kVecThreads, 0, s>>>(f, y, n_v, n_v - n_s, partial);
  k_fin_bnorm<<<1, kVecThreads, 0, s>>>(partial, kVecBlocks, sc, rtol, atol);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pcg_init(const double *f, const T *Ax, T *r, T *p, const T *dinv, int64_t n_v, int64_t n_s,
                           double *partial, PcgScalars *sc, bool relative_tol, double inner_rtol, hipStream_t s) {
  k_pcg_init<T><<<kVecBlocks, kVecThreads, 0, s>>>(f, Ax, r, p, dinv, n_v, n_v - n_s, partial);
  k_fin_init<<<1, kVecThreads, 0, s>>>(partial, kVecBlocks, sc, relative_tol ? 1 : 0, inner_rtol);
  return hipGetLastError();
}
template hipError_t launch_pcg_init<double>(const double *, const double *, double *, double *, const double *,
                                            int64_t, int64_t, double *, PcgScalars *, bool, double, hipStream_t);

hipError_t launch_resid_to32(const double *f, const double *Ax, float *r, float *p, float *d, const float *dinv,
                             int64_t n_v, int64_t n_s, double *partial, PcgScalars *outer, PcgScalars *inner,
                             double inner_rtol, hipStream_t s) {
  k_resid_to32<<<kVecBlocks, kVecThreads, 0, s>>>(f, Ax, r, p, d, dinv, n_v, n_v - n_s, partial);
  k_fin_outer<<<1, kVecThreads, 0, s>>>(partial, kVecBlocks, outer, inner, inner_rtol);
  return hipGetLastError();
}

hipError_t launch_finalize_pq(const double *partial, int np, PcgScalars *sc, hipStream_t s) {
  k_fin_pq<<<1, kVecThreads, 0, s>>>(partial, np, sc);
  return hipGetLastError();
}

template <typename T, typename TX>
hipError_t launch_pcg_update(TX *x, T *r, const T *p, const T *q, const T *dinv, int64_t n_v, double *partial,
                             PcgScalars *sc, hipStream_t s) {
  // every vector here is a device allocation (256-byte aligned) except x, which may be a caller
  // tensor: the vectorised kernel requires 16-byte alignment of all operands
  if ((reinterpret_cast<uintptr_t>(x) & 15) != 0)
    k_pcg_update_scalar<T><<<kVecBlocks, kVecThreads, 0, s>>>(x, r, p, q, dinv, n_v, partial, sc);
  else
    k_pcg_update<T, TX><<<kVecBlocks, kVecThreads, 0, s>>>(x, r, p, q, dinv, n_v, partial, sc);
  k_fin_rz<<<1, kVecThreads, 0, s>>>(partial, kVecBlocks, sc);
  return hipGetLastError();
}
template hipError_t launch_pcg_update<double, double>(double *, double *, const double *, const double *,
                                                      const double *, int64_t, double *, PcgScalars *, hipStream_t);
template hipError_t launch_pcg_update<float, float>(float *, float *, const float *, const float *, const float *,
                                                    int64_t, double *, PcgScalars *, hipStream_t);

hipError_t launch_finalize_rz(const double *partial, int np, PcgScalars *sc, hipStream_t s) {
  k_fin_rz<<<1, kVecThreads, 0, s>>>(partial, np, sc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pcg_dir(T *p, const T *r, const T *dinv, int64_t n_v, PcgScalars *sc, hipStream_t s) {
  k_pcg_dir<T><<<kVecBlocks, kVecThreads, 0, s>>>(p, r, dinv, n_v, sc);
  return hipGetLastError();
}
template hipError_t launch_pcg_dir<double>(double *, const double *, const double *, int64_t, PcgScalars *,
                                           hipStream_t);
template hipError_t launch_pcg_dir<float>(float *, const float *, const float *, int64_t, PcgScalars *, hipStream_t);

hipError_t launch_add_f32(double *x, const float *d, int64_t n_v, hipStream_t s) {
  k_add_f32<<<kVecBlocks, kVecThreads, 0, s>>>(x, d, n_v);
  return hipGetLastError();
}

}  // namespace fnpf
