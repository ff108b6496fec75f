// Vertical line smoother of the p-multigrid preconditioner.
//
// The paper's Laplace solves use CG with algebraic multigrid (Sec. 4, solver settings).  The
// extruded meshes here are strongly anisotropic between the horizontal and the vertical (thin
// layers, GLL points clustered at element faces), where a point smoother leaves error modes that
// are smooth along the vertical and rough across it.  The line smoother replaces the Jacobi
// diagonal D of the Chebyshev smoothing by B, the block-diagonal part of A_II whose blocks couple
// the unknowns of one vertical node line (levels 0 .. p nz - 1 of one horizontal node; the free
// surface level is Dirichlet).  B is symmetric positive definite (principal submatrices of A_II),
// so Chebyshev smoothing of B^-1 A on an interval of its spectrum keeps the V-cycle symmetric.
//
// Each line block is banded with half bandwidth p.  Layout of a level's band arrays, one thread
// per horizontal node n walking the levels v (consecutive n are consecutive in memory):
//   L[d][v][n], d = 0 .. p:  d = 0 holds 1 / L[v][v], d >= 1 the sub-diagonal entry L[v][v - d]
// of the Cholesky factor B_n = L_n L_n^T (the assembly kernel leaves B's sub-diagonals in the
// same places; the diagonal of B is the Jacobi diagonal).  The top level keeps 1/L = 0, so every
// solve leaves it at zero.

#include <hip/hip_runtime.h>

#include "fnpf_internal.h"

namespace fnpf {

// In place: B's sub-diagonals in L[1..p] (and its diagonal in diag) -> the Cholesky factor.  Row
// v: L[v][v-d] = (B[v][v-d] - sum_{m>d} L[v][v-m] L[v-d][v-m]) / L[v-d][v-d] for d = p .. 1, then
// L[v][v] = sqrt(B[v][v] - sum_d L[v][v-d]^2).  The last p rows of the factor stay in registers.
template <int P>
__global__ __launch_bounds__(256) void k_line_factor(double *__restrict__ L, const double *__restrict__ diag,
                                                     int64_t n_s, int nlev, int32_t *__restrict__ err) {
  const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (n >= n_s) return;
  const int64_t st = (int64_t)nlev * n_s;
  double w[P][P + 1];   // w[r][m]: row v-1-r of the factor, m = 0 diagonal, m >= 1 sub-diagonal m
#pragma unroll
  for (int r = 0; r < P; ++r)
#pragma unroll
    for (int m = 0; m <= P; ++m) w[r][m] = (m == 0) ? 1.0 : 0.0;
  bool ok = true;
  for (int v = 0; v < nlev - 1; ++v) {
    double row[P + 1];
#pragma unroll
    for (int d = P; d >= 1; --d) {
      double a = (v - d >= 0) ? L[d * st + (int64_t)v * n_s + n] : 0.0;
#pragma unroll
      for (int m = d + 1; m <= P; ++m) a -= row[m] * w[d - 1][m - d];
      row[d] = (v - d >= 0) ? a / w[d - 1][0] : 0.0;
    }
    double dd = diag[(int64_t)v * n_s + n];
#pragma unroll
    for (int d = 1; d <= P; ++d) dd -= row[d] * row[d];
    if (!(dd > 0.0)) {
      ok = false;
      dd = 1.0;
    }
    row[0] = sqrt(dd);
    L[(int64_t)v * n_s + n] = 1.0 / row[0];
#pragma unroll
    for (int d = 1; d <= P; ++d) L[d * st + (int64_t)v * n_s + n] = row[d];
#pragma unroll
    for (int r = P - 1; r >= 1; --r)
#pragma unroll
      for (int m = 0; m <= P; ++m) w[r][m] = w[r - 1][m];
#pragma unroll
    for (int m = 0; m <= P; ++m) w[0][m] = row[m];
  }
  const int v = nlev - 1;
#pragma unroll
  for (int d = 0; d <= P; ++d) L[d * st + (int64_t)v * n_s + n] = 0.0;
  if (!ok) *err = 1;
}

// Line solve z = B^-1 w with the factor, one thread per horizontal node: forward substitution
// y = L^-1 w over v = 0 .. V-2 (the last p values of y in registers, y stored in tmp), then back
// substitution z = L^-T y over v = V-2 .. 0 (the last p values of z in registers).  The modes fold
// the Chebyshev step around it into the same pass (c: the level's coefficient table, k: step):
//   kApply  w = in0;                 out = z                      (tmp may be out)
//   kCheb0  w = b = in0;             r = b, d = c0 z, x = d       (tmp = d)
//   kCheb1  w = r = b - q (in0, in1) r, d = c0 z, x += d          (tmp = q)
//   kChebK  w = r = r - q            r, d = c1 d + c2 z, x += d   (tmp = q)
//   kLanczos w = q (in0); vp = z - alpha v - beta vp               (tmp = q)
constexpr int kApply = 0, kCheb0 = 1, kCheb1 = 2, kChebK = 3, kLanczos = 4;

template <typename T, int P, int MODE>
__global__ __launch_bounds__(256) void k_line_solve(const T *__restrict__ L, const T *in0, const T *in1, T *r, T *d,
                                                    T *x, T *tmp, T *out, const double *__restrict__ cf, int k,
                                                    int64_t n_s, int nlev, const double *alpha_p,
                                                    const double *beta_p, const int32_t *__restrict__ skip) {
  if (skip != nullptr && *skip) return;
  const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (n >= n_s) return;
  const int64_t st = (int64_t)nlev * n_s;
  T c0 = T(0), c1 = T(0), c2 = T(0), al = T(0), be = T(0);
  if constexpr (MODE == kCheb0 || MODE == kCheb1) c0 = (T)cf[0];
  if constexpr (MODE == kChebK) {
    c1 = (T)cf[3 + 2 * (k - 2)];
    c2 = (T)cf[4 + 2 * (k - 2)];
  }
  if constexpr (MODE == kLanczos) {
    al = (T)*alpha_p;
    be = beta_p != nullptr ? (T)*beta_p : T(0);
  }
  // forward
  T yw[P];
#pragma unroll
  for (int m = 0; m < P; ++m) yw[m] = T(0);
  for (int v = 0; v < nlev; ++v) {
    const int64_t idx = (int64_t)v * n_s + n;
    T w;
    if constexpr (MODE == kApply || MODE == kLanczos) {
      w = in0[idx];
    } else if constexpr (MODE == kCheb0) {
      w = in0[idx];
      r[idx] = w;
    } else if constexpr (MODE == kCheb1) {
      w = in0[idx] - in1[idx];
      r[idx] = w;
    } else {
      w = r[idx] - in1[idx];
      r[idx] = w;
    }
    if (v == nlev - 1) break;   // the Dirichlet level takes no part in the solve
    T a = w;
#pragma unroll
    for (int m = 1; m <= P; ++m) a -= L[m * st + idx] * yw[m - 1];
    const T y = a * L[idx];
    tmp[idx] = y;
#pragma unroll
    for (int m = P - 1; m >= 1; --m) yw[m] = yw[m - 1];
    yw[0] = y;
  }
  // backward (z = 0 on the Dirichlet level)
  T zw[P];
#pragma unroll
  for (int m = 0; m < P; ++m) zw[m] = T(0);
  for (int v = nlev - 1; v >= 0; --v) {
    const int64_t idx = (int64_t)v * n_s + n;
    T z = T(0);
    if (v < nlev - 1) {
      T a = tmp[idx];
#pragma unroll
      for (int m = 1; m <= P; ++m)
        if (v + m < nlev - 1) a -= L[m * st + idx + (int64_t)m * n_s] * zw[m - 1];
      z = a * L[idx];
    }
    if constexpr (MODE == kApply) {
      out[idx] = z;
    } else if constexpr (MODE == kCheb0) {
      const T dv = c0 * z;
      d[idx] = dv;
      x[idx] = dv;
    } else if constexpr (MODE == kCheb1) {
      const T dv = c0 * z;
      d[idx] = dv;
      x[idx] += dv;
    } else if constexpr (MODE == kChebK) {
      const T dv = c1 * d[idx] + c2 * z;
      d[idx] = dv;
      x[idx] += dv;
    } else {
      out[idx] = z - al * x[idx] - be * out[idx];   // x = v, out = vp
    }
#pragma unroll
    for (int m = P - 1; m >= 1; --m) zw[m] = zw[m - 1];
    zw[0] = z;
  }
}

// Partials of <w, w>_B = |L^T w|^2 over the unknowns (FP64 sums, fixed grid): (L^T w)_j =
// sum_{m=0..p} L[j+m][j] w[j+m], with L[j][j] = 1 / (1/L[j][j]).
template <typename T, int P>
__global__ __launch_bounds__(kVecThreads) void k_line_bnorm(const T *__restrict__ L, const T *__restrict__ w,
                                                            int64_t n_s, int nlev, double *__restrict__ partial) {
  const int64_t st = (int64_t)nlev * n_s;
  double acc = 0.0;
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < n_s; n += (int64_t)gridDim.x * blockDim.x) {
    for (int j = 0; j < nlev - 1; ++j) {
      const int64_t idx = (int64_t)j * n_s + n;
      double a = (double)w[idx] / (double)L[idx];
#pragma unroll
      for (int m = 1; m <= P; ++m)
        if (j + m < nlev - 1) a += (double)L[m * st + idx + (int64_t)m * n_s] * (double)w[idx + (int64_t)m * n_s];
      acc += a * a;
    }
  }
  // deterministic block sum: wave shuffles, then the waves in order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __shared__ double sw[kVecThreads / 64];
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < kVecThreads / 64; ++q) s += sw[q];
    partial[blockIdx.x] = s;
  }
}

#define LINE_DISPATCH(PV, CALL)                             \
  switch (PV) {                                             \
    case 1: { constexpr int P_ = 1; CALL; } break;          \
    case 2: { constexpr int P_ = 2; CALL; } break;          \
    case 3: { constexpr int P_ = 3; CALL; } break;          \
    case 4: { constexpr int P_ = 4; CALL; } break;          \
    case 5: { constexpr int P_ = 5; CALL; } break;          \
    case 6: { constexpr int P_ = 6; CALL; } break;          \
    case 7: { constexpr int P_ = 7; CALL; } break;          \
    case 8: { constexpr int P_ = 8; CALL; } break;          \
    default: return hipErrorInvalidValue;                   \
  }

static unsigned line_blocks(const Ctx &c) { return (unsigned)((c.n_s + 255) / 256); }

// (Re)builds the level's factor from its current geometry: B's band assembled by colour, the
// factor in place (FP64), and its FP32 copy when the level keeps FP32 data.
hipError_t line_setup(Ctx &c, hipStream_t s) {
  const size_t nb = (size_t)(c.p + 1) * (size_t)(c.p * c.nz + 1) * (size_t)c.n_s;
  if (c.d_lb64 == nullptr && hipMalloc((void **)&c.d_lb64, nb * sizeof(double)) != hipSuccess)
    return hipErrorOutOfMemory;
  if (c.want32 && c.d_lb32 == nullptr && hipMalloc((void **)&c.d_lb32, nb * sizeof(float)) != hipSuccess)
    return hipErrorOutOfMemory;
  hipError_t e = ensure_diag(c, s);   // the factor's diagonal
  if (e != hipSuccess) return e;
  e = launch_line_band(c, c.d_lb64, s);
  if (e != hipSuccess) return e;
  const int nlev = c.p * c.nz + 1;
  LINE_DISPATCH(c.p, (k_line_factor<P_><<<line_blocks(c), 256, 0, s>>>(c.d_lb64, c.d_diag, c.n_s, nlev, c.d_err)));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (c.want32) return launch_cast_f32(c.d_lb64, c.d_lb32, (int64_t)nb, s);
  return hipSuccess;
}

template <typename T>
static const T *line_factor(const Ctx &c);
template <>
const double *line_factor<double>(const Ctx &c) { return c.d_lb64; }
template <>
const float *line_factor<float>(const Ctx &c) { return c.d_lb32; }

template <typename T, int MODE>
static hipError_t line_launch(const Ctx &c, const T *in0, const T *in1, T *r, T *d, T *x, T *tmp, T *out,
                              const double *cf, int k, const double *al, const double *be, const int32_t *skip,
                              hipStream_t s) {
  const T *L = line_factor<T>(c);
  if (L == nullptr) return hipErrorInvalidValue;
  const int nlev = c.p * c.nz + 1;
  LINE_DISPATCH(c.p, (k_line_solve<T, P_, MODE><<<line_blocks(c), 256, 0, s>>>(
                         L, in0, in1, r, d, x, tmp, out, cf, k, c.n_s, nlev, al, be, skip)));
  return hipGetLastError();
}

template <typename T>
hipError_t line_apply(const Ctx &c, const T *w, T *z, hipStream_t s) {
  return line_launch<T, kApply>(c, w, nullptr, nullptr, nullptr, nullptr, z, z, nullptr, 0, nullptr, nullptr,
                                nullptr, s);
}
template hipError_t line_apply<double>(const Ctx &, const double *, double *, hipStream_t);
template hipError_t line_apply<float>(const Ctx &, const float *, float *, hipStream_t);

template <typename T>
hipError_t line_cheb0(const Ctx &c, const T *b, T *r, T *d, T *x, const double *cf, const int32_t *skip,
                      hipStream_t s) {
  return line_launch<T, kCheb0>(c, b, nullptr, r, d, x, d, nullptr, cf, 0, nullptr, nullptr, skip, s);
}
template <typename T>
hipError_t line_cheb1(const Ctx &c, const T *b, T *q, T *r, T *d, T *x, const double *cf, const int32_t *skip,
                      hipStream_t s) {
  return line_launch<T, kCheb1>(c, b, q, r, d, x, q, nullptr, cf, 0, nullptr, nullptr, skip, s);
}
template <typename T>
hipError_t line_chebk(const Ctx &c, T *q, T *r, T *d, T *x, const double *cf, int k, const int32_t *skip,
                      hipStream_t s) {
  return line_launch<T, kChebK>(c, nullptr, q, r, d, x, q, nullptr, cf, k, nullptr, nullptr, skip, s);
}
template <typename T>
hipError_t line_lanczos_w(const Ctx &c, T *q, const T *v, T *vp, const double *al, const double *be, hipStream_t s) {
  return line_launch<T, kLanczos>(c, q, nullptr, nullptr, nullptr, const_cast<T *>(v), q, vp, nullptr, 0, al, be,
                                  nullptr, s);
}
template <typename T>
hipError_t line_bnorm_partials(const Ctx &c, const T *w, double *partial, int nblocks, hipStream_t s) {
  const T *L = line_factor<T>(c);
  if (L == nullptr) return hipErrorInvalidValue;
  const int nlev = c.p * c.nz + 1;
  LINE_DISPATCH(c.p, (k_line_bnorm<T, P_><<<nblocks, kVecThreads, 0, s>>>(L, w, c.n_s, nlev, partial)));
  return hipGetLastError();
}

#define LINE_INST(T)                                                                                          \
  template hipError_t line_cheb0<T>(const Ctx &, const T *, T *, T *, T *, const double *, const int32_t *,   \
                                    hipStream_t);                                                             \
  template hipError_t line_cheb1<T>(const Ctx &, const T *, T *, T *, T *, T *, const double *,               \
                                    const int32_t *, hipStream_t);                                            \
  template hipError_t line_chebk<T>(const Ctx &, T *, T *, T *, T *, const double *, int, const int32_t *,     \
                                    hipStream_t);                                                             \
  template hipError_t line_lanczos_w<T>(const Ctx &, T *, const T *, T *, const double *, const double *,      \
                                        hipStream_t);                                                         \
  template hipError_t line_bnorm_partials<T>(const Ctx &, const T *, double *, int, hipStream_t);
LINE_INST(double)
LINE_INST(float)

}  // namespace fnpf
