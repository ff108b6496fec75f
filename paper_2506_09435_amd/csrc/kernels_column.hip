// Column kernels of the extruded spectral-element mesh (gfx950, wave64).
//
// Work decomposition shared by every kernel here: a workgroup holds CPB
// element columns; one thread per (column, horizontal GLL node (i, j)) walks
// its vertical node line bottom to top, layer by layer, keeping the line in
// registers.  Element tiles of one layer are staged in LDS for the xi/eta
// contractions; the zeta contraction stays in registers.  The node level
// shared by two stacked layers is carried in a register, so each thread
// writes every volume node of its line exactly once.
//
// Assembly across columns uses a colouring of the columns (columns of one
// colour share no horizontal node), one launch per colour, no atomics: the
// first colour that touches a horizontal node stores, later colours
// read-add-store, and the last one sees the assembled value (used for fused
// dot products, w recovery and the RK4 update).
//
// Notation: D is the GLL derivative matrix, W the GLL weights, G the six
// (3D) or three (2D) symmetric per-point factors w_q det(J) (J^-1 J^-T)_ab of
// the Laplace bilinear form (paper Eq. 4).  Volume vectors are layer-major:
// index = v * n_s + hn.

#include <hip/hip_runtime.h>

#include "fnpf_internal.h"
#include "stage_update.h"

namespace fnpf {

__constant__ double c_D64[kMaxN1 * kDStride];
__constant__ float c_D32[kMaxN1 * kDStride];
__constant__ double c_W[kMaxN1 * kMaxN1];
__constant__ double c_DSQ64[kMaxN1 * kDStride];   // D[r][c]^2 (the assembled diagonal's line sums)

// Even-odd coefficient tables of the line contractions with D (tr = 0) and D^T (tr = 1), per
// degree p, with H = (p+1)/2 pairs (r, p-r) and, for even p, the middle index c = p/2.  Both
// matrices are centro-antisymmetric, M[p-r][p-m] = -M[r][m]; the table stores
//   A[r][m] = (M[r][m] - M[r][p-m]) / 2,  B[r][m] = (M[r][m] + M[r][p-m]) / 2   (r, m < H),
//   Bc[r] = M[r][c],  Cc[m] = M[c][m]                                            (even p),
// taken from the antisymmetrised M~[r][m] = (M[r][m] - M[p-r][p-m]) / 2.
constexpr int kMaxH = kMaxN1 / 2;
constexpr int kEOStride = 2 * kMaxH * kMaxH + 2 * kMaxH;
__constant__ double c_EO64[(kMaxP + 1) * 2 * kEOStride];
__constant__ float c_EO32[(kMaxP + 1) * 2 * kEOStride];
// Even-odd table of the squared-derivative line sum out_r = sum_m D[m][r]^2 in_m (the diagonal's
// line sums): its matrix Q[r][m] = D[m][r]^2 is centro-symmetric, Q[p-r][p-m] = Q[r][m]; the
// table stores A[r][m] = (Q[r][m] - Q[r][p-m]) / 2, B[r][m] = (Q[r][m] + Q[r][p-m]) / 2 (r, m < H)
// and, for even p, Bc[r] = Q[r][c], Cc[m] = Q[c][m] (m < H) and Q[c][c].
constexpr int kSqStride = 2 * kMaxH * kMaxH + 2 * kMaxH + 1;
__constant__ double c_SQEO64[(kMaxP + 1) * kSqStride];

// Face-slot scratch of the allocation-free apply (fnpf_laplace_apply_noalloc): a file-scope array
// in the library's device code, one copy per GPU, allocated when the code object is loaded and
// held until the process ends.  Host code never passes its name to a kernel (on the host it is a
// stand-in, not a device address): init_noalloc_scratch stores each device's address of it, taken
// with hipGetSymbolAddress while that device is current, and the apply takes that address.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];
constexpr int kMaxDevices = 64;
static void *g_scratch_dev[kMaxDevices] = {nullptr};

hipError_t init_noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (g_scratch_dev[device] != nullptr) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_dev[device] = ptr;
  return hipSuccess;
}

void *noalloc_scratch(int device) {
  return (device >= 0 && device < kMaxDevices) ? g_scratch_dev[device] : nullptr;
}

size_t noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

hipError_t upload_constants(int /*device*/) {
  static double D64[kMaxN1 * kDStride];
  static double DSQ64[kMaxN1 * kDStride];
  static float D32[kMaxN1 * kDStride];
  static double W[kMaxN1 * kMaxN1];
  static double EO64[(kMaxP + 1) * 2 * kEOStride];
  static float EO32[(kMaxP + 1) * 2 * kEOStride];
  static double SQEO64[(kMaxP + 1) * kSqStride];
  for (int p = 1; p <= kMaxP; ++p) {
    double x[kMaxN1], w[kMaxN1], D[kMaxN1 * kMaxN1];
    gll_host(p, x, w, D);
    const int n1 = p + 1;
    for (int i = 0; i < n1 * n1; ++i) {
      D64[p * kDStride + i] = D[i];
      DSQ64[p * kDStride + i] = D[i] * D[i];
      D32[p * kDStride + i] = (float)D[i];
    }
    for (int i = 0; i < n1; ++i) W[p * kMaxN1 + i] = w[i];
    const int H = n1 / 2, c = p / 2;
    for (int tr = 0; tr < 2; ++tr) {
      auto M = [&](int r, int m) {
        const double a = tr ? D[m * n1 + r] : D[r * n1 + m];
        const double b = tr ? D[(p - m) * n1 + (p - r)] : D[(p - r) * n1 + (p - m)];
        return 0.5 * (a - b);
      };
      double *E = EO64 + (p * 2 + tr) * kEOStride;
      for (int r = 0; r < H; ++r)
        for (int m = 0; m < H; ++m) {
          E[r * H + m] = 0.5 * (M(r, m) - M(r, p - m));
          E[H * H + r * H + m] = 0.5 * (M(r, m) + M(r, p - m));
        }
      if (n1 & 1)
        for (int r = 0; r < H; ++r) {
          E[2 * H * H + r] = M(r, c);
          E[2 * H * H + H + r] = M(c, r);
        }
      for (int k = 0; k < kEOStride; ++k) EO32[(p * 2 + tr) * kEOStride + k] = (float)E[k];
    }
    {
      auto Q = [&](int r, int m) { return D[m * n1 + r] * D[m * n1 + r]; };
      double *E = SQEO64 + p * kSqStride;
      for (int r = 0; r < H; ++r)
        for (int m = 0; m < H; ++m) {
          E[r * H + m] = 0.5 * (Q(r, m) - Q(r, p - m));
          E[H * H + r * H + m] = 0.5 * (Q(r, m) + Q(r, p - m));
        }
      if (n1 & 1) {
        for (int r = 0; r < H; ++r) {
          E[2 * H * H + r] = Q(r, c);
          E[2 * H * H + H + r] = Q(c, r);
        }
        E[2 * H * H + 2 * H] = Q(c, c);
      }
    }
  }
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_D64), D64, sizeof(D64));
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_DSQ64), DSQ64, sizeof(DSQ64));
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_D32), D32, sizeof(D32));
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_EO64), EO64, sizeof(EO64));
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_EO32), EO32, sizeof(EO32));
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_SQEO64), SQEO64, sizeof(SQEO64));
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_W), W, sizeof(W));
}

template <int P, int DIM>
struct Sh {
  static constexpr int N1 = P + 1;
  static constexpr int NH = DIM == 3 ? N1 * N1 : N1;
  static constexpr int NP = NH * N1;
  static constexpr int NG = DIM == 3 ? 6 : 3;
  static constexpr int CPB = 256 / NH;
  static constexpr int NT = CPB * NH;
};

template <typename T>
__device__ __forceinline__ T dmat(int P, int r, int c);
template <>
__device__ __forceinline__ double dmat<double>(int P, int r, int c) {
  return c_D64[P * kDStride + r * (P + 1) + c];
}
template <>
__device__ __forceinline__ float dmat<float>(int P, int r, int c) {
  return c_D32[P * kDStride + r * (P + 1) + c];
}
__device__ __forceinline__ double wgt(int P, int i) { return c_W[P * kMaxN1 + i]; }
// 1/a for the Jacobi inverses: the hardware reciprocal estimate refined by two Newton steps
// (r <- r + r (1 - a r)), within an ulp or two of the correctly rounded quotient at a fraction of
// the IEEE division's instruction count; a is a positive diagonal entry
__device__ __forceinline__ double recip(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = fma(r, fma(-a, r, 1.0), r);
  return fma(r, fma(-a, r, 1.0), r);
}
// The squared-derivative table of degree P behind an opaque zero offset that depends on `dep`:
// its scalar loads cannot be hoisted above `dep` (so the 49 FP64 entries at P = 6 are not held in
// scalar registers across the whole kernel, which spills them to vector lanes).
template <typename U>
__device__ __forceinline__ const double *dsq_ptr(int P, const U &dep) {
  int z = 0;
  asm volatile("" : "+s"(z) : "v"(dep));
  return c_DSQ64 + P * kDStride + z;
}

// Raw buffer access: a per-thread 32-bit byte offset plus a wave-uniform row offset, so the
// vertical walk needs one address register per thread.  The descriptor's record count is the
// vector's size: accesses beyond it read 0 and drop writes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t vec_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_st(double v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  using V1 = unsigned long long __attribute__((ext_vector_type(1)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V1, v), r, voff, soff, 0);
}
__device__ __forceinline__ void buf_st(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}

template <typename T>
__device__ __forceinline__ const T *eo_table();
template <>
__device__ __forceinline__ const double *eo_table<double>() { return c_EO64; }
template <>
__device__ __forceinline__ const float *eo_table<float>() { return c_EO32; }

// out = M in along one line of N1 = P+1 nodes, M = D (TR = 0) or D^T (TR = 1), in even-odd
// form: e_m = in_m + in_{P-m}, o_m = in_m - in_{P-m} for m < H, then
//   out_r = sum_m A_rm o_m + S_r,  out_{P-r} = sum_m A_rm o_m - S_r,
//   S_r = sum_m B_rm e_m (+ Bc_r in_c for even P),  out_c = sum_m Cc_m o_m,
// about half the multiply-adds of the dense product.  The coefficients are read through the
// scalar cache at every call (the zero offset is opaque to the compiler), so they occupy
// scalar registers only while the line is computed.
// Even-odd table of D (TR = 0) or D^T (TR = 1) for degree P.  The zero offset passes through an
// empty asm statement that takes `dep` as an input, so the table's scalar loads cannot be
// scheduled before `dep` exists: a caller ties them to the data of the phase that uses them, and
// only one table (48 SGPRs in FP64 at P = 6) is live at a time.
template <int P, typename T, int TR, typename U>
__device__ __forceinline__ const T *eo_ptr(const U &dep) {
  int z = 0;
  asm volatile("" : "+s"(z) : "v"(dep));
  return eo_table<T>() + (P * 2 + TR) * kEOStride + z;
}

template <int P, typename T>
__device__ __forceinline__ void line_eo(const T (&in)[P + 1], T (&out)[P + 1], const T *__restrict__ E) {
  constexpr int N1 = P + 1, H = N1 / 2, C = P / 2;
  T e[H], o[H];
#pragma unroll
  for (int m = 0; m < H; ++m) {
    e[m] = in[m] + in[P - m];
    o[m] = in[m] - in[P - m];
  }
#pragma unroll
  for (int r = 0; r < H; ++r) {
    T so = E[r * H] * o[0];
    T se = E[H * H + r * H] * e[0];
#pragma unroll
    for (int m = 1; m < H; ++m) {
      so += E[r * H + m] * o[m];
      se += E[H * H + r * H + m] * e[m];
    }
    if constexpr ((N1 & 1) != 0) se += E[2 * H * H + r] * in[C];
    out[r] = so + se;
    out[P - r] = so - se;
  }
  if constexpr ((N1 & 1) != 0) {
    T sc = E[2 * H * H + H] * o[0];
#pragma unroll
    for (int m = 1; m < H; ++m) sc += E[2 * H * H + H + m] * o[m];
    out[C] = sc;
  }
}

// The squared-derivative line sum out_r = sum_m D[m][r]^2 in_m in even-odd form (table above),
// for degrees up to 6 (with positive inputs its rounding error stays within 3e-15 relative there,
// against 2e-14 at degrees 7 and 8, where the dense sum is kept):
//   out_r = S_r + O_r,  out_{P-r} = S_r - O_r,  S_r = sum_m B_rm e_m (+ Bc_r in_c),  O_r = sum_m A_rm o_m,
//   out_c = sum_m Cc_m e_m + Q_cc in_c  (even P).  Q points at the degree's table behind an opaque
// offset (sqeo_ptr), as the other line tables.
template <typename U>
__device__ __forceinline__ const double *sqeo_ptr(int P, const U &dep) {
  int z = 0;
  asm volatile("" : "+s"(z) : "v"(dep));
  return c_SQEO64 + P * kSqStride + z;
}
template <int P>
__device__ __forceinline__ void line_sq_eo(const double (&in)[P + 1], double (&out)[P + 1],
                                           const double *__restrict__ Q) {
  constexpr int N1 = P + 1, H = N1 / 2, C = P / 2;
  static_assert(P <= 6, "the differences o_m cancel more at higher degree: use the dense sum there");
  double e[H], o[H];
#pragma unroll
  for (int m = 0; m < H; ++m) {
    e[m] = in[m] + in[P - m];
    o[m] = in[m] - in[P - m];
  }
#pragma unroll
  for (int r = 0; r < H; ++r) {
    double so = Q[r * H] * o[0];
    double se = Q[H * H + r * H] * e[0];
#pragma unroll
    for (int m = 1; m < H; ++m) {
      so += Q[r * H + m] * o[m];
      se += Q[H * H + r * H + m] * e[m];
    }
    if constexpr ((N1 & 1) != 0) se += Q[2 * H * H + r] * in[C];
    out[r] = se + so;
    out[P - r] = se - so;
  }
  if constexpr ((N1 & 1) != 0) {
    double sc = Q[2 * H * H + 2 * H] * in[C];
#pragma unroll
    for (int m = 0; m < H; ++m) sc += Q[2 * H * H + H + m] * e[m];
    out[C] = sc;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic block sum: wave shuffles, then wave partials in LDS summed in order.
template <int NT>
__device__ __forceinline__ double block_sum(double v) {
  constexpr int NW = (NT + 63) / 64;
  __shared__ double s_red[NW];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) s_red[wv] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < NW; ++k) s += s_red[k];
  return s;
}

// Assemble one value into a global vector following the colour schedule.
// Returns the value now stored (the assembled one when this column is last).
template <typename T>
__device__ __forceinline__ T scatter(T *y, int64_t idx, T val, uint8_t fl) {
  if (fl & kFirst) {
    y[idx] = val;
    return val;
  }
  T s = y[idx] + val;
  y[idx] = s;
  return s;
}

// ---------------------------------------------------------------------------------------------
// Stiffness apply y = A x (paper Eq. 4), sum-factorised, stored geometric factors.
// ---------------------------------------------------------------------------------------------
template <int P, int DIM, typename T, bool MASK, bool DOT>
__global__ __launch_bounds__(256) void k_apply(const T *__restrict__ x, T *__restrict__ y, const T *__restrict__ G,
                                               const int32_t *__restrict__ eh_nodes, const uint8_t *__restrict__ flags,
                                               const int32_t *__restrict__ cols, int ncols, int nz, int64_t n_s,
                                               double *__restrict__ partial, const int32_t *__restrict__ skip) {
  using S = Sh<P, DIM>;
  constexpr int N1 = S::N1, NH = S::NH, NP = S::NP, NG = S::NG, CPB = S::CPB;
  __shared__ T su[CPB * NP];
  __shared__ T sx[CPB * NP];
  __shared__ T sy[DIM == 3 ? CPB * NP : 1];
  if (skip != nullptr && *skip) return;

  const int lc = threadIdx.x / NH;
  const int t = threadIdx.x - lc * NH;
  const int i = t % N1, j = t / N1;
  const int ci = blockIdx.x * CPB + lc;
  const bool active = ci < ncols;
  const int col = active ? cols[ci] : 0;
  const int hn = active ? eh_nodes[(int64_t)col * NH + t] : 0;
  const uint8_t fl = active ? flags[(int64_t)col * NH + t] : 0;

  T Dri[N1], Drj[N1], Dci[N1], Dcj[N1];
#pragma unroll
  for (int m = 0; m < N1; ++m) {
    Dri[m] = dmat<T>(P, i, m);
    Dci[m] = dmat<T>(P, m, i);
    Drj[m] = dmat<T>(P, j, m);
    Dcj[m] = dmat<T>(P, m, j);
  }
  T *u_c = su + lc * NP;
  T *x_c = sx + lc * NP;
  T *y_c = sy + (DIM == 3 ? lc * NP : 0);

  T ucol[N1];
  T carry = T(0);
  double dot = 0.0;
  ucol[0] = active ? x[hn] : T(0);
  const int64_t e0 = (int64_t)col * nz;
  const int vtop = P * nz;

  for (int l = 0; l < nz; ++l) {
#pragma unroll
    for (int k = 1; k < N1; ++k) ucol[k] = active ? x[(int64_t)(l * P + k) * n_s + hn] : T(0);
#pragma unroll
    for (int k = 0; k < N1; ++k) u_c[k * NH + t] = ucol[k];
    __syncthreads();

    const T *Ge = G + (e0 + l) * (int64_t)(NG * NP);
    T vz[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      T ux = T(0), uy = T(0), uz = T(0);
#pragma unroll
      for (int m = 0; m < N1; ++m) ux += Dri[m] * u_c[k * NH + j * N1 + m];
      if constexpr (DIM == 3) {
#pragma unroll
        for (int m = 0; m < N1; ++m) uy += Drj[m] * u_c[k * NH + m * N1 + i];
      }
#pragma unroll
      for (int m = 0; m < N1; ++m) uz += dmat<T>(P, k, m) * ucol[m];
      const int q = k * NH + t;
      if constexpr (DIM == 3) {
        T g00 = active ? Ge[0 * NP + q] : T(0);
        T g01 = active ? Ge[1 * NP + q] : T(0);
        T g02 = active ? Ge[2 * NP + q] : T(0);
        T g11 = active ? Ge[3 * NP + q] : T(0);
        T g12 = active ? Ge[4 * NP + q] : T(0);
        T g22 = active ? Ge[5 * NP + q] : T(0);
        x_c[q] = g00 * ux + g01 * uy + g02 * uz;
        y_c[q] = g01 * ux + g11 * uy + g12 * uz;
        vz[k] = g02 * ux + g12 * uy + g22 * uz;
      } else {
        T g00 = active ? Ge[0 * NP + q] : T(0);
        T g01 = active ? Ge[1 * NP + q] : T(0);
        T g11 = active ? Ge[2 * NP + q] : T(0);
        x_c[q] = g00 * ux + g01 * uz;
        vz[k] = g01 * ux + g11 * uz;
      }
    }
    __syncthreads();

    T yk[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      T acc = T(0);
#pragma unroll
      for (int m = 0; m < N1; ++m) acc += Dci[m] * x_c[k * NH + j * N1 + m];
      if constexpr (DIM == 3) {
#pragma unroll
        for (int m = 0; m < N1; ++m) acc += Dcj[m] * y_c[k * NH + m * N1 + i];
      }
#pragma unroll
      for (int m = 0; m < N1; ++m) acc += dmat<T>(P, m, k) * vz[m];
      yk[k] = acc;
    }
    yk[0] += carry;
    if (active) {
      const int kend = (l == nz - 1) ? N1 : P;
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        if (k < kend) {
          const int v = l * P + k;
          const int64_t idx = (int64_t)v * n_s + hn;
          T val;
          if (MASK && v == vtop) {
            y[idx] = T(0);
            val = T(0);
          } else {
            val = scatter(y, idx, yk[k], fl);
          }
          if (DOT && (fl & kLast)) dot += (double)ucol[k] * (double)val;
        }
      }
    }
    carry = yk[P];
    ucol[0] = ucol[P];
  }
  if constexpr (DOT) {
    double s = block_sum<S::NT>(dot);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------------------------
// Stiffness apply with the geometric factors recomputed in registers (fused geometry).
// For the extruded sigma-mesh, J = [[J_h, 0], [z_xi, z_eta, z_zeta]] with
//   z_xi = sigma_v H_xi - h_xi,  z_eta = sigma_v H_eta - h_eta,  z_zeta = (ds_l / 2) H,
// H = eta + h, so every factor of G = w det(J) B B^T (B = J^-1) follows from five numbers per
// column node (H, H_xi, h_xi, H_eta, h_eta) and the static horizontal metrics A = J_h^-1,
// det J_h.  G r is evaluated as f B (B^T r), f = w_q det J_h z_zeta.  Same operator as the
// stored-factor kernel; HBM traffic drops to the vectors x and y.
// ---------------------------------------------------------------------------------------------
// Same operator, register-lean schedule: the forward (gradient) loop over the zeta index k
// runs at run time, reading the uniform row D[k][.] through the scalar cache, and scatters the
// zeta part of the transposed contraction, y_zeta[k'] += D[k][k'] v_zeta[k], straight into a
// register line; the backward loop is unrolled.  Live registers: the thread's D rows, its
// vertical line, the y_zeta line and the column geometry.
template <int P, int DIM, typename T, bool MASK, bool DOT>
__global__ __launch_bounds__(256) void k_apply_fused2(const T *__restrict__ x, T *__restrict__ y,
                                                      const T *__restrict__ cg, const T *__restrict__ hmT,
                                                      int64_t hstride, const T *__restrict__ sig,
                                                      const T *__restrict__ half_ds,
                                                      const int32_t *__restrict__ eh_nodes,
                                                      const uint8_t *__restrict__ flags,
                                                      const int32_t *__restrict__ cols, int ncols, int nz, int64_t n_s,
                                                      double *__restrict__ partial, const int32_t *__restrict__ skip) {
  using S = Sh<P, DIM>;
  constexpr int N1 = S::N1, NH = S::NH, NP = S::NP, CPB = S::CPB;
  __shared__ T su[CPB * NP];
  __shared__ T sx[CPB * NP];
  __shared__ T sy[DIM == 3 ? CPB * NP : 1];
  if (skip != nullptr && *skip) return;

  const int lc = threadIdx.x / NH;
  const int t = threadIdx.x - lc * NH;
  const int i = t % N1, j = t / N1;
  const int ci = blockIdx.x * CPB + lc;
  const bool active = ci < ncols;
  const int col = active ? cols[ci] : 0;
  const int hn = active ? eh_nodes[(int64_t)col * NH + t] : 0;
  const uint8_t fl = active ? flags[(int64_t)col * NH + t] : 0;
  const int64_t ho = (int64_t)col * NH + t;

  T H = T(1), Hx = T(0), hx = T(0), Hy = T(0), hy = T(0);
  T A00 = T(1), A01 = T(0), A10 = T(0), A11 = T(1), dJ = T(1);
  if (active) {
    H = cg[0 * hstride + ho];
    Hx = cg[1 * hstride + ho];
    hx = cg[2 * hstride + ho];
    if constexpr (DIM == 3) {
      Hy = cg[3 * hstride + ho];
      hy = cg[4 * hstride + ho];
      A00 = hmT[0 * hstride + ho];
      A01 = hmT[1 * hstride + ho];
      A10 = hmT[2 * hstride + ho];
      A11 = hmT[3 * hstride + ho];
      dJ = hmT[4 * hstride + ho];
    } else {
      A00 = hmT[0 * hstride + ho];
      dJ = hmT[1 * hstride + ho];
    }
  }
  const T wdJ = (T)(DIM == 3 ? wgt(P, i) * wgt(P, j) : wgt(P, i)) * dJ;

  T Dri[N1], Drj[N1], Dci[N1], Dcj[N1];
#pragma unroll
  for (int m = 0; m < N1; ++m) {
    Dri[m] = dmat<T>(P, i, m);
    Dci[m] = dmat<T>(P, m, i);
    if constexpr (DIM == 3) {
      Drj[m] = dmat<T>(P, j, m);
      Dcj[m] = dmat<T>(P, m, j);
    }
  }
  T *u_c = su + lc * NP;
  T *x_c = sx + lc * NP;
  T *y_c = sy + (DIM == 3 ? lc * NP : 0);

  T ucol[N1];
  T carry = T(0);
  double dot = 0.0;
  ucol[0] = active ? x[hn] : T(0);
  const int vtop = P * nz;

  T nxt[N1];
#pragma unroll
  for (int k = 1; k < N1; ++k) nxt[k] = active ? x[(int64_t)k * n_s + hn] : T(0);
  for (int l = 0; l < nz; ++l) {
#pragma unroll
    for (int k = 1; k < N1; ++k) ucol[k] = nxt[k];
#pragma unroll
    for (int k = 0; k < N1; ++k) u_c[k * NH + t] = ucol[k];
    __syncthreads();
    // issue the next layer's loads now; they complete behind this layer's arithmetic
    if (l + 1 < nz) {
#pragma unroll
      for (int k = 1; k < N1; ++k) nxt[k] = active ? x[(int64_t)((l + 1) * P + k) * n_s + hn] : T(0);
    }

    const T zz = half_ds[l] * H;
    const T izz = T(1) / zz;
    const T fl0 = wdJ * zz;
    T yz[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) yz[k] = T(0);
#pragma unroll 1
    for (int k = 0; k < N1; ++k) {
      T ux = T(0), uy = T(0), uz = T(0);
      const T *row = u_c + k * NH;
#pragma unroll
      for (int m = 0; m < N1; ++m) ux += Dri[m] * row[j * N1 + m];
      if constexpr (DIM == 3) {
#pragma unroll
        for (int m = 0; m < N1; ++m) uy += Drj[m] * row[m * N1 + i];
      }
#pragma unroll
      for (int m = 0; m < N1; ++m) uz += dmat<T>(P, k, m) * ucol[m];
      const T sg = sig[l * P + k];
      const T f = (T)wgt(P, k) * fl0;
      const T zx = sg * Hx - hx;
      const int q = k * NH + t;
      T vz;
      if constexpr (DIM == 3) {
        const T zy = sg * Hy - hy;
        const T b2x = -(zx * A00 + zy * A10) * izz;
        const T b2y = -(zx * A01 + zy * A11) * izz;
        const T gx = A00 * ux + A10 * uy + b2x * uz;
        const T gy = A01 * ux + A11 * uy + b2y * uz;
        const T gz = izz * uz;
        x_c[q] = f * (A00 * gx + A01 * gy);
        y_c[q] = f * (A10 * gx + A11 * gy);
        vz = f * (b2x * gx + b2y * gy + izz * gz);
      } else {
        const T b1x = -zx * A00 * izz;
        const T g0 = A00 * ux + b1x * uz;
        const T g1 = izz * uz;
        x_c[q] = f * (A00 * g0);
        vz = f * (b1x * g0 + izz * g1);
      }
#pragma unroll
      for (int k2 = 0; k2 < N1; ++k2) yz[k2] += dmat<T>(P, k, k2) * vz;
    }
    __syncthreads();

    // own u entries are no longer read by other threads: reuse them for the output line
#pragma unroll
    for (int k = 0; k < N1; ++k) u_c[k * NH + t] = yz[k];
#pragma unroll 1
    for (int k = 0; k < N1; ++k) {
      // independent partial sums keep the FP64 FMA chains short
      T a0 = u_c[k * NH + t], a1 = T(0), a2 = T(0), a3 = T(0);
      const T *rx = x_c + k * NH;
#pragma unroll
      for (int m = 0; m < N1; m += 2) {
        a1 += Dci[m] * rx[j * N1 + m];
        if (m + 1 < N1) a2 += Dci[m + 1] * rx[j * N1 + m + 1];
      }
      if constexpr (DIM == 3) {
        const T *ry = y_c + k * NH;
        T b1 = T(0);
#pragma unroll
        for (int m = 0; m < N1; m += 2) {
          a3 += Dcj[m] * ry[m * N1 + i];
          if (m + 1 < N1) b1 += Dcj[m + 1] * ry[(m + 1) * N1 + i];
        }
        a3 += b1;
      }
      u_c[k * NH + t] = (a0 + a1) + (a2 + a3);
    }
    if (active) {
      const int kend = (l == nz - 1) ? N1 : P;
      T yv[N1], old[N1];
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        yv[k] = u_c[k * NH + t];
        old[k] = T(0);
      }
      yv[0] += carry;
      // colour schedule: all read-add-write loads of the line in flight together
      if (!(fl & kFirst)) {
#pragma unroll
        for (int k = 0; k < N1; ++k)
          if (k < kend) old[k] = y[(int64_t)(l * P + k) * n_s + hn];
      }
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        if (k < kend) {
          const int v = l * P + k;
          const T val = (MASK && v == vtop) ? T(0) : yv[k] + old[k];
          y[(int64_t)v * n_s + hn] = val;
          if (DOT && (fl & kLast)) dot += (double)ucol[k] * (double)val;
        }
      }
    }
    carry = u_c[P * NH + t];
    ucol[0] = ucol[P];
  }
  if constexpr (DOT) {
    double s = block_sum<CPB * NH>(dot);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// Same operator (3D), line schedule.  Between barriers a thread owns either its vertical line
// (i, j) or, in the two horizontal phases, the xi-line (j = a, k = b) and the eta-line
// (i = a, k = b) with t = b N1 + a.  Every contraction then runs over compile-time indices, so
// its D entries are wave-uniform scalar operands, and each LDS word read feeds N1 FMAs.
// Phases per layer element (4 barriers):
//   0  line (i,j): store u into both sA and sB; u_zeta in registers
//   1  xi/eta lines: u_xi -> sA, u_eta -> sB, each line in place
//   2  line (i,j): per point g = J^-T grad u, v = w detJ J^-1 g; v_xi, v_eta back into sA, sB
//      in place; zeta part of the transposed contraction into registers
//   3  xi/eta lines: transposed contractions in place in sA, sB
//   4  line (i,j): y = sA + sB + zeta part, assembled into global y under the colour schedule
//
// OWN = false: colour schedule (cols = the colour's columns, read-add-write of shared nodes).
// OWN = true: one launch over all columns (cols unused, column = index); the CPB columns of a
// workgroup form a tile.  At a node shared by several columns of the tile, the others pass their
// values through LDS exchange entries (xch: the entry a column writes, and the up to three its
// representative reads) to the node's representative column, which stores the tile's sum into y
// where the tile owns the node and into its face slot F[v][slot] elsewhere (as does a column
// whose exchange entry did not fit); k_apply_faces then adds the slots to the owners.  Blocks are
// mapped so that each XCD (blocks dispatched round-robin over 8) walks a contiguous range of
// tiles, keeping neighbouring tiles' shared cache lines in the same L2.
template <int P, typename T, bool MASK, bool DOT, bool OWN = false>
__global__ __launch_bounds__(256) void k_apply_lines(const T *__restrict__ x, T *__restrict__ y,
                                                     const T *__restrict__ cg, const T *__restrict__ hmT,
                                                     int64_t hstride, const T *__restrict__ sig,
                                                     const T *__restrict__ half_ds,
                                                     const int32_t *__restrict__ eh_nodes,
                                                     const uint8_t *__restrict__ flags,
                                                     const int32_t *__restrict__ cols, int ncols, int nz, int64_t n_s,
                                                     double *__restrict__ partial, const int32_t *__restrict__ skip,
                                                     T *__restrict__ F = nullptr,
                                                     const int32_t *__restrict__ slot = nullptr,
                                                     int64_t n_slots = 0,
                                                     const int16_t *__restrict__ xch = nullptr) {
  using S = Sh<P, 3>;
  constexpr int N1 = S::N1, NH = S::NH, NP = S::NP, CPB = S::CPB;
  constexpr int XM = CPB * NH / 2;   // exchange entries per tile (the host's tile_xmax)
  // sA holds the xi-lines (planes of NH, line stride N1: lane t reads from 7t, conflict-free);
  // sB the eta-lines with the plane stride padded to SB = N1 (mod 64), so that lane t = b N1 + a
  // of the eta-line (i = a, k = b) starts at b SB + a = t (mod 64) and a wave's loads fall in
  // distinct banks (degrees < 4: N1 mod 16, to bound the LDS of their many columns per block)
  constexpr int SBM = P >= 4 ? 64 : 16;
  constexpr int SB = NH + (((N1 - NH) % SBM) + SBM) % SBM;
  constexpr int NPB = N1 * SB;
  __shared__ T sA[CPB * NP];
  __shared__ T sB[CPB * NPB];
  __shared__ T sX[OWN ? N1 * XM : 1];
  if (skip != nullptr && *skip) return;

  const int lc = threadIdx.x / NH;
  const int t = threadIdx.x - lc * NH;
  const int i = t % N1, j = t / N1;
  int blk = blockIdx.x;
  if constexpr (OWN) {
    const int nb = gridDim.x, q = nb >> 3, r = nb & 7, xc = blk & 7;
    blk = (xc < r ? xc * (q + 1) : r * (q + 1) + (xc - r) * q) + (blk >> 3);
  }
  const int ci = blk * CPB + lc;
  const bool active = ci < ncols;
  const int col = active ? (OWN ? ci : cols[ci]) : 0;
  const int hn = active ? eh_nodes[(int64_t)col * NH + t] : 0;
  const uint8_t fl = active ? flags[(int64_t)col * NH + t] : 0;
  const int64_t ho = (int64_t)col * NH + t;

  T H = T(1), Hx = T(0), hx = T(0), Hy = T(0), hy = T(0);
  T A00 = T(1), A01 = T(0), A10 = T(0), A11 = T(1), dJ = T(1);
  if (active) {
    H = cg[0 * hstride + ho];
    Hx = cg[1 * hstride + ho];
    hx = cg[2 * hstride + ho];
    Hy = cg[3 * hstride + ho];
    hy = cg[4 * hstride + ho];
    A00 = hmT[0 * hstride + ho];
    A01 = hmT[1 * hstride + ho];
    A10 = hmT[2 * hstride + ho];
    A11 = hmT[3 * hstride + ho];
    dJ = hmT[4 * hstride + ho];
  }
  const T wdJ = (T)(wgt(P, i) * wgt(P, j)) * dJ;

  T *Ab = sA + lc * NP;
  T *Bb = sB + lc * NPB;
  // the thread's lines in the horizontal phases: xi-line (j = a, k = b), eta-line (i = a, k = b)
  const int xi_base = t * N1;                       // b NH + a N1
  const int eta_base = (t / N1) * SB + (t % N1);    // b SB + a, stride N1
  // node (v, hn) at byte offset v n_s sizeof(T) (uniform) + hn sizeof(T) (per thread); the
  // launcher guarantees that n_v sizeof(T) fits in 32 bits
  const uint32_t nbytes = (uint32_t)((int64_t)(P * nz + 1) * n_s * (int64_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t rx = vec_rsrc(x, nbytes), ry = vec_rsrc(y, nbytes);
  const uint32_t hb = (uint32_t)hn * (uint32_t)sizeof(T);
  const uint32_t rowb = (uint32_t)n_s * (uint32_t)sizeof(T);
  // face slots (OWN): [p nz + 1][n_slots]
  __amdgpu_buffer_rsrc_t rf = ry;
  uint32_t fb = 0, rowf = 0, fbytes = 0;
  bool has_slot = false;
  int xw = -1, xr0 = -1, xr1 = -1, xr2 = -1;
  if constexpr (OWN) {
    fbytes = (uint32_t)((int64_t)(P * nz + 1) * n_slots * (int64_t)sizeof(T));
    rf = vec_rsrc(F, fbytes);
    const int32_t sl = active ? slot[ho] : -1;
    has_slot = sl >= 0;
    fb = (uint32_t)(sl < 0 ? 0 : sl) * (uint32_t)sizeof(T);
    rowf = (uint32_t)n_slots * (uint32_t)sizeof(T);
    if (active) {
      xw = xch[ho * 4];
      xr0 = xch[ho * 4 + 1];
      xr1 = xch[ho * 4 + 2];
      xr2 = xch[ho * 4 + 3];
    }
  }

  T ucol[N1];
  T carry = T(0);
  double dot = 0.0;
  ucol[0] = active ? buf_ld<T>(rx, hb, 0) : T(0);
  const int vtop = P * nz;
  T nxt[N1];
#pragma unroll
  for (int k = 1; k < N1; ++k) nxt[k] = active ? buf_ld<T>(rx, hb, (uint32_t)k * rowb) : T(0);

  for (int l = 0; l < nz; ++l) {
    // FP64 up to degree 7: the row strides pass through an opaque copy per layer, so that the
    // level offsets below are formed by scalar arithmetic where they are used (kept live across
    // the loop, one per level, they spilled from scalar to vector registers; FP32 has the scalar
    // registers for them, and at degree 8 the even-odd tables leave too few either way)
    constexpr bool kRemat = sizeof(T) == 8 && P <= 7;
    uint32_t rb = rowb, rfs = rowf;
    if constexpr (kRemat) asm volatile("" : "+s"(rb), "+s"(rfs));
    // phase 0
#pragma unroll
    for (int k = 1; k < N1; ++k) ucol[k] = nxt[k];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      Ab[k * NH + t] = ucol[k];
      Bb[k * SB + t] = ucol[k];
    }
    T uz[N1];
    const T *E0 = eo_ptr<P, T, 0>(ucol[0]);
    line_eo<P, T>(ucol, uz, E0);
    __syncthreads();
    // next layer's x loads complete behind this layer's arithmetic
    if (l + 1 < nz) {
#pragma unroll
      for (int k = 1; k < N1; ++k) nxt[k] = active ? buf_ld<T>(rx, hb, (uint32_t)((l + 1) * P + k) * rb) : T(0);
    }

    // phase 1 (in place: each line is read and written by its one thread)
    {
      T in[N1], out[N1];
#pragma unroll
      for (int m = 0; m < N1; ++m) in[m] = Ab[xi_base + m];
      line_eo<P, T>(in, out, E0);
#pragma unroll
      for (int r = 0; r < N1; ++r) Ab[xi_base + r] = out[r];
#pragma unroll
      for (int m = 0; m < N1; ++m) in[m] = Bb[eta_base + m * N1];
      line_eo<P, T>(in, out, E0);
#pragma unroll
      for (int r = 0; r < N1; ++r) Bb[eta_base + r * N1] = out[r];
    }
    __syncthreads();

    // phase 2
    const T zz = half_ds[l] * H;
    const T izz = T(1) / zz;
    const T fl0 = wdJ * zz;
    // the horizontal part of J^-T grad u picks up b2 = -(J_h^-T grad z) / z_zeta, and
    // grad z = sigma grad H - grad h is linear in sigma along the line: b2 = sigma a + b
    const T ax = -(Hx * A00 + Hy * A10) * izz, bx = (hx * A00 + hy * A10) * izz;
    const T ay = -(Hx * A01 + Hy * A11) * izz, by = (hx * A01 + hy * A11) * izz;
    const T izz2 = izz * izz;
    T vz[N1], yz[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      const int q = k * NH + t, qb = k * SB + t;
      const T ux = Ab[q], uy = Bb[qb];
      const T sg = sig[l * P + k];
      const T f = (T)wgt(P, k) * fl0;
      const T b2x = sg * ax + bx;
      const T b2y = sg * ay + by;
      const T gx = A00 * ux + A10 * uy + b2x * uz[k];
      const T gy = A01 * ux + A11 * uy + b2y * uz[k];
      Ab[q] = f * (A00 * gx + A01 * gy);
      Bb[qb] = f * (A10 * gx + A11 * gy);
      vz[k] = f * (b2x * gx + b2y * gy + izz2 * uz[k]);
    }
    const T *E1 = eo_ptr<P, T, 1>(vz[0]);
    line_eo<P, T>(vz, yz, E1);
    __syncthreads();

    // phase 3 (in place: only this thread touches these lines now)
    {
      T in[N1], out[N1];
#pragma unroll
      for (int m = 0; m < N1; ++m) in[m] = Ab[xi_base + m];
      line_eo<P, T>(in, out, E1);
#pragma unroll
      for (int r = 0; r < N1; ++r) Ab[xi_base + r] = out[r];
#pragma unroll
      for (int m = 0; m < N1; ++m) in[m] = Bb[eta_base + m * N1];
      line_eo<P, T>(in, out, E1);
#pragma unroll
      for (int r = 0; r < N1; ++r) Bb[eta_base + r * N1] = out[r];
    }
    // read-add-write loads of the colour schedule, in flight across the barrier
    const int kend = (l == nz - 1) ? N1 : P;
    T old[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) old[k] = T(0);
    if (!OWN && active && !(fl & kFirst)) {
#pragma unroll
      for (int k = 0; k < N1; ++k)
        if (k < kend) old[k] = buf_ld<T>(ry, hb, (uint32_t)(l * P + k) * rb);
    }
    __syncthreads();

    // phase 4
    T yv[N1];
#pragma unroll
    for (int k = 0; k < N1; ++k) yv[k] = yz[k] + (Ab[k * NH + t] + Bb[k * SB + t]);
    yv[0] += carry;
    carry = yv[P];
    if constexpr (OWN) {
      // tile assembly: the tile's other columns at a shared node hand their values (this
      // layer's stored levels) to the node's representative
      if (xw >= 0) {
#pragma unroll
        for (int k = 0; k < N1; ++k)
          if (k < kend) sX[k * XM + xw] = yv[k];
      }
      __syncthreads();
      if (active && (fl & kTRep)) {
#pragma unroll
        for (int k = 0; k < N1; ++k) {
          if (k < kend) {
            T a = yv[k];
            if (xr0 >= 0) a += sX[k * XM + xr0];
            if (xr1 >= 0) a += sX[k * XM + xr1];
            if (xr2 >= 0) a += sX[k * XM + xr2];
            yv[k] = a;
          }
        }
      }
      if (active && ((fl & kTRep) || has_slot)) {
        // the same for the stores' descriptors: formed here from opaque copies of the pointers,
        // so that they are not held (and spilled) across the layer loop
        T *yo = y, *fo = F;
        if constexpr (kRemat) asm volatile("" : "+s"(yo), "+s"(fo));
        const __amdgpu_buffer_rsrc_t rys = vec_rsrc(yo, nbytes), rfo = vec_rsrc(fo, fbytes);
#pragma unroll
        for (int k = 0; k < N1; ++k) {
          if (k < kend) {
            const int v = l * P + k;
            if (fl & kTOwn) {
              const T val = (MASK && v == vtop) ? T(0) : yv[k];
              buf_st(val, rys, hb, (uint32_t)v * rb);
              if (DOT && !(fl & kTShared)) dot += (double)ucol[k] * (double)val;
            } else if (!(MASK && v == vtop)) {
              buf_st(yv[k], rfo, fb, (uint32_t)v * rfs);
            }
          }
        }
      }
    } else if (active) {
#pragma unroll
      for (int k = 0; k < N1; ++k) {
        if (k < kend) {
          const int v = l * P + k;
          const T val = (MASK && v == vtop) ? T(0) : yv[k] + old[k];
          buf_st(val, ry, hb, (uint32_t)v * rb);
          if (DOT && (fl & kLast)) dot += (double)ucol[k] * (double)val;
        }
      }
    }
    ucol[0] = ucol[P];
  }
  if constexpr (DOT) {
    double s = block_sum<CPB * NH>(dot);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// Second pass of the owner-computes apply: y[v][n] += sum of the face slots of the other
// columns at shared node n (slots in increasing column order), for every node level v; the
// dot-product contribution x.y of the shared nodes is taken here.  A thread takes one shared
// node and a chunk of kFaceLevels levels, with all its loads issued before the sums.  Blocks
// are remapped so that each XCD walks a contiguous range of nodes of one level chunk (the slots
// of neighbouring columns then meet in the same L2).
constexpr int kFaceLevels = 8;

template <typename T, bool MASK, bool DOT>
__global__ __launch_bounds__(256) void k_apply_faces(const T *__restrict__ x, T *__restrict__ y,
                                                     const T *__restrict__ F, const int32_t *__restrict__ ps_node,
                                                     const int32_t *__restrict__ ps_ptr,
                                                     const int32_t *__restrict__ ps_slot, int n_ps, int nlev,
                                                     int64_t n_s, int64_t n_slots, double *__restrict__ partial,
                                                     const int32_t *__restrict__ skip) {
  if (skip != nullptr && *skip) return;
  constexpr int LC = kFaceLevels;
  int blk = blockIdx.x;
  {
    const int nb = gridDim.x, q = nb >> 3, r = nb & 7, xc = blk & 7;
    blk = (xc < r ? xc * (q + 1) : r * (q + 1) + (xc - r) * q) + (blk >> 3);
  }
  const int nbx = (n_ps + 255) >> 8;
  const int chunk = blk / nbx;
  const int k = (blk - chunk * nbx) * 256 + threadIdx.x;
  const int v0 = chunk * LC;
  const int vend = MASK ? nlev - 1 : nlev;   // the masked top level stays 0
  double dot = 0.0;
  if (k < n_ps) {
    const int64_t n = ps_node[k];
    const int a = ps_ptr[k], b = ps_ptr[k + 1];
    T acc[LC];
#pragma unroll
    for (int u = 0; u < LC; ++u) acc[u] = (v0 + u < vend) ? y[(v0 + u) * n_s + n] : T(0);
    for (int q = a; q < b; ++q) {
      const int64_t sl = ps_slot[q];
      T f[LC];
#pragma unroll
      for (int u = 0; u < LC; ++u) f[u] = (v0 + u < vend) ? F[(v0 + u) * n_slots + sl] : T(0);
#pragma unroll
      for (int u = 0; u < LC; ++u) acc[u] += f[u];
    }
    T xv[LC];
    if constexpr (DOT) {
#pragma unroll
      for (int u = 0; u < LC; ++u) xv[u] = (v0 + u < vend) ? x[(v0 + u) * n_s + n] : T(0);
    }
#pragma unroll
    for (int u = 0; u < LC; ++u) {
      if (v0 + u < vend) {
        y[(v0 + u) * n_s + n] = acc[u];
        if (DOT) dot += (double)xv[u] * (double)acc[u];
      }
    }
  }
  if constexpr (DOT) {
    double s = block_sum<256>(dot);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

bool owner_apply_active(const Ctx &c) {
  if (c.dim != 3 || c.apply_variant != 0 || !c.apply_owner) return false;
  const int64_t lim = int64_t(1) << 32;
  return c.n_v * 8 < lim && (int64_t)(c.p * c.nz + 1) * std::max(c.n_slots, c.n_tslots) * 8 < lim;
}

// blocks of a face pass over n nodes with face slots
static int face_blocks_n(const Ctx &c, int n) {
  return ((n + 255) / 256) * ((c.p * c.nz + 1 + kFaceLevels - 1) / kFaceLevels);
}
static int face_blocks(const Ctx &c) { return face_blocks_n(c, c.n_ps); }

// the face pass alone (k_apply_faces without the dot product): y at the shared nodes += the face
// slots of the context's F buffer of y's precision
hipError_t launch_faces(Ctx &c, fnpf_dtype dt, void *y, bool mask, hipStream_t s, const int32_t *skip) {
  if (c.n_ps == 0) return hipSuccess;
  const int nb = face_blocks(c);
  const int nlev = c.p * c.nz + 1;
  if (dt == FNPF_F64) {
    if (mask)
      k_apply_faces<double, true, false><<<nb, 256, 0, s>>>(nullptr, (double *)y, c.d_F64, c.d_ps_node, c.d_ps_ptr,
                                                            c.d_ps_slot, c.n_ps, nlev, c.n_s, c.n_slots, nullptr,
                                                            skip);
    else
      k_apply_faces<double, false, false><<<nb, 256, 0, s>>>(nullptr, (double *)y, c.d_F64, c.d_ps_node,
                                                             c.d_ps_ptr, c.d_ps_slot, c.n_ps, nlev, c.n_s,
                                                             c.n_slots, nullptr, skip);
  } else {
    if (mask)
      k_apply_faces<float, true, false><<<nb, 256, 0, s>>>(nullptr, (float *)y, c.d_F32, c.d_ps_node, c.d_ps_ptr,
                                                           c.d_ps_slot, c.n_ps, nlev, c.n_s, c.n_slots, nullptr,
                                                           skip);
    else
      k_apply_faces<float, false, false><<<nb, 256, 0, s>>>(nullptr, (float *)y, c.d_F32, c.d_ps_node, c.d_ps_ptr,
                                                            c.d_ps_slot, c.n_ps, nlev, c.n_s, c.n_slots, nullptr,
                                                            skip);
  }
  return hipGetLastError();
}

int owner_apply_blocks(const Ctx &c) {
  if (c.dim != 3) return 0;
  const int cpb = 256 / c.nh;
  return (c.n_eh + cpb - 1) / cpb + face_blocks_n(c, c.n_tps);
}

// ---------------------------------------------------------------------------------------------
// Geometry (paper Sec. 3.1.2, Step 4.1): z = -h + sigma_v (eta + h) per node level; per point
// G = w det(J) J^-1 J^-T with J = [[J_h, 0], [z_xi, z_eta, z_zeta]]; assembled Jacobi diagonal.
// ---------------------------------------------------------------------------------------------
//
// OWN = false: colour schedule over the columns of one colour (cols), the diagonal assembled by
// read-add-write.  OWN = true (3D): one launch over all columns, the CPB columns of a workgroup a
// tile as in the owner-computes apply: the tile's columns pass their diagonal contributions at
// shared nodes to the node's representative through LDS exchange entries (xch), which stores the
// inverses (and the diagonal if kept) where no other tile contributes and otherwise writes its
// tile's sum to its place in the geometry's face layout (slot, n_slots entries per level);
// k_diag_faces completes the nodes with face slots.  SG: also store the per-point factors
// (G64, G32) for the stored-factor apply; without them the off-diagonal factors are dead code and
// the kernel needs about two thirds of the registers.
template <int P, int DIM, bool OWN = false, bool SG = true>
__global__ __launch_bounds__(256) void k_geom(const double *__restrict__ eta, const double *__restrict__ hb,
                                              const double *__restrict__ hm, int64_t hstride,
                                              const int32_t *__restrict__ eh_nodes, const uint8_t *__restrict__ flags,
                                              const int32_t *__restrict__ cols, int ncols, int nz, int64_t n_s,
                                              const double *__restrict__ sigma, const double *__restrict__ layer_s,
                                              double *__restrict__ G64, float *__restrict__ G32,
                                              double *__restrict__ diag, double *__restrict__ dinv,
                                              float *__restrict__ dinv32, double *__restrict__ Hout,
                                              double *__restrict__ hout, double *__restrict__ cg64,
                                              float *__restrict__ cg32, int h_is_total, int32_t *__restrict__ err,
                                              double *__restrict__ F = nullptr,
                                              const int32_t *__restrict__ slot = nullptr, int64_t n_slots = 0,
                                              const int16_t *__restrict__ xch = nullptr, int full_diag = 1) {
  using S = Sh<P, DIM>;
  constexpr int N1 = S::N1, NH = S::NH, NP = S::NP, NG = S::NG, CPB = S::CPB;
  constexpr int XM = CPB * NH / 2;   // exchange entries per tile (the host's tile_xmax)
  // The diagonal at node (i, j, k) of an element, collocated quadrature:
  //   sum_m D[m][i]^2 G_xx(m, j, k) + sum_m D[m][j]^2 G_yy(i, m, k) + sum_m D[m][k]^2 G_zz(i, j, m)
  //   + 2 (D_ii D_jj G_xy + D_ii D_kk G_xz + D_jj D_kk G_yz)(i, j, k).
  // sA holds G_xx at the element's points (plane k, row j, entry i at k NH + j N1 + i) and then, in
  // place, its xi-line sums; sB the same for G_yy along eta-lines; the zeta sums use the thread's
  // own vertical line in registers.  sX: the partners' values at shared nodes (OWN) and, before
  // the layer loop, the surface H and h of the block's columns.
  constexpr int NX0 = 2 * CPB * NH, NX1 = OWN ? N1 * XM : 0;
  // sB's plane stride padded as the apply's eta-line array: SB = N1 (mod 64), so the 64 lanes of
  // a wave reading their eta-lines start in distinct banks (degrees < 4: N1 mod 16)
  constexpr int SBM = P >= 4 ? 64 : 16;
  constexpr int SB = DIM == 3 ? NH + (((N1 - NH) % SBM) + SBM) % SBM : NH;
  __shared__ double sA[CPB * NP];
  __shared__ double sB[DIM == 3 ? CPB * N1 * SB : 1];
  __shared__ double sX[NX0 > NX1 ? NX0 : NX1];
  double *sH = sX, *sh = sX + CPB * NH;

  const int lc = threadIdx.x / NH;
  const int t = threadIdx.x - lc * NH;
  const int i = t % N1, j = t / N1;
  int blk = blockIdx.x;
  if constexpr (OWN) {
    const int nb = gridDim.x, q = nb >> 3, r = nb & 7, xc = blk & 7;
    blk = (xc < r ? xc * (q + 1) : r * (q + 1) + (xc - r) * q) + (blk >> 3);
  }
  const int ci = blk * CPB + lc;
  const bool active = ci < ncols;
  const int col = active ? (OWN ? ci : cols[ci]) : 0;
  const int hn = active ? eh_nodes[(int64_t)col * NH + t] : 0;
  const uint8_t fl = active ? flags[(int64_t)col * NH + t] : 0;
  const int64_t ho = (int64_t)col * NH + t;
  int xw = -1, xr0 = -1, xr1 = -1, xr2 = -1;
  int32_t sl = -1;
  if (OWN && active) {
    xw = xch[ho * 4];
    xr0 = xch[ho * 4 + 1];
    xr1 = xch[ho * 4 + 2];
    xr2 = xch[ho * 4 + 3];
    sl = slot[ho];
  }
  const bool stores = OWN && active && ((fl & kTRep) || sl >= 0);
  // OWN stores through raw buffer descriptors with 32-bit byte offsets (the launcher checks that
  // the level rows of diag and of the face layout fit): where its tile owns a node that no other
  // tile touches, a storing thread writes the inverses (and the diagonal if the whole diagonal is
  // kept); elsewhere it writes its tile's value to its place sl in the geometry's face layout (the
  // owner's place where its tile owns the node), from which k_diag_faces completes the node
  constexpr int kSmStore = 1, kSmDiag = 2, kSmInv = 4, kSmSlot = 8, kSmX0 = 16, kSmX1 = 32, kSmX2 = 64;
  const bool own_only = (fl & kTOwn) && !(fl & kTShared);
  const int smode = !stores ? 0
                            : kSmStore | (own_only && full_diag ? kSmDiag : 0) | (own_only ? kSmInv : 0) |
                                  (!own_only ? kSmSlot : 0) | (xr0 >= 0 ? kSmX0 : 0) | (xr1 >= 0 ? kSmX1 : 0) |
                                  (xr2 >= 0 ? kSmX2 : 0);
  const int xc0 = xr0 < 0 ? 0 : xr0, xc1 = xr1 < 0 ? 0 : xr1, xc2 = xr2 < 0 ? 0 : xr2;
  const uint32_t row8 = (uint32_t)n_s * 8u, rowF8 = (uint32_t)n_slots * 8u;
  const uint32_t hb8 = (uint32_t)hn * 8u, fb8 = (uint32_t)(sl < 0 ? 0 : sl) * 8u;
  const uint32_t nlv = (uint32_t)(P * nz + 1);
  const __amdgpu_buffer_rsrc_t r_diag = vec_rsrc(diag, OWN ? nlv * row8 : 0u);
  const __amdgpu_buffer_rsrc_t r_dinv = vec_rsrc(dinv, OWN ? nlv * row8 : 0u);
  const __amdgpu_buffer_rsrc_t r_dinv32 = vec_rsrc(dinv32, OWN ? nlv * (row8 >> 1) : 0u);
  const __amdgpu_buffer_rsrc_t r_F = vec_rsrc(F, OWN ? nlv * rowF8 : 0u);

  const double Hn = active ? (h_is_total ? eta[hn] : eta[hn] + hb[hn]) : 1.0;
  const double hnv = active ? hb[hn] : 0.0;
  if (active && !(Hn > 0.0)) *err = 1;
  if (active && (fl & (OWN ? kOwned : kFirst))) {
    Hout[hn] = Hn;
    hout[hn] = hnv;
  }
  sH[lc * NH + t] = Hn;
  sh[lc * NH + t] = hnv;
  __syncthreads();
  double Hx = 0.0, hx = 0.0, Hy = 0.0, hy = 0.0;
#pragma unroll
  for (int m = 0; m < N1; ++m) {
    Hx += dmat<double>(P, i, m) * sH[lc * NH + j * N1 + m];
    hx += dmat<double>(P, i, m) * sh[lc * NH + j * N1 + m];
  }
  if constexpr (DIM == 3) {
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      Hy += dmat<double>(P, j, m) * sH[lc * NH + m * N1 + i];
      hy += dmat<double>(P, j, m) * sh[lc * NH + m * N1 + i];
    }
  }
  // per (column, node) vertical data used by the fused-geometry apply
  if (active) {
    cg64[0 * hstride + ho] = Hn;
    cg64[1 * hstride + ho] = Hx;
    cg64[2 * hstride + ho] = hx;
    if (cg32) {
      cg32[0 * hstride + ho] = (float)Hn;
      cg32[1 * hstride + ho] = (float)Hx;
      cg32[2 * hstride + ho] = (float)hx;
    }
    if constexpr (DIM == 3) {
      cg64[3 * hstride + ho] = Hy;
      cg64[4 * hstride + ho] = hy;
      if (cg32) {
        cg32[3 * hstride + ho] = (float)Hy;
        cg32[4 * hstride + ho] = (float)hy;
      }
    }
  }
  double A00, A01 = 0.0, A10 = 0.0, A11 = 0.0, detJh;
  if constexpr (DIM == 3) {
    A00 = active ? hm[0 * hstride + ho] : 1.0;
    A01 = active ? hm[1 * hstride + ho] : 0.0;
    A10 = active ? hm[2 * hstride + ho] : 0.0;
    A11 = active ? hm[3 * hstride + ho] : 1.0;
    detJh = active ? hm[4 * hstride + ho] : 1.0;
  } else {
    A00 = active ? hm[0 * hstride + ho] : 1.0;
    detJh = active ? hm[1 * hstride + ho] : 1.0;
  }
  const double wh = DIM == 3 ? wgt(P, i) * wgt(P, j) : wgt(P, i);
  const double Dii = dmat<double>(P, i, i), Djj = DIM == 3 ? dmat<double>(P, j, j) : 0.0;
  double *Ab = sA + lc * NP;
  double *Bb = sB + (DIM == 3 ? lc * N1 * SB : 0);

  // 3D: the horizontal part of J^-T grad(.) picks up b2 = -(J_h^-T grad z) / z_zeta, and
  // grad z = sigma grad H - grad h is linear in sigma along the line: b2 = (sigma a0 + b0) / z_zeta
  // with a0, b0 per column node; the products of A in the factors are per column node as well
  const double ax0 = -(Hx * A00 + Hy * A10), bx0 = hx * A00 + hy * A10;
  const double ay0 = -(Hx * A01 + Hy * A11), by0 = hx * A01 + hy * A11;
  const double c00 = A00 * A00 + A01 * A01, c11 = A10 * A10 + A11 * A11, c01 = A00 * A10 + A01 * A11;
  const double whd = wh * detJh;

  double carry = 0.0;
  const int64_t e0 = (int64_t)col * nz;
  for (int l = 0; l < nz; ++l) {
    const double zz = 0.5 * (layer_s[l + 1] - layer_s[l]) * Hn;   // z_zeta (sigma-linear per layer)
    const double izz = 1.0 / zz;
    const double ax = ax0 * izz, bx = bx0 * izz, ay = ay0 * izz, by = by0 * izz, izz2 = izz * izz;
    const double fzl = whd * zz;   // the point's factor w_i w_j w_k det J is w_k fzl
    double gz[N1];
    double *Ge64 = G64 ? G64 + (e0 + l) * (int64_t)(NG * NP) : nullptr;
    float *Ge32 = G32 ? G32 + (e0 + l) * (int64_t)(NG * NP) : nullptr;
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      const double sg = sigma[l * P + k];
      const int q = k * NH + t;
      if constexpr (DIM == 3) {
        const double f = wgt(P, k) * fzl;
        const double b2x = sg * ax + bx;
        const double b2y = sg * ay + by;
        const double g00 = f * c00;
        const double g11 = f * c11;
        const double g22 = f * (b2x * b2x + b2y * b2y + izz2);
        if (SG && active && Ge64) {
          const double g01 = f * c01;
          const double g02 = f * (A00 * b2x + A01 * b2y);
          const double g12 = f * (A10 * b2x + A11 * b2y);
          Ge64[0 * NP + q] = g00;
          Ge64[1 * NP + q] = g01;
          Ge64[2 * NP + q] = g02;
          Ge64[3 * NP + q] = g11;
          Ge64[4 * NP + q] = g12;
          Ge64[5 * NP + q] = g22;
          if (Ge32) {
            Ge32[0 * NP + q] = (float)g00;
            Ge32[1 * NP + q] = (float)g01;
            Ge32[2 * NP + q] = (float)g02;
            Ge32[3 * NP + q] = (float)g11;
            Ge32[4 * NP + q] = (float)g12;
            Ge32[5 * NP + q] = (float)g22;
          }
        }
        Ab[q] = g00;
        Bb[k * SB + t] = g11;
        gz[k] = g22;
      } else {
        const double zx = -hx + sg * Hx;
        const double f = wh * wgt(P, k) * detJh * zz;
        const double b1x = -zx * A00 * izz;
        const double b1z = izz;
        const double g00 = f * A00 * A00;
        const double g11 = f * (b1x * b1x + b1z * b1z);
        if (SG && active && Ge64) {
          const double g01 = f * A00 * b1x;
          Ge64[0 * NP + q] = g00;
          Ge64[1 * NP + q] = g01;
          Ge64[2 * NP + q] = g11;
          if (Ge32) {
            Ge32[0 * NP + q] = (float)g00;
            Ge32[1 * NP + q] = (float)g01;
            Ge32[2 * NP + q] = (float)g11;
          }
        }
        Ab[q] = g00;
        gz[k] = g11;
      }
    }
    __syncthreads();
    // line sums in place: the thread's xi-line (j = a, k = b) and, in 3D, eta-line (i = a,
    // k = b), t = b N1 + a; out_r = sum_m D[m][r]^2 in_m (even-odd form up to degree 6)
    {
      auto line_sum = [&](const double(&in)[N1], double(&out)[N1]) {
        if constexpr (P <= 6) {
          line_sq_eo<P>(in, out, sqeo_ptr(P, in[0]));
        } else {
          const double *Q = dsq_ptr(P, in[0]);
#pragma unroll
          for (int r = 0; r < N1; ++r) {
            double a = 0.0;
#pragma unroll
            for (int m = 0; m < N1; ++m) a += Q[m * N1 + r] * in[m];
            out[r] = a;
          }
        }
      };
      double in[N1], out[N1];
#pragma unroll
      for (int m = 0; m < N1; ++m) in[m] = Ab[t * N1 + m];
      line_sum(in, out);
#pragma unroll
      for (int r = 0; r < N1; ++r) Ab[t * N1 + r] = out[r];
      if constexpr (DIM == 3) {
        const int eb = (t / N1) * SB + t % N1;
#pragma unroll
        for (int m = 0; m < N1; ++m) in[m] = Bb[eb + m * N1];
        line_sum(in, out);
#pragma unroll
        for (int r = 0; r < N1; ++r) Bb[eb + r * N1] = out[r];
      }
    }
    __syncthreads();
    // the node's diagonal at each level of the layer element, one level at a time; the node's own
    // entry of sA (read here by this thread only) then holds its value for the tile assembly
    const int kh = (l == nz - 1) ? N1 : P;   // levels stored by this layer (the top one by the next)
    double top = 0.0;
#pragma unroll 1
    for (int k = 0; k < N1; ++k) {
      double d = Ab[k * NH + t];
      if constexpr (DIM == 3) d += Bb[k * SB + t];
      const double *Qk = dsq_ptr(P, d) + k;
#pragma unroll
      for (int m = 0; m < N1; ++m) d += Qk[m * N1] * gz[m];
      const double Dkk = dmat<double>(P, k, k);
      const double sg = sigma[l * P + k];
      if constexpr (DIM == 3) {
        const double f = wgt(P, k) * fzl;
        const double f01 = f * c01;
        if (Dkk != 0.0) {   // uniform: D_kk vanishes except at the element's bottom and top levels
          const double b2x = sg * ax + bx;
          const double b2y = sg * ay + by;
          const double f02 = f * (A00 * b2x + A01 * b2y);
          const double f12 = f * (A10 * b2x + A11 * b2y);
          d += 2.0 * (Dii * Djj * f01 + Dii * Dkk * f02 + Djj * Dkk * f12);
        } else {
          d += 2.0 * (Dii * Djj * f01);
        }
      } else {
        const double zx = -hx + sg * Hx;
        const double f = wh * wgt(P, k) * detJh * zz;
        const double b1x = -zx * A00 * izz;
        const double c01 = f * A00 * b1x;
        d += 2.0 * Dii * Dkk * c01;
      }
      if (k == 0) d += carry;
      if (k == P) top = d;
      if (k < kh) {
        if constexpr (OWN) {
          if (xw >= 0)
            sX[k * XM + xw] = d;
          else
            Ab[k * NH + t] = d;
        } else if (active) {
          const int v = l * P + k;
          const int64_t idx = (int64_t)v * n_s + hn;
          const double val = scatter(diag, idx, d, fl);
          if (fl & kLast) {
            const double di = (v == P * nz) ? 0.0 : recip(val);
            dinv[idx] = di;
            if (dinv32) dinv32[idx] = (float)di;
          }
        }
      }
    }
    carry = top;
    if constexpr (OWN) {
      __syncthreads();
      // representatives add their partners' values and store (the next writes to sX follow the
      // next layer's first barrier; sA's own entries are rewritten by this thread only)
      // the per-thread conditions are re-derived here from one opaque word, so the compiler does
      // not keep a 64-bit lane mask per condition live across the layer loop (which spilled
      // scalar registers to vector lanes)
      int sm = smode;
      asm volatile("" : "+v"(sm));
      if (sm & kSmStore) {
#pragma unroll
        for (int k = 0; k < N1; ++k) {
          if (k < kh) {
            // partners' entries read unconditionally at clamped (valid) places, then selected
            const double p0 = sX[k * XM + xc0], p1 = sX[k * XM + xc1], p2 = sX[k * XM + xc2];
            double a = Ab[k * NH + t];
            a += (sm & kSmX0) ? p0 : 0.0;
            a += (sm & kSmX1) ? p1 : 0.0;
            a += (sm & kSmX2) ? p2 : 0.0;
            const uint32_t v = (uint32_t)(l * P + k);
            if (sm & kSmDiag) buf_st(a, r_diag, hb8, v * row8);
            if (sm & kSmInv) {
              const double di = (v == (uint32_t)(P * nz)) ? 0.0 : recip(a);
              buf_st(di, r_dinv, hb8, v * row8);
              if (dinv32) buf_st((float)di, r_dinv32, hb8 >> 1, v * (row8 >> 1));
            }
            if (sm & kSmSlot) buf_st(a, r_F, fb8, v * rowF8);
          }
        }
      }
    }
  }
}

// Face pass of the owner-computes geometry: at the k-th node with face slots (node[k]), the
// diagonal is the owner tile's value (F at k) plus the node's first slot (F at n_tps + k) plus its
// further slots (F at xslot[xptr[k]..xptr[k+1]), in increasing slot order); the inverses are
// stored there (0 on the top level), and the sum itself only when the whole diagonal is kept.
// F's level rows have n_g entries.  The two leading reads follow the thread index, so they are
// issued at once with the node index.  Same thread layout as k_apply_faces: a thread takes one node
// and a chunk of kFaceLevels levels, and each XCD walks a contiguous range of nodes.
__global__ __launch_bounds__(256) void k_diag_faces(double *__restrict__ diag, double *__restrict__ dinv,
                                                    float *__restrict__ dinv32, const double *__restrict__ F,
                                                    const int32_t *__restrict__ node,
                                                    const int32_t *__restrict__ xptr,
                                                    const int32_t *__restrict__ xslot, int n_tps, int nlev,
                                                    int64_t n_s, int64_t n_g, int full_diag) {
  constexpr int LC = kFaceLevels;
  int blk = blockIdx.x;
  {
    const int nb = gridDim.x, q = nb >> 3, r = nb & 7, xc = blk & 7;
    blk = (xc < r ? xc * (q + 1) : r * (q + 1) + (xc - r) * q) + (blk >> 3);
  }
  const int nbx = (n_tps + 255) >> 8;
  const int chunk = blk / nbx;
  const int k = (blk - chunk * nbx) * 256 + threadIdx.x;
  const int v0 = chunk * LC;
  if (k >= n_tps) return;
  const int64_t n = node[k];
  const int a = xptr[k], b = xptr[k + 1];
  double acc[LC], f1[LC];
#pragma unroll
  for (int u = 0; u < LC; ++u) {
    const int64_t row = (int64_t)(v0 + u) * n_g;
    acc[u] = (v0 + u < nlev) ? F[row + k] : 0.0;
    f1[u] = (v0 + u < nlev) ? F[row + n_tps + k] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < LC; ++u) acc[u] += f1[u];
  for (int q = a; q < b; ++q) {
    const int64_t sl = xslot[q];
    double f[LC];
#pragma unroll
    for (int u = 0; u < LC; ++u) f[u] = (v0 + u < nlev) ? F[(int64_t)(v0 + u) * n_g + sl] : 0.0;
#pragma unroll
    for (int u = 0; u < LC; ++u) acc[u] += f[u];
  }
#pragma unroll
  for (int u = 0; u < LC; ++u) {
    const int v = v0 + u;
    if (v < nlev) {
      const int64_t idx = (int64_t)v * n_s + n;
      if (full_diag) diag[idx] = acc[u];
      const double di = (v == nlev - 1) ? 0.0 : recip(acc[u]);
      dinv[idx] = di;
      if (dinv32) dinv32[idx] = (float)di;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Vertical line blocks of A_II (the line smoother of the p-multigrid preconditioner): the entries
// A[(v, n), (v - d, n)], d = 1..p, coupling the nodes of one vertical node line.  For the node
// (i, j) of a column and levels k != k' of one element layer (collocated quadrature), only the
// zeta-zeta term and, at element edges (D_ii or D_jj nonzero), the mixed terms survive:
//   sum_c D[c][k] D[c][k'] G_zz(c) + D_ii (D[k][k'] G_xz(k) + D[k'][k] G_xz(k'))
//                                  + D_jj (D[k][k'] G_yz(k) + D[k'][k] G_yz(k')),
// all at points of the thread's own vertical line.  Row v = l p + k (k = 1..p) takes its
// sub-diagonals from layer l; row 0 has none.  Colour schedule (read-add-write over the columns
// of a horizontal node).  Band layout: band[d][v][n] (d = 1..p; d = 0 is left to the factor).
// ---------------------------------------------------------------------------------------------
template <int P, int DIM>
__global__ __launch_bounds__(256) void k_line_band(const double *__restrict__ cg, const double *__restrict__ hm,
                                                   int64_t hstride, const int32_t *__restrict__ eh_nodes,
                                                   const uint8_t *__restrict__ flags,
                                                   const int32_t *__restrict__ cols, int ncols, int nz, int64_t n_s,
                                                   const double *__restrict__ sigma,
                                                   const double *__restrict__ layer_s, double *__restrict__ band) {
  using S = Sh<P, DIM>;
  constexpr int N1 = S::N1, NH = S::NH, CPB = S::CPB;
  const int lc = threadIdx.x / NH;
  const int t = threadIdx.x - lc * NH;
  const int i = t % N1, j = t / N1;
  const int ci = blockIdx.x * CPB + lc;
  if (ci >= ncols) return;
  const int col = cols[ci];
  const int hn = eh_nodes[(int64_t)col * NH + t];
  const uint8_t fl = flags[(int64_t)col * NH + t];
  const int64_t ho = (int64_t)col * NH + t;
  const int64_t nlev = (int64_t)P * nz + 1;
  const double H = cg[0 * hstride + ho], Hx = cg[1 * hstride + ho], hx = cg[2 * hstride + ho];
  double Hy = 0.0, hy = 0.0, A00, A01 = 0.0, A10 = 0.0, A11 = 0.0, detJh;
  if constexpr (DIM == 3) {
    Hy = cg[3 * hstride + ho];
    hy = cg[4 * hstride + ho];
    A00 = hm[0 * hstride + ho];
    A01 = hm[1 * hstride + ho];
    A10 = hm[2 * hstride + ho];
    A11 = hm[3 * hstride + ho];
    detJh = hm[4 * hstride + ho];
  } else {
    A00 = hm[0 * hstride + ho];
    detJh = hm[1 * hstride + ho];
  }
  const double wh = DIM == 3 ? wgt(P, i) * wgt(P, j) : wgt(P, i);
  const double Dii = dmat<double>(P, i, i), Djj = DIM == 3 ? dmat<double>(P, j, j) : 0.0;
  // row 0 (bottom level) has no sub-diagonal entries
#pragma unroll
  for (int d = 1; d <= P; ++d) scatter(band, ((int64_t)d * nlev + 0) * n_s + hn, 0.0, fl);
  for (int l = 0; l < nz; ++l) {
    const double zz = 0.5 * (layer_s[l + 1] - layer_s[l]) * H;
    const double izz = 1.0 / zz;
    double gzz[N1], gxz[N1], gyz[N1];
#pragma unroll
    for (int c = 0; c < N1; ++c) {
      const double sg = sigma[l * P + c];
      const double zx = -hx + sg * Hx;
      const double f = wh * wgt(P, c) * detJh * zz;
      if constexpr (DIM == 3) {
        const double zy = -hy + sg * Hy;
        const double b2x = -(zx * A00 + zy * A10) * izz;
        const double b2y = -(zx * A01 + zy * A11) * izz;
        gxz[c] = f * (A00 * b2x + A01 * b2y);
        gyz[c] = f * (A10 * b2x + A11 * b2y);
        gzz[c] = f * (b2x * b2x + b2y * b2y + izz * izz);
      } else {
        const double b1x = -zx * A00 * izz;
        gxz[c] = f * A00 * b1x;
        gyz[c] = 0.0;
        gzz[c] = f * (b1x * b1x + izz * izz);
      }
    }
#pragma unroll
    for (int k = 1; k <= P; ++k) {
      const int64_t v = (int64_t)l * P + k;
#pragma unroll
      for (int d = 1; d <= P; ++d) {
        double val = 0.0;
        if (d <= k) {
          const int kp = k - d;
#pragma unroll
          for (int c = 0; c < N1; ++c) val += dmat<double>(P, c, k) * dmat<double>(P, c, kp) * gzz[c];
          const double dk = dmat<double>(P, k, kp), dkp = dmat<double>(P, kp, k);
          val += Dii * (dk * gxz[k] + dkp * gxz[kp]) + Djj * (dk * gyz[k] + dkp * gyz[kp]);
        }
        scatter(band, ((int64_t)d * nlev + v) * n_s + hn, val, fl);
      }
    }
  }
}

// ---------------------------------------------------------------------------------------------
// Neumann load (paper Eq. 1): f_i = sum over bottom and wall/body faces of int (q.n) l_i dS.
// ---------------------------------------------------------------------------------------------
template <int P, int DIM>
__global__ __launch_bounds__(256) void k_neumann(const double *__restrict__ qv, double *__restrict__ f,
                                                 const double *__restrict__ Hg, const double *__restrict__ hg,
                                                 const double *__restrict__ hm, int64_t hstride,
                                                 const int32_t *__restrict__ eh_nodes,
                                                 const uint8_t *__restrict__ flags, const int32_t *__restrict__ tags,
                                                 const int32_t *__restrict__ cols, int ncols, int nz, int64_t n_s,
                                                 int64_t n_v, const double *__restrict__ sigma,
                                                 const double *__restrict__ layer_s) {
  using S = Sh<P, DIM>;
  constexpr int N1 = S::N1, NH = S::NH, CPB = S::CPB;
  __shared__ double sH[CPB * NH];
  __shared__ double sh[CPB * NH];
  const int lc = threadIdx.x / NH;
  const int t = threadIdx.x - lc * NH;
  const int i = t % N1, j = t / N1;
  const int ci = blockIdx.x * CPB + lc;
  const bool active = ci < ncols;
  const int col = active ? cols[ci] : 0;
  const int hn = active ? eh_nodes[(int64_t)col * NH + t] : 0;
  const uint8_t fl = active ? flags[(int64_t)col * NH + t] : 0;
  const int64_t ho = (int64_t)col * NH + t;
  const double Hn = active ? Hg[hn] : 1.0;
  sH[lc * NH + t] = Hn;
  sh[lc * NH + t] = active ? hg[hn] : 0.0;
  __syncthreads();
  double Hx = 0.0, hx = 0.0, Hy = 0.0, hy = 0.0;
#pragma unroll
  for (int m = 0; m < N1; ++m) {
    Hx += dmat<double>(P, i, m) * sH[lc * NH + j * N1 + m];
    hx += dmat<double>(P, i, m) * sh[lc * NH + j * N1 + m];
    if constexpr (DIM == 3) {
      Hy += dmat<double>(P, j, m) * sH[lc * NH + m * N1 + i];
      hy += dmat<double>(P, j, m) * sh[lc * NH + m * N1 + i];
    }
  }
  if (!active) return;   // no barriers below
  constexpr int NS = DIM == 3 ? 4 : 2;
  int tg[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) tg[s] = tags ? tags[(int64_t)col * NS + s] : 0;
  const int nlev = P * nz + 1;
  for (int v = 0; v < nlev; ++v) {
    const int l = v == P * nz ? nz - 1 : v / P;
    const int k = v - l * P;
    const double sg = sigma[v];
    const double zz = 0.5 * (layer_s[l + 1] - layer_s[l]) * Hn;
    const double zx = -hx + sg * Hx;
    const int64_t idx = (int64_t)v * n_s + hn;
    // a node on a layer interface (k = 0 or P, inside the column) belongs to two layers:
    // side faces of both layers contribute with their own vertical weights
    double val = 0.0;
    if constexpr (DIM == 3) {
      const double xxi = hm[5 * hstride + ho], xet = hm[6 * hstride + ho];
      const double yxi = hm[7 * hstride + ho], yet = hm[8 * hstride + ho];
      const double zy = -hy + sg * Hy;
      const double qx = qv[idx], qy = qv[n_v + idx], qz = qv[2 * n_v + idx];
      const double wi = wgt(P, i), wj = wgt(P, j);
      if (v == 0) {   // bottom: -(J_xi x J_eta)
        const double nx = -(yxi * zy - zx * yet), ny = -(zx * xet - xxi * zy), nzv = -(xxi * yet - yxi * xet);
        val += wi * wj * (qx * nx + qy * ny + qz * nzv);
      }
      // vertical weight of this node: one or two layers
      for (int pass = 0; pass < 2; ++pass) {
        int ll, kk;
        if (pass == 0) {
          ll = l;
          kk = k;
        } else {
          if (!(k == 0 && l > 0)) break;
          ll = l - 1;
          kk = P;
        }
        const double zzl = 0.5 * (layer_s[ll + 1] - layer_s[ll]) * Hn;
        const double wk = wgt(P, kk);
        if (j == 0 && tg[0]) val += wi * wk * (-(-zzl * yxi) * qx - (zzl * xxi) * qy);
        if (i == P && tg[1]) val += wj * wk * ((yet * zzl) * qx + (-xet * zzl) * qy);
        if (j == P && tg[2]) val += wi * wk * ((-zzl * yxi) * qx + (zzl * xxi) * qy);
        if (i == 0 && tg[3]) val += wj * wk * (-(yet * zzl) * qx - (-xet * zzl) * qy);
      }
      (void)zz;
    } else {
      const double xxi = hm[1 * hstride + ho];
      const double qx = qv[idx], qz = qv[n_v + idx];
      const double wi = wgt(P, i);
      if (v == 0) val += wi * (zx * qx - xxi * qz);
      for (int pass = 0; pass < 2; ++pass) {
        int ll, kk;
        if (pass == 0) {
          ll = l;
          kk = k;
        } else {
          if (!(k == 0 && l > 0)) break;
          ll = l - 1;
          kk = P;
        }
        const double zzl = 0.5 * (layer_s[ll + 1] - layer_s[ll]) * Hn;
        const double wk = wgt(P, kk);
        if (i == 0 && tg[0]) val += wk * (-zzl * qx);
        if (i == P && tg[1]) val += wk * (zzl * qx);
      }
      (void)zz;
    }
    scatter(f, idx, val, fl);
  }
}

// ---------------------------------------------------------------------------------------------
// Vertical velocity at the free surface (Steps 4.4-4.5): lumped-GLL L2 projection of dphi/dz.
// For extruded elements d/dz = (1/z_zeta) d/dzeta and det J = det J_h z_zeta, and z_zeta at a
// surface node is the same in every adjacent top element, so
//   w_n = sum_e w_i w_j w_p det J_h (dphi/dzeta)_e / (z_zeta sum_e w_i w_j w_p det J_h).
// ---------------------------------------------------------------------------------------------
template <int P, int DIM>
__global__ __launch_bounds__(256) void k_wsurf(const double *__restrict__ phi, const int32_t *__restrict__ eh_nodes,
                                               const uint8_t *__restrict__ flags, const int32_t *__restrict__ cols,
                                               int ncols, int nz, int64_t n_s, const double *__restrict__ hm,
                                               int64_t hstride, const double *__restrict__ Hg,
                                               const double *__restrict__ mlump, double half_ds,
                                               double *__restrict__ wnum, double *__restrict__ w) {
  using S = Sh<P, DIM>;
  constexpr int N1 = S::N1, NH = S::NH, CPB = S::CPB;
  const int lc = threadIdx.x / NH;
  const int t = threadIdx.x - lc * NH;
  const int i = t % N1, j = t / N1;
  const int ci = blockIdx.x * CPB + lc;
  if (ci >= ncols) return;
  const int col = cols[ci];
  const int hn = eh_nodes[(int64_t)col * NH + t];
  const uint8_t fl = flags[(int64_t)col * NH + t];
  const int64_t ho = (int64_t)col * NH + t;
  const int v0 = (nz - 1) * P;
  double dz = 0.0;
#pragma unroll
  for (int m = 0; m < N1; ++m) dz += dmat<double>(P, P, m) * phi[(int64_t)(v0 + m) * n_s + hn];
  const double det = DIM == 3 ? hm[4 * hstride + ho] : hm[1 * hstride + ho];
  const double wq = (DIM == 3 ? wgt(P, i) * wgt(P, j) : wgt(P, i)) * wgt(P, P);
  const double num = scatter(wnum, hn, wq * det * dz, fl);
  if (fl & kLast) w[hn] = num / (half_ds * Hg[hn] * mlump[hn]);
}

// ---------------------------------------------------------------------------------------------
// Free-surface right-hand side (Step 4.6, Eqs. 2-3, lumped surface mass; linear potential flow:
// their linear terms only), fused with the ERK4 stage update (Sec. 3.2) and, after the last
// stage, the relaxation zones (Sec. 3.3).
// ---------------------------------------------------------------------------------------------
template <int P, int DIM>
__global__ __launch_bounds__(256) void k_rhs(const double *__restrict__ eta, const double *__restrict__ phs,
                                             const double *__restrict__ wv, const int32_t *__restrict__ eh_nodes,
                                             const uint8_t *__restrict__ flags, const int32_t *__restrict__ cols,
                                             int ncols, const double *__restrict__ hm, int64_t hstride,
                                             const double *__restrict__ mlump_s, double g, double *__restrict__ nk,
                                             double *__restrict__ nd, RkStageArgs a) {
  using S = Sh<P, DIM>;
  constexpr int N1 = S::N1, NH = S::NH, CPB = S::CPB;
  __shared__ double se[CPB * NH];
  __shared__ double sp[CPB * NH];
  const int lc = threadIdx.x / NH;
  const int t = threadIdx.x - lc * NH;
  const int i = t % N1, j = t / N1;
  const int ci = blockIdx.x * CPB + lc;
  const bool active = ci < ncols;
  const int col = active ? cols[ci] : 0;
  const int hn = active ? eh_nodes[(int64_t)col * NH + t] : 0;
  const uint8_t fl = active ? flags[(int64_t)col * NH + t] : 0;
  const int64_t ho = (int64_t)col * NH + t;
  const double en = active ? eta[hn] : 0.0;
  const double pn = active ? phs[hn] : 0.0;
  se[lc * NH + t] = en;
  sp[lc * NH + t] = pn;
  __syncthreads();
  if (!active) return;
  double exi = 0.0, pxi = 0.0, eet = 0.0, pet = 0.0;
#pragma unroll
  for (int m = 0; m < N1; ++m) {
    exi += dmat<double>(P, i, m) * se[lc * NH + j * N1 + m];
    pxi += dmat<double>(P, i, m) * sp[lc * NH + j * N1 + m];
    if constexpr (DIM == 3) {
      eet += dmat<double>(P, j, m) * se[lc * NH + m * N1 + i];
      pet += dmat<double>(P, j, m) * sp[lc * NH + m * N1 + i];
    }
  }
  double ex, ey = 0.0, px, py = 0.0, det, ws;
  if constexpr (DIM == 3) {
    const double A00 = hm[0 * hstride + ho], A01 = hm[1 * hstride + ho];
    const double A10 = hm[2 * hstride + ho], A11 = hm[3 * hstride + ho];
    det = hm[4 * hstride + ho];
    ex = A00 * exi + A10 * eet;
    ey = A01 * exi + A11 * eet;
    px = A00 * pxi + A10 * pet;
    py = A01 * pxi + A11 * pet;
    ws = wgt(P, i) * wgt(P, j);
  } else {
    const double A = hm[0 * hstride + ho];
    det = hm[1 * hstride + ho];
    ex = A * exi;
    px = A * pxi;
    ws = wgt(P, i);
  }
  const double w = wv[hn];
  const double ee = ex * ex + ey * ey;
  const double Ek = a.linear ? w : -(ex * px + ey * py) + w * (1.0 + ee);
  const double Ed = a.linear ? -g * en : -g * en - 0.5 * (px * px + py * py) + 0.5 * w * w * (1.0 + ee);
  const double ms = ws * det;
  const double sk = scatter(nk, hn, ms * Ek, fl);
  const double sd = scatter(nd, hn, ms * Ed, fl);
  if (!(fl & kLast)) return;
  stage_update(a, hn, sk / mlump_s[hn], sd / mlump_s[hn]);
}

// ---------------------------------------------------------------------------------------------
// Host-side dispatch over (dim, p).
// ---------------------------------------------------------------------------------------------
#define FNPF_DISPATCH(DIMV, PV, CALL)                       \
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

template <int P, int DIM>
static hipError_t geom_impl(Ctx &c, const double *eta, const double *h, bool store_G, bool h_is_total,
                            hipStream_t s, bool full) {
  using S = Sh<P, DIM>;
  const int64_t hs = (int64_t)c.n_eh * c.nh;
  if constexpr (DIM == 3) {
    // owner-computes with the apply's tiles and face slots (same 32-bit range conditions)
    const int64_t lim = int64_t(1) << 32;
    if (c.tile_cols == S::CPB && c.n_v * 8 < lim && (int64_t)(c.p * c.nz + 1) * c.n_gslots * 8 < lim) {
      const int nb = (c.n_eh + S::CPB - 1) / S::CPB;
      auto kern = store_G ? k_geom<P, DIM, true, true> : k_geom<P, DIM, true, false>;
      kern<<<nb, S::NT, 0, s>>>(
          eta, h, c.d_hm, hs, c.d_eh_nodes, c.d_flags, nullptr, c.n_eh, c.nz, c.n_s, c.d_sigma, c.d_layer_s,
          store_G ? c.d_G64 : nullptr, (store_G && c.want32) ? c.d_G32 : nullptr, c.d_diag, c.d_dinv,
          c.want32 ? c.d_dinv32 : nullptr, c.d_geoH, c.d_geoh, c.d_cg64, c.want32 ? c.d_cg32 : nullptr,
          h_is_total ? 1 : 0, c.d_err, c.d_F64, c.d_gslot, c.n_gslots, c.d_xch, full ? 1 : 0);
      if (c.n_tps > 0)
        k_diag_faces<<<face_blocks_n(c, c.n_tps), 256, 0, s>>>(c.d_diag, c.d_dinv, c.want32 ? c.d_dinv32 : nullptr,
                                                                c.d_F64, c.d_tps_node, c.d_gx_ptr, c.d_gx_slot,
                                                                c.n_tps, c.p * c.nz + 1, c.n_s, c.n_gslots,
                                                                full ? 1 : 0);
      c.have_diag = full;
      return hipGetLastError();
    }
  }
  for (const auto &cr : c.colours) {
    if (cr.count == 0) continue;
    const int nb = (cr.count + S::CPB - 1) / S::CPB;
    auto kern = store_G ? k_geom<P, DIM, false, true> : k_geom<P, DIM, false, false>;
    kern<<<nb, S::NT, 0, s>>>(eta, h, c.d_hm, hs, c.d_eh_nodes, c.d_flags, c.d_cols + cr.offset, cr.count, c.nz,
                              c.n_s, c.d_sigma, c.d_layer_s, store_G ? c.d_G64 : nullptr,
                              (store_G && c.want32) ? c.d_G32 : nullptr, c.d_diag, c.d_dinv,
                              c.want32 ? c.d_dinv32 : nullptr, c.d_geoH, c.d_geoh, c.d_cg64,
                              c.want32 ? c.d_cg32 : nullptr, h_is_total ? 1 : 0, c.d_err, nullptr, nullptr, 0,
                              nullptr, 1);
  }
  c.have_diag = true;   // the colour schedule assembles every node's diagonal in place
  return hipGetLastError();
}

hipError_t launch_geom(Ctx &c, const double *eta, const double *h, bool store_G, bool h_is_total, hipStream_t s,
                       bool full_diag) {
  const bool full = store_G || full_diag || c.keep_diag;
  c.have_diag = false;
  if (c.dim == 3) {
    FNPF_DISPATCH(3, c.p, return (geom_impl<P_, 3>(c, eta, h, store_G, h_is_total, s, full)));
  } else {
    FNPF_DISPATCH(2, c.p, return (geom_impl<P_, 2>(c, eta, h, store_G, h_is_total, s, full)));
  }
  return hipSuccess;
}

hipError_t ensure_diag(Ctx &c, hipStream_t s) {
  if (c.have_diag) return hipSuccess;
  // the surface H and h of the last update, saved by the geometry kernel at every surface node
  return launch_geom(c, c.d_geoH, c.d_geoh, false, true, s, true);
}

template <int P, int DIM, typename T, bool MASK, bool DOT>
static hipError_t apply_impl(Ctx &c, const T *x, T *y, const T *G, double *partial, const int32_t *skip,
                             hipStream_t s, T *face_scratch) {
  using S = Sh<P, DIM>;
  const int64_t hs = (int64_t)c.n_eh * c.nh;
  const bool fused = c.apply_variant == 0;
  const T *cg = nullptr, *hmT = nullptr, *sig = nullptr, *hds = nullptr;
  if constexpr (sizeof(T) == 8) {
    cg = (const T *)c.d_cg64;
    hmT = (const T *)c.d_hm;
    sig = (const T *)c.d_sigma;
    hds = (const T *)c.d_half_ds;
  } else {
    cg = (const T *)c.d_cg32;
    hmT = (const T *)c.d_hm32;
    sig = (const T *)c.d_sigma32;
    hds = (const T *)c.d_half_ds32;
  }
  int off = 0;
  for (const auto &cr : c.colours) {
    if (cr.count == 0) continue;
    const int nb = (cr.count + S::CPB - 1) / S::CPB;
    if (fused) {
      if constexpr (DIM == 3) {
        if (owner_apply_active(c)) {
          if (c.tile_cols != S::CPB) return hipErrorInvalidValue;   // host tiles = workgroups
          T *F = face_scratch;
          if (F == nullptr) {
            if constexpr (sizeof(T) == 8) F = (T *)c.d_F64; else F = (T *)c.d_F32;
          }
          const int nb1 = (c.n_eh + S::CPB - 1) / S::CPB;
          k_apply_lines<P, T, MASK, DOT, true><<<nb1, S::NT, 0, s>>>(
              x, y, cg, hmT, hs, sig, hds, c.d_eh_nodes, c.d_flags, nullptr, c.n_eh, c.nz, c.n_s,
              DOT ? partial : nullptr, skip, F, c.d_tslot, c.n_tslots, c.d_xch);
          if (c.n_tps > 0)
            k_apply_faces<T, MASK, DOT><<<face_blocks_n(c, c.n_tps), 256, 0, s>>>(
                x, y, F, c.d_tps_node, c.d_tps_ptr, c.d_tps_slot, c.n_tps, c.p * c.nz + 1, c.n_s, c.n_tslots,
                DOT ? partial + nb1 : nullptr, skip);
          return hipGetLastError();
        }
        if (c.apply_lines && (int64_t)c.n_v * (int64_t)sizeof(T) < (int64_t(1) << 32)) {
          k_apply_lines<P, T, MASK, DOT><<<nb, S::NT, 0, s>>>(x, y, cg, hmT, hs, sig, hds, c.d_eh_nodes, c.d_flags,
                                                               c.d_cols + cr.offset, cr.count, c.nz, c.n_s,
                                                               DOT ? partial + off : nullptr, skip);
          off += nb;
          continue;
        }
      }
      k_apply_fused2<P, DIM, T, MASK, DOT><<<nb, S::NT, 0, s>>>(x, y, cg, hmT, hs, sig, hds, c.d_eh_nodes, c.d_flags,
                                                                c.d_cols + cr.offset, cr.count, c.nz, c.n_s,
                                                                DOT ? partial + off : nullptr, skip);
    }
    else
      k_apply<P, DIM, T, MASK, DOT><<<nb, S::NT, 0, s>>>(x, y, G, c.d_eh_nodes, c.d_flags, c.d_cols + cr.offset,
                                                         cr.count, c.nz, c.n_s, DOT ? partial + off : nullptr, skip);
    off += nb;
  }
  return hipGetLastError();
}

template <int P, int DIM>
static hipError_t apply_dispatch(Ctx &c, fnpf_dtype dt, const void *x, void *y, bool mask, double *partial,
                                 const int32_t *skip, hipStream_t s, void *fs) {
  const bool dot = partial != nullptr;
  if (dt == FNPF_F64) {
    const double *xx = (const double *)x;
    double *yy = (double *)y;
    double *F = (double *)fs;
    if (!mask) return apply_impl<P, DIM, double, false, false>(c, xx, yy, c.d_G64, nullptr, skip, s, F);
    if (!dot) return apply_impl<P, DIM, double, true, false>(c, xx, yy, c.d_G64, nullptr, skip, s, F);
    return apply_impl<P, DIM, double, true, true>(c, xx, yy, c.d_G64, partial, skip, s, F);
  }
  const float *xx = (const float *)x;
  float *yy = (float *)y;
  float *F = (float *)fs;
  if (!mask) return apply_impl<P, DIM, float, false, false>(c, xx, yy, c.d_G32, nullptr, skip, s, F);
  if (!dot) return apply_impl<P, DIM, float, true, false>(c, xx, yy, c.d_G32, nullptr, skip, s, F);
  return apply_impl<P, DIM, float, true, true>(c, xx, yy, c.d_G32, partial, skip, s, F);
}

// face_scratch: device memory for the face slots in place of the context's own (nullptr: the
// context's); it must hold (p nz + 1) * n_tslots elements of the apply's precision
hipError_t launch_apply(Ctx &c, fnpf_dtype dt, const void *x, void *y, bool mask, double *partial,
                        const int32_t *skip, hipStream_t s, void *face_scratch) {
  // one partial per block of every launch when the dot product is fused
  if (partial != nullptr &&
      !partials_fit(c.n_partial, owner_apply_active(c) ? owner_apply_blocks(c) : c.max_colour_blocks, 1))
    return hipErrorInvalidValue;
  if (c.dim == 3) {
    FNPF_DISPATCH(3, c.p, return (apply_dispatch<P_, 3>(c, dt, x, y, mask, partial, skip, s, face_scratch)));
  } else {
    FNPF_DISPATCH(2, c.p, return (apply_dispatch<P_, 2>(c, dt, x, y, mask, partial, skip, s, face_scratch)));
  }
  return hipSuccess;
}

template <int P, int DIM>
static hipError_t line_band_impl(Ctx &c, double *band, hipStream_t s) {
  using S = Sh<P, DIM>;
  const int64_t hs = (int64_t)c.n_eh * c.nh;
  for (const auto &cr : c.colours) {
    if (cr.count == 0) continue;
    const int nb = (cr.count + S::CPB - 1) / S::CPB;
    k_line_band<P, DIM><<<nb, S::NT, 0, s>>>(c.d_cg64, c.d_hm, hs, c.d_eh_nodes, c.d_flags, c.d_cols + cr.offset,
                                             cr.count, c.nz, c.n_s, c.d_sigma, c.d_layer_s, band);
  }
  return hipGetLastError();
}

// band[d][v][n] (d = 1..p) of the current geometry's vertical line blocks (colour schedule)
hipError_t launch_line_band(Ctx &c, double *band, hipStream_t s) {
  if (c.dim == 3) {
    FNPF_DISPATCH(3, c.p, return (line_band_impl<P_, 3>(c, band, s)));
  } else {
    FNPF_DISPATCH(2, c.p, return (line_band_impl<P_, 2>(c, band, s)));
  }
  return hipSuccess;
}

template <int P, int DIM>
static hipError_t neumann_impl(Ctx &c, const double *q, double *f, hipStream_t s) {
  using S = Sh<P, DIM>;
  const int64_t hs = (int64_t)c.n_eh * c.nh;
  for (const auto &cr : c.colours) {
    if (cr.count == 0) continue;
    const int nb = (cr.count + S::CPB - 1) / S::CPB;
    k_neumann<P, DIM><<<nb, S::NT, 0, s>>>(q, f, c.d_geoH, c.d_geoh, c.d_hm, hs, c.d_eh_nodes, c.d_flags,
                                           c.d_face_tag, c.d_cols + cr.offset, cr.count, c.nz, c.n_s, c.n_v,
                                           c.d_sigma, c.d_layer_s);
  }
  return hipGetLastError();
}

hipError_t launch_neumann(Ctx &c, const double *q, double *f, hipStream_t s) {
  if (c.dim == 3) {
    FNPF_DISPATCH(3, c.p, return (neumann_impl<P_, 3>(c, q, f, s)));
  } else {
    FNPF_DISPATCH(2, c.p, return (neumann_impl<P_, 2>(c, q, f, s)));
  }
  return hipSuccess;
}

template <int P, int DIM>
static hipError_t wsurf_impl(Ctx &c, const double *phi, double *w, hipStream_t s) {
  using S = Sh<P, DIM>;
  const int64_t hs = (int64_t)c.n_eh * c.nh;
  const double half_ds = 0.5 * (c.h_layer_s[c.nz] - c.h_layer_s[c.nz - 1]);
  for (const auto &cr : c.colours) {
    if (cr.count == 0) continue;
    const int nb = (cr.count + S::CPB - 1) / S::CPB;
    k_wsurf<P, DIM><<<nb, S::NT, 0, s>>>(phi, c.d_eh_nodes, c.d_flags, c.d_cols + cr.offset, cr.count, c.nz, c.n_s,
                                         c.d_hm, hs, c.d_geoH, c.d_mlump_w, half_ds, c.d_wnum, w);
  }
  return hipGetLastError();
}

hipError_t launch_wsurf(Ctx &c, const double *phi, double *w, hipStream_t s) {
  if (c.dim == 3) {
    FNPF_DISPATCH(3, c.p, return (wsurf_impl<P_, 3>(c, phi, w, s)));
  } else {
    FNPF_DISPATCH(2, c.p, return (wsurf_impl<P_, 2>(c, phi, w, s)));
  }
  return hipSuccess;
}

template <int P, int DIM>
static hipError_t rhs_impl(Ctx &c, const double *eta, const double *phs, const double *w, const RkStageArgs &a,
                           hipStream_t s) {
  using S = Sh<P, DIM>;
  const int64_t hs = (int64_t)c.n_eh * c.nh;
  for (const auto &cr : c.colours) {
    if (cr.count == 0) continue;
    const int nb = (cr.count + S::CPB - 1) / S::CPB;
    k_rhs<P, DIM><<<nb, S::NT, 0, s>>>(eta, phs, w, c.d_eh_nodes, c.d_flags, c.d_cols + cr.offset, cr.count, c.d_hm,
                                       hs, c.d_mlump_s, c.g, c.d_nk, c.d_nd, a);
  }
  return hipGetLastError();
}

hipError_t launch_rhs(Ctx &c, const double *eta, const double *phi_s, const double *w, const RkStageArgs &a,
                      hipStream_t s) {
  if (c.dim == 3) {
    FNPF_DISPATCH(3, c.p, return (rhs_impl<P_, 3>(c, eta, phi_s, w, a, s)));
  } else {
    FNPF_DISPATCH(2, c.p, return (rhs_impl<P_, 2>(c, eta, phi_s, w, a, s)));
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------------------------
// Modal filter of a surface field (Sec. 3.2, modal filtering), tensor-product form on one
// surface element: the nodal filter matrix M = V diag(sigma) V^-1 acts along xi and then along
// eta (one direction in 2D).  Shared nodes take the mean of the element results (colour-ordered
// accumulation, scaled by 1/multiplicity by the last writer).  TR: the transpose map, which
// scales by 1/multiplicity first, applies M^T and adds the sums into out.
// ---------------------------------------------------------------------------------------------
template <int P, int DIM, bool TR>
__global__ __launch_bounds__(256) void k_modal_filter(const double *__restrict__ in, double *__restrict__ out,
                                                      const int32_t *__restrict__ eh_nodes,
                                                      const uint8_t *__restrict__ flags,
                                                      const int32_t *__restrict__ cols, int ncols,
                                                      const double *__restrict__ Mg,
                                                      const double *__restrict__ inv_mult,
                                                      double *__restrict__ acc) {
  using S = Sh<P, DIM>;
  constexpr int N1 = S::N1, NH = S::NH, CPB = S::CPB;
  __shared__ double sM[N1 * N1];
  __shared__ double sg[CPB * NH];
  __shared__ double st[CPB * NH];
  const int lc = threadIdx.x / NH;
  const int t = threadIdx.x - lc * NH;
  const int i = t % N1, j = t / N1;
  const int ci = blockIdx.x * CPB + lc;
  const bool active = ci < ncols;
  const int col = active ? cols[ci] : 0;
  const int hn = active ? eh_nodes[(int64_t)col * NH + t] : 0;
  const uint8_t fl = active ? flags[(int64_t)col * NH + t] : 0;
  if (threadIdx.x < N1 * N1) {
    // stored transposed for the TR map: A[r][k] = M[k][r]
    const int r = threadIdx.x / N1, k = threadIdx.x - r * N1;
    sM[threadIdx.x] = TR ? Mg[k * N1 + r] : Mg[threadIdx.x];
  }
  double g = active ? in[hn] : 0.0;
  if (TR && active) g *= inv_mult[hn];
  sg[lc * NH + t] = g;
  __syncthreads();
  double v = 0.0;
#pragma unroll
  for (int k = 0; k < N1; ++k) v += sM[i * N1 + k] * sg[lc * NH + j * N1 + k];
  if constexpr (DIM == 3) {
    st[lc * NH + t] = v;
    __syncthreads();
    v = 0.0;
#pragma unroll
    for (int k = 0; k < N1; ++k) v += sM[j * N1 + k] * st[lc * NH + k * N1 + i];
  }
  if (!active) return;
  const double sum = scatter(acc, hn, v, fl);
  if (fl & kLast) {
    if (TR)
      out[hn] += sum;
    else
      out[hn] = sum * inv_mult[hn];
  }
}

template <int P, int DIM>
static hipError_t modal_filter_impl(Ctx &c, const double *in, double *out, bool tr, hipStream_t s) {
  using S = Sh<P, DIM>;
  for (const auto &cr : c.colours) {
    if (cr.count == 0) continue;
    const int nb = (cr.count + S::CPB - 1) / S::CPB;
    if (tr)
      k_modal_filter<P, DIM, true><<<nb, S::NT, 0, s>>>(in, out, c.d_eh_nodes, c.d_flags, c.d_cols + cr.offset,
                                                        cr.count, c.d_filt_M, c.d_filt_inv_mult, c.d_filt_acc);
    else
      k_modal_filter<P, DIM, false><<<nb, S::NT, 0, s>>>(in, out, c.d_eh_nodes, c.d_flags, c.d_cols + cr.offset,
                                                         cr.count, c.d_filt_M, c.d_filt_inv_mult, c.d_filt_acc);
  }
  return hipGetLastError();
}

hipError_t launch_modal_filter(Ctx &c, const double *in, double *out, bool transpose, hipStream_t s) {
  if (c.dim == 3) {
    FNPF_DISPATCH(3, c.p, return (modal_filter_impl<P_, 3>(c, in, out, transpose, s)));
  } else {
    FNPF_DISPATCH(2, c.p, return (modal_filter_impl<P_, 2>(c, in, out, transpose, s)));
  }
  return hipSuccess;
}

#include "adjoint_kernels.inc"

}  // namespace fnpf
