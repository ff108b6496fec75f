// Consistent, over-integrated free-surface right-hand side (Eq. 5 with the over-integration of
// Sec. 3.2): the integrands of Eqs. 2-3 are evaluated at nq x nq Gauss-Legendre points of each
// surface element (nq per direction in 2D slices), tested against the degree-p Lagrange basis,
// and the consistent surface mass system M k = b is solved by a preconditioned Chebyshev
// iteration with the lumped GLL mass as preconditioner.
//
// The eigenvalues of M_L^{-1} M lie in a range known from the element data alone: with u the
// degree-p field of a coefficient vector, u^T M_e u = sum_q W_q det_q u(x_q)^2 lies between
// min/max det_q times the exact L2 norm (the rule integrates u^2 exactly), the lumped form lies
// between min/max det_i times the GLL norm, and the GLL norm exceeds the L2 norm by a factor in
// [1, ((2p+1)/p)^d] (only the top Legendre mode per direction is integrated inexactly).  The
// iteration count follows from that interval for a 1e-15 contraction of the M-norm error, so the
// solve has a fixed length, needs no reductions and is a symmetric linear map of b (its VJP is
// the same solve).
//
// Elements are processed up to four per workgroup (one wave each), colour by colour (columns of
// one colour share no surface node), accumulating shared nodes in colour order like the other
// surface kernels.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fnpf_internal.h"
#include "stage_update.h"

namespace fnpf {

namespace {

constexpr int kSqThreads = 256;

__device__ __forceinline__ double acc_colour(double *y, int64_t idx, double val, uint8_t fl) {
  if (fl & kFirst) {
    y[idx] = val;
    return val;
  }
  const double s = y[idx] + val;
  y[idx] = s;
  return s;
}

// Dynamic LDS carve-out helper.
struct Carve {
  double *p;
  __device__ double *take(int n) {
    double *r = p;
    p += n;
    return r;
  }
};

// Every kernel below handles epb elements per block, tpe = 256 / epb threads per element, each
// element with its own LDS region of `per` doubles after the shared tables.  Groups without an
// element (the ragged end of a colour) take part in the barriers only.

// Forward: b_k, b_d (colour-accumulated, final at the last writer).
template <int P, int DIM>
__global__ __launch_bounds__(kSqThreads) void k_sq_rhs(const double *__restrict__ eta, const double *__restrict__ phs,
                                                       const double *__restrict__ wv,
                                                       const int32_t *__restrict__ eh_nodes,
                                                       const uint8_t *__restrict__ flags,
                                                       const int32_t *__restrict__ cols, int count, int epb, int per,
                                                       const double *__restrict__ Bg,
                                                       const double *__restrict__ Bdg, int nq,
                                                       const double *__restrict__ met, int64_t mstride, double g,
                                                       double *__restrict__ bk, double *__restrict__ bd) {
  constexpr int N1 = P + 1, NH = DIM == 3 ? N1 * N1 : N1;
  extern __shared__ double lds[];
  const int tpe = kSqThreads / epb, grp = threadIdx.x / tpe, tid = threadIdx.x - grp * tpe;
  const int ci = blockIdx.x * epb + grp;
  const bool act = ci < count;
  const int col = act ? cols[ci] : 0;
  const int nqd = DIM == 3 ? nq * nq : nq;
  double *sB = lds, *sBd = lds + nq * N1;
  Carve cv{lds + 2 * nq * N1 + grp * per};
  double *se = cv.take(NH), *sp = cv.take(NH), *sw = cv.take(NH);
  double *Qk = cv.take(nqd), *Qd = cv.take(nqd);
  for (int k = threadIdx.x; k < nq * N1; k += kSqThreads) {
    sB[k] = Bg[k];
    sBd[k] = Bdg[k];
  }
  for (int t = tid; act && t < NH; t += tpe) {
    const int hn = eh_nodes[(int64_t)col * NH + t];
    se[t] = eta[hn];
    sp[t] = phs[hn];
    sw[t] = wv[hn];
  }
  __syncthreads();
  const int64_t mb = (int64_t)col * nqd;
  if constexpr (DIM == 3) {
    double *Te = cv.take(N1 * nq), *Ted = cv.take(N1 * nq), *Tp = cv.take(N1 * nq), *Tpd = cv.take(N1 * nq),
           *Tw = cv.take(N1 * nq);
    double *Uk = cv.take(N1 * nq), *Ud = cv.take(N1 * nq);
    // along xi: (j, qx)
    for (int k = tid; act && k < N1 * nq; k += tpe) {
      const int j = k / nq, qx = k - j * nq;
      double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        const double b = sB[qx * N1 + i], bdx = sBd[qx * N1 + i];
        a0 += b * se[j * N1 + i];
        a1 += bdx * se[j * N1 + i];
        a2 += b * sp[j * N1 + i];
        a3 += bdx * sp[j * N1 + i];
        a4 += b * sw[j * N1 + i];
      }
      Te[k] = a0;
      Ted[k] = a1;
      Tp[k] = a2;
      Tpd[k] = a3;
      Tw[k] = a4;
    }
    __syncthreads();
    // along eta: (qy, qx); integrands times W det
    for (int k = tid; act && k < nqd; k += tpe) {
      const int qy = k / nq, qx = k - qy * nq;
      double ev = 0, exi = 0, eet = 0, pxi = 0, pet = 0, w = 0;
#pragma unroll
      for (int j = 0; j < N1; ++j) {
        const double b = sB[qy * N1 + j], bdy = sBd[qy * N1 + j];
        const int o = j * nq + qx;
        ev += b * Te[o];
        exi += b * Ted[o];
        eet += bdy * Te[o];
        pxi += b * Tpd[o];
        pet += bdy * Tp[o];
        w += b * Tw[o];
      }
      const double A00 = met[0 * mstride + mb + k], A01 = met[1 * mstride + mb + k];
      const double A10 = met[2 * mstride + mb + k], A11 = met[3 * mstride + mb + k];
      const double wd = met[4 * mstride + mb + k];
      const double ex = A00 * exi + A10 * eet, ey = A01 * exi + A11 * eet;
      const double px = A00 * pxi + A10 * pet, py = A01 * pxi + A11 * pet;
      const double ee = ex * ex + ey * ey;
      Qk[k] = wd * (-(ex * px + ey * py) + w * (1.0 + ee));
      Qd[k] = wd * (-g * ev - 0.5 * (px * px + py * py) + 0.5 * w * w * (1.0 + ee));
    }
    __syncthreads();
    // test functions, along eta then xi
    for (int k = tid; act && k < N1 * nq; k += tpe) {
      const int j = k / nq, qx = k - j * nq;
      double a0 = 0, a1 = 0;
      for (int qy = 0; qy < nq; ++qy) {
        const double b = sB[qy * N1 + j];
        a0 += b * Qk[qy * nq + qx];
        a1 += b * Qd[qy * nq + qx];
      }
      Uk[k] = a0;
      Ud[k] = a1;
    }
    __syncthreads();
    for (int t = tid; act && t < NH; t += tpe) {
      const int j = t / N1, i = t - j * N1;
      double a0 = 0, a1 = 0;
      for (int qx = 0; qx < nq; ++qx) {
        const double b = sB[qx * N1 + i];
        a0 += b * Uk[j * nq + qx];
        a1 += b * Ud[j * nq + qx];
      }
      const int64_t o = (int64_t)col * NH + t;
      const int hn = eh_nodes[o];
      const uint8_t fl = flags[o];
      acc_colour(bk, hn, a0, fl);
      acc_colour(bd, hn, a1, fl);
    }
  } else {
    for (int q = tid; act && q < nq; q += tpe) {
      double ev = 0, exi = 0, pxi = 0, w = 0;
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        const double b = sB[q * N1 + i], bdx = sBd[q * N1 + i];
        ev += b * se[i];
        exi += bdx * se[i];
        pxi += bdx * sp[i];
        w += b * sw[i];
      }
      const double A = met[0 * mstride + mb + q], wd = met[1 * mstride + mb + q];
      const double ex = A * exi, px = A * pxi;
      const double ee = ex * ex;
      Qk[q] = wd * (-(ex * px) + w * (1.0 + ee));
      Qd[q] = wd * (-g * ev - 0.5 * px * px + 0.5 * w * w * (1.0 + ee));
    }
    __syncthreads();
    for (int i = tid; act && i < N1; i += tpe) {
      double a0 = 0, a1 = 0;
      for (int q = 0; q < nq; ++q) {
        a0 += sB[q * N1 + i] * Qk[q];
        a1 += sB[q * N1 + i] * Qd[q];
      }
      const int64_t o = (int64_t)col * NH + i;
      const int hn = eh_nodes[o];
      const uint8_t fl = flags[o];
      acc_colour(bk, hn, a0, fl);
      acc_colour(bd, hn, a1, fl);
    }
  }
}

// y = M x for two fields stored [2][n_s] (consistent surface mass, W det at the Gauss points).
template <int P, int DIM>
__global__ __launch_bounds__(kSqThreads) void k_sq_mass(const double *__restrict__ x, double *__restrict__ y,
                                                        int64_t n_s, const int32_t *__restrict__ eh_nodes,
                                                        const uint8_t *__restrict__ flags,
                                                        const int32_t *__restrict__ cols, int count, int epb,
                                                        int per, const double *__restrict__ Bg, int nq,
                                                        const double *__restrict__ wdet) {
  constexpr int N1 = P + 1, NH = DIM == 3 ? N1 * N1 : N1;
  extern __shared__ double lds[];
  const int tpe = kSqThreads / epb, grp = threadIdx.x / tpe, tid = threadIdx.x - grp * tpe;
  const int ci = blockIdx.x * epb + grp;
  const bool act = ci < count;
  const int col = act ? cols[ci] : 0;
  const int nqd = DIM == 3 ? nq * nq : nq;
  double *sB = lds;
  Carve cv{lds + nq * N1 + grp * per};
  double *u0 = cv.take(NH), *u1 = cv.take(NH);
  double *Q0 = cv.take(nqd), *Q1 = cv.take(nqd);
  for (int k = threadIdx.x; k < nq * N1; k += kSqThreads) sB[k] = Bg[k];
  for (int t = tid; act && t < NH; t += tpe) {
    const int hn = eh_nodes[(int64_t)col * NH + t];
    u0[t] = x[hn];
    u1[t] = x[n_s + hn];
  }
  __syncthreads();
  const int64_t mb = (int64_t)col * nqd;
  if constexpr (DIM == 3) {
    double *T0 = cv.take(N1 * nq), *T1 = cv.take(N1 * nq);
    for (int k = tid; act && k < N1 * nq; k += tpe) {
      const int j = k / nq, qx = k - j * nq;
      double a0 = 0, a1 = 0;
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        const double b = sB[qx * N1 + i];
        a0 += b * u0[j * N1 + i];
        a1 += b * u1[j * N1 + i];
      }
      T0[k] = a0;
      T1[k] = a1;
    }
    __syncthreads();
    for (int k = tid; act && k < nqd; k += tpe) {
      const int qy = k / nq, qx = k - qy * nq;
      double a0 = 0, a1 = 0;
#pragma unroll
      for (int j = 0; j < N1; ++j) {
        const double b = sB[qy * N1 + j];
        a0 += b * T0[j * nq + qx];
        a1 += b * T1[j * nq + qx];
      }
      const double wd = wdet[mb + k];
      Q0[k] = wd * a0;
      Q1[k] = wd * a1;
    }
    __syncthreads();
    for (int k = tid; act && k < N1 * nq; k += tpe) {
      const int j = k / nq, qx = k - j * nq;
      double a0 = 0, a1 = 0;
      for (int qy = 0; qy < nq; ++qy) {
        const double b = sB[qy * N1 + j];
        a0 += b * Q0[qy * nq + qx];
        a1 += b * Q1[qy * nq + qx];
      }
      T0[k] = a0;   // T is free again after the barrier above
      T1[k] = a1;
    }
    __syncthreads();
    for (int t = tid; act && t < NH; t += tpe) {
      const int j = t / N1, i = t - j * N1;
      double a0 = 0, a1 = 0;
      for (int qx = 0; qx < nq; ++qx) {
        const double b = sB[qx * N1 + i];
        a0 += b * T0[j * nq + qx];
        a1 += b * T1[j * nq + qx];
      }
      const int64_t o = (int64_t)col * NH + t;
      const int hn = eh_nodes[o];
      const uint8_t fl = flags[o];
      acc_colour(y, hn, a0, fl);
      acc_colour(y + n_s, hn, a1, fl);
    }
  } else {
    for (int q = tid; act && q < nq; q += tpe) {
      double a0 = 0, a1 = 0;
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        a0 += sB[q * N1 + i] * u0[i];
        a1 += sB[q * N1 + i] * u1[i];
      }
      Q0[q] = wdet[mb + q] * a0;
      Q1[q] = wdet[mb + q] * a1;
    }
    __syncthreads();
    for (int i = tid; act && i < N1; i += tpe) {
      double a0 = 0, a1 = 0;
      for (int q = 0; q < nq; ++q) {
        a0 += sB[q * N1 + i] * Q0[q];
        a1 += sB[q * N1 + i] * Q1[q];
      }
      const int64_t o = (int64_t)col * NH + i;
      const int hn = eh_nodes[o];
      const uint8_t fl = flags[o];
      acc_colour(y, hn, a0, fl);
      acc_colour(y + n_s, hn, a1, fl);
    }
  }
}

// VJP of k_sq_rhs: from bbar = (bbar_k, bbar_d) [2][n_s], adds to eta_bar, phi_bar, w_bar
// (colour-accumulated in scratch scr[3][n_s], added by the last writer).
template <int P, int DIM>
__global__ __launch_bounds__(kSqThreads) void k_sq_rhs_vjp(
    const double *__restrict__ eta, const double *__restrict__ phs, const double *__restrict__ wv,
    const double *__restrict__ bbar, int64_t n_s, const int32_t *__restrict__ eh_nodes,
    const uint8_t *__restrict__ flags, const int32_t *__restrict__ cols, int count, int epb, int per,
    const double *__restrict__ Bg, const double *__restrict__ Bdg, int nq, const double *__restrict__ met,
    int64_t mstride, double g, double *__restrict__ scr, double *__restrict__ eta_bar, double *__restrict__ phi_bar,
    double *__restrict__ w_bar) {
  constexpr int N1 = P + 1, NH = DIM == 3 ? N1 * N1 : N1;
  extern __shared__ double lds[];
  const int tpe = kSqThreads / epb, grp = threadIdx.x / tpe, tid = threadIdx.x - grp * tpe;
  const int ci = blockIdx.x * epb + grp;
  const bool act = ci < count;
  const int col = act ? cols[ci] : 0;
  const int nqd = DIM == 3 ? nq * nq : nq;
  double *sB = lds, *sBd = lds + nq * N1;
  Carve cv{lds + 2 * nq * N1 + grp * per};
  double *se = cv.take(NH), *sp = cv.take(NH), *sw = cv.take(NH), *sk = cv.take(NH), *sd = cv.take(NH);
  // adjoints at the Gauss points: eta value, eta_xi, eta_eta, phi_xi, phi_eta, w
  double *Qe = cv.take(nqd), *Qex = cv.take(nqd), *Qey = cv.take(nqd), *Qpx = cv.take(nqd), *Qpy = cv.take(nqd),
         *Qw = cv.take(nqd);
  for (int k = threadIdx.x; k < nq * N1; k += kSqThreads) {
    sB[k] = Bg[k];
    sBd[k] = Bdg[k];
  }
  for (int t = tid; act && t < NH; t += tpe) {
    const int hn = eh_nodes[(int64_t)col * NH + t];
    se[t] = eta[hn];
    sp[t] = phs[hn];
    sw[t] = wv[hn];
    sk[t] = bbar[hn];
    sd[t] = bbar[n_s + hn];
  }
  __syncthreads();
  const int64_t mb = (int64_t)col * nqd;
  // the adjoint of one Gauss point, from the forward values there
  auto point = [&](int k, double ev, double exi, double eet, double pxi, double pet, double w, double kb,
                   double db) {
    double A00, A01, A10, A11, wd;
    if constexpr (DIM == 3) {
      A00 = met[0 * mstride + mb + k];
      A01 = met[1 * mstride + mb + k];
      A10 = met[2 * mstride + mb + k];
      A11 = met[3 * mstride + mb + k];
      wd = met[4 * mstride + mb + k];
    } else {
      A00 = met[0 * mstride + mb + k];
      A01 = A10 = A11 = 0.0;
      wd = met[1 * mstride + mb + k];
    }
    (void)ev;
    const double ex = A00 * exi + A10 * eet, ey = A01 * exi + A11 * eet;
    const double px = A00 * pxi + A10 * pet, py = A01 * pxi + A11 * pet;
    const double ee = ex * ex + ey * ey;
    const double Ekb = wd * kb, Edb = wd * db;   // adjoints of the two integrands
    const double gex = Ekb * (-px + 2.0 * w * ex) + Edb * w * w * ex;
    const double gey = Ekb * (-py + 2.0 * w * ey) + Edb * w * w * ey;
    const double gpx = -Ekb * ex - Edb * px;
    const double gpy = -Ekb * ey - Edb * py;
    Qe[k] = -g * Edb;
    Qw[k] = Ekb * (1.0 + ee) + Edb * w * (1.0 + ee);
    Qex[k] = A00 * gex + A01 * gey;
    Qey[k] = A10 * gex + A11 * gey;
    Qpx[k] = A00 * gpx + A01 * gpy;
    Qpy[k] = A10 * gpx + A11 * gpy;
  };
  double r_e = 0, r_p = 0, r_w = 0;
  int t_out = -1;
  if constexpr (DIM == 3) {
    double *Te = cv.take(N1 * nq), *Ted = cv.take(N1 * nq), *Tp = cv.take(N1 * nq), *Tpd = cv.take(N1 * nq),
           *Tw = cv.take(N1 * nq), *Tk = cv.take(N1 * nq), *Td = cv.take(N1 * nq);
    for (int k = tid; act && k < N1 * nq; k += tpe) {
      const int j = k / nq, qx = k - j * nq;
      double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, a6 = 0;
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        const double b = sB[qx * N1 + i], bdx = sBd[qx * N1 + i];
        a0 += b * se[j * N1 + i];
        a1 += bdx * se[j * N1 + i];
        a2 += b * sp[j * N1 + i];
        a3 += bdx * sp[j * N1 + i];
        a4 += b * sw[j * N1 + i];
        a5 += b * sk[j * N1 + i];
        a6 += b * sd[j * N1 + i];
      }
      Te[k] = a0;
      Ted[k] = a1;
      Tp[k] = a2;
      Tpd[k] = a3;
      Tw[k] = a4;
      Tk[k] = a5;
      Td[k] = a6;
    }
    __syncthreads();
    for (int k = tid; act && k < nqd; k += tpe) {
      const int qy = k / nq, qx = k - qy * nq;
      double ev = 0, exi = 0, eet = 0, pxi = 0, pet = 0, w = 0, kb = 0, db = 0;
#pragma unroll
      for (int j = 0; j < N1; ++j) {
        const double b = sB[qy * N1 + j], bdy = sBd[qy * N1 + j];
        const int o = j * nq + qx;
        ev += b * Te[o];
        exi += b * Ted[o];
        eet += bdy * Te[o];
        pxi += b * Tpd[o];
        pet += bdy * Tp[o];
        w += b * Tw[o];
        kb += b * Tk[o];
        db += b * Td[o];
      }
      point(k, ev, exi, eet, pxi, pet, w, kb, db);
    }
    __syncthreads();
    // transposed interpolation, along eta: (j, qx); reuse the T arrays
    double *Uae = Te, *Ube = Ted, *Uap = Tp, *Ubp = Tpd, *Uw = Tw;
    for (int k = tid; act && k < N1 * nq; k += tpe) {
      const int j = k / nq, qx = k - j * nq;
      double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
      for (int qy = 0; qy < nq; ++qy) {
        const double b = sB[qy * N1 + j], bdy = sBd[qy * N1 + j];
        const int o = qy * nq + qx;
        a0 += b * Qe[o] + bdy * Qey[o];
        a1 += b * Qex[o];
        a2 += bdy * Qpy[o];
        a3 += b * Qpx[o];
        a4 += b * Qw[o];
      }
      Uae[k] = a0;
      Ube[k] = a1;
      Uap[k] = a2;
      Ubp[k] = a3;
      Uw[k] = a4;
    }
    __syncthreads();
    if (act && tid < NH) {
      const int j = tid / N1, i = tid - j * N1;
      for (int qx = 0; qx < nq; ++qx) {
        const double b = sB[qx * N1 + i], bdx = sBd[qx * N1 + i];
        const int o = j * nq + qx;
        r_e += b * Uae[o] + bdx * Ube[o];
        r_p += b * Uap[o] + bdx * Ubp[o];
        r_w += b * Uw[o];
      }
      t_out = tid;
    }
  } else {
    for (int q = tid; act && q < nq; q += tpe) {
      double ev = 0, exi = 0, pxi = 0, w = 0, kb = 0, db = 0;
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        const double b = sB[q * N1 + i], bdx = sBd[q * N1 + i];
        ev += b * se[i];
        exi += bdx * se[i];
        pxi += bdx * sp[i];
        w += b * sw[i];
        kb += b * sk[i];
        db += b * sd[i];
      }
      point(q, ev, exi, 0.0, pxi, 0.0, w, kb, db);
    }
    __syncthreads();
    if (act && tid < NH) {
      for (int q = 0; q < nq; ++q) {
        const double b = sB[q * N1 + tid], bdx = sBd[q * N1 + tid];
        r_e += b * Qe[q] + bdx * Qex[q];
        r_p += bdx * Qpx[q];
        r_w += b * Qw[q];
      }
      t_out = tid;
    }
  }
  if (t_out >= 0) {
    const int64_t o = (int64_t)col * NH + t_out;
    const int hn = eh_nodes[o];
    const uint8_t fl = flags[o];
    const double se_ = acc_colour(scr, hn, r_e, fl);
    const double sp_ = acc_colour(scr + n_s, hn, r_p, fl);
    const double sw_ = acc_colour(scr + 2 * n_s, hn, r_w, fl);
    if (fl & kLast) {
      eta_bar[hn] += se_;
      phi_bar[hn] += sp_;
      w_bar[hn] += sw_;
    }
  }
}

// Chebyshev vector kernels on [2][n_s]; ml = lumped surface mass [n_s].
__global__ void k_sq_init(const double *__restrict__ b, const double *__restrict__ ml, double *__restrict__ x,
                          int64_t n_s) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < 2 * n_s; k += (int64_t)gridDim.x * blockDim.x)
    x[k] = b[k] / ml[k < n_s ? k : k - n_s];
}

__global__ void k_sq_start(const double *__restrict__ b, const double *__restrict__ ax, const double *__restrict__ ml,
                           double inv_theta, double *__restrict__ r, double *__restrict__ d, int64_t n_s) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < 2 * n_s;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double rr = b[k] - ax[k];
    r[k] = rr;
    d[k] = inv_theta * rr / ml[k < n_s ? k : k - n_s];
  }
}

__global__ void k_sq_cheb(double *__restrict__ x, double *__restrict__ r, double *__restrict__ d,
                          const double *__restrict__ ad, const double *__restrict__ ml, double c1, double c2,
                          int64_t n_s) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < 2 * n_s;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double dk = d[k];
    x[k] += dk;
    const double rr = r[k] - ad[k];
    r[k] = rr;
    d[k] = c1 * dk + c2 * rr / ml[k < n_s ? k : k - n_s];
  }
}

__global__ void k_sq_stage(RkStageArgs a, const double *__restrict__ k2, int64_t n_s) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_s; k += (int64_t)gridDim.x * blockDim.x)
    stage_update(a, k, k2[k], k2[n_s + k]);
}

__global__ void k_sq_pack(const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ out,
                          int64_t n_s) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_s; k += (int64_t)gridDim.x * blockDim.x) {
    out[k] = a[k];
    out[n_s + k] = b[k];
  }
}

int vec_blocks(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 4096); }

#define SQ_DISPATCH(DIMV, PV, CALL)                       \
  switch (PV) {                                           \
    case 1: { constexpr int P_ = 1; CALL; } break;        \
    case 2: { constexpr int P_ = 2; CALL; } break;        \
    case 3: { constexpr int P_ = 3; CALL; } break;        \
    case 4: { constexpr int P_ = 4; CALL; } break;        \
    case 5: { constexpr int P_ = 5; CALL; } break;        \
    case 6: { constexpr int P_ = 6; CALL; } break;        \
    case 7: { constexpr int P_ = 7; CALL; } break;        \
    case 8: { constexpr int P_ = 8; CALL; } break;        \
    default: return hipErrorInvalidValue;                 \
  }

// Per-element LDS (doubles) and the shared tables in front of them, per kernel.
struct SqLds {
  int table, per;
};
SqLds lds_rhs(const Ctx &c) {
  const int n1 = c.p + 1, nq = c.sq_nq, nh = c.nh;
  const int nqd = c.dim == 3 ? nq * nq : nq;
  return {2 * nq * n1, 3 * nh + 2 * nqd + (c.dim == 3 ? 7 * n1 * nq : 0)};
}
SqLds lds_mass(const Ctx &c) {
  const int n1 = c.p + 1, nq = c.sq_nq, nh = c.nh;
  const int nqd = c.dim == 3 ? nq * nq : nq;
  return {nq * n1, 2 * nh + 2 * nqd + (c.dim == 3 ? 2 * n1 * nq : 0)};
}
SqLds lds_vjp(const Ctx &c) {
  const int n1 = c.p + 1, nq = c.sq_nq, nh = c.nh;
  const int nqd = c.dim == 3 ? nq * nq : nq;
  return {2 * nq * n1, 5 * nh + 6 * nqd + (c.dim == 3 ? 7 * n1 * nq : 0)};
}

// Elements per block: 4 (one wave each) while the LDS fits in 64 KiB, else 2, else 1.
struct SqLaunch {
  int epb, per;
  size_t bytes;
};
SqLaunch sq_launch(const SqLds &l) {
  for (int epb = 4; epb > 1; epb /= 2) {
    const size_t bytes = (size_t)(l.table + epb * l.per) * sizeof(double);
    if (bytes <= 65536) return {epb, l.per, bytes};
  }
  return {1, l.per, (size_t)(l.table + l.per) * sizeof(double)};
}

template <int P, int DIM>
hipError_t sq_rhs_impl(Ctx &c, const double *eta, const double *phs, const double *w, double *b, hipStream_t s) {
  const int64_t ms = (int64_t)c.n_eh * (c.dim == 3 ? c.sq_nq * c.sq_nq : c.sq_nq);
  const SqLaunch L = sq_launch(lds_rhs(c));
  for (const auto &cr : c.colours) {
    if (cr.count == 0) continue;
    const int nb = (cr.count + L.epb - 1) / L.epb;
    k_sq_rhs<P, DIM><<<nb, kSqThreads, L.bytes, s>>>(eta, phs, w, c.d_eh_nodes, c.d_flags, c.d_cols + cr.offset,
                                                      cr.count, L.epb, L.per, c.d_sq_B, c.d_sq_Bd, c.sq_nq,
                                                      c.d_sq_met, ms, c.g, b, b + c.n_s);
  }
  return hipGetLastError();
}

template <int P, int DIM>
hipError_t sq_mass_impl(Ctx &c, const double *x, double *y, hipStream_t s) {
  const int64_t ms = (int64_t)c.n_eh * (c.dim == 3 ? c.sq_nq * c.sq_nq : c.sq_nq);
  const double *wdet = c.d_sq_met + (c.dim == 3 ? 4 : 1) * ms;
  const SqLaunch L = sq_launch(lds_mass(c));
  for (const auto &cr : c.colours) {
    if (cr.count == 0) continue;
    const int nb = (cr.count + L.epb - 1) / L.epb;
    k_sq_mass<P, DIM><<<nb, kSqThreads, L.bytes, s>>>(x, y, c.n_s, c.d_eh_nodes, c.d_flags, c.d_cols + cr.offset,
                                                       cr.count, L.epb, L.per, c.d_sq_B, c.sq_nq, wdet);
  }
  return hipGetLastError();
}

template <int P, int DIM>
hipError_t sq_vjp_impl(Ctx &c, const double *eta, const double *phs, const double *w, const double *bbar,
                       double *eta_bar, double *phi_bar, double *w_bar, hipStream_t s) {
  const int64_t ms = (int64_t)c.n_eh * (c.dim == 3 ? c.sq_nq * c.sq_nq : c.sq_nq);
  const SqLaunch L = sq_launch(lds_vjp(c));
  for (const auto &cr : c.colours) {
    if (cr.count == 0) continue;
    const int nb = (cr.count + L.epb - 1) / L.epb;
    k_sq_rhs_vjp<P, DIM><<<nb, kSqThreads, L.bytes, s>>>(
        eta, phs, w, bbar, c.n_s, c.d_eh_nodes, c.d_flags, c.d_cols + cr.offset, cr.count, L.epb, L.per, c.d_sq_B,
        c.d_sq_Bd, c.sq_nq, c.d_sq_met, ms, c.g, c.d_sq_scr, eta_bar, phi_bar, w_bar);
  }
  return hipGetLastError();
}

hipError_t sq_mass(Ctx &c, const double *x, double *y, hipStream_t s) {
  if (c.dim == 3) {
    SQ_DISPATCH(3, c.p, return (sq_mass_impl<P_, 3>(c, x, y, s)));
  } else {
    SQ_DISPATCH(2, c.p, return (sq_mass_impl<P_, 2>(c, x, y, s)));
  }
  return hipSuccess;
}

// Gauss-Legendre nodes and weights (Newton iteration on P_n from the classical cosine guesses).
void gauss_legendre(int n, double *x, double *w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) {
        p1 = z;
        p0 = 1.0;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) p0 = 1.0;
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[n - 1 - i] = z;   // ascending
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

}  // namespace

hipError_t launch_sq_rhs(Ctx &c, const double *eta, const double *phs, const double *w, double *b, hipStream_t s) {
  if (c.dim == 3) {
    SQ_DISPATCH(3, c.p, return (sq_rhs_impl<P_, 3>(c, eta, phs, w, b, s)));
  } else {
    SQ_DISPATCH(2, c.p, return (sq_rhs_impl<P_, 2>(c, eta, phs, w, b, s)));
  }
  return hipSuccess;
}

hipError_t launch_sq_rhs_vjp(Ctx &c, const double *eta, const double *phs, const double *w, const double *bbar,
                             double *eta_bar, double *phi_bar, double *w_bar, hipStream_t s) {
  if (c.dim == 3) {
    SQ_DISPATCH(3, c.p, return (sq_vjp_impl<P_, 3>(c, eta, phs, w, bbar, eta_bar, phi_bar, w_bar, s)));
  } else {
    SQ_DISPATCH(2, c.p, return (sq_vjp_impl<P_, 2>(c, eta, phs, w, bbar, eta_bar, phi_bar, w_bar, s)));
  }
  return hipSuccess;
}

// x = M^{-1} b for two fields [2][n_s] by the fixed-length preconditioned Chebyshev iteration.
// Uses c.d_sq_r, d_sq_d, d_sq_ad as work vectors; b and x must not overlap them.
hipError_t sq_solve(Ctx &c, const double *b, double *x, hipStream_t s) {
  const int64_t ns = c.n_s;
  const int nb = vec_blocks(2 * ns);
  const double theta = 0.5 * (c.sq_hi + c.sq_lo), delta = 0.5 * (c.sq_hi - c.sq_lo);
  const double sigma = theta / delta;
  k_sq_init<<<nb, 256, 0, s>>>(b, c.d_mlump_s, x, ns);
  hipError_t e = sq_mass(c, x, c.d_sq_ad, s);
  if (e != hipSuccess) return e;
  k_sq_start<<<nb, 256, 0, s>>>(b, c.d_sq_ad, c.d_mlump_s, 1.0 / theta, c.d_sq_r, c.d_sq_d, ns);
  double rho = 1.0 / sigma;
  for (int k = 0; k < c.sq_iters; ++k) {
    e = sq_mass(c, c.d_sq_d, c.d_sq_ad, s);
    if (e != hipSuccess) return e;
    const double rho_n = 1.0 / (2.0 * sigma - rho);
    k_sq_cheb<<<nb, 256, 0, s>>>(x, c.d_sq_r, c.d_sq_d, c.d_sq_ad, c.d_mlump_s, rho_n * rho, 2.0 * rho_n / delta,
                                  ns);
    rho = rho_n;
  }
  return hipGetLastError();
}

hipError_t launch_sq_stage(const RkStageArgs &a, const double *k2, int64_t n_s, hipStream_t s) {
  k_sq_stage<<<vec_blocks(n_s), 256, 0, s>>>(a, k2, n_s);
  return hipGetLastError();
}

hipError_t launch_sq_pack(const double *a, const double *b, double *out, int64_t n_s, hipStream_t s) {
  k_sq_pack<<<vec_blocks(n_s), 256, 0, s>>>(a, b, out, n_s);
  return hipGetLastError();
}

void sq_free(Ctx &c) {
  double **bufs[] = {&c.d_sq_B, &c.d_sq_Bd, &c.d_sq_met, &c.d_sq_b, &c.d_sq_x,
                     &c.d_sq_r, &c.d_sq_d,  &c.d_sq_ad,  &c.d_sq_scr};
  for (double **p : bufs) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
  c.sq_nq = 0;
}

// Tables, Gauss-point metrics and the Chebyshev interval for nq points per direction.
const char *sq_setup(Ctx &c, int nq) {
  const int p = c.p, n1 = p + 1, dim = c.dim;
  std::vector<double> xg(n1), wg(n1), D((size_t)n1 * n1), xq(nq), wq(nq);
  gll_host(p, xg.data(), wg.data(), D.data());
  gauss_legendre(nq, xq.data(), wq.data());
  std::vector<double> B((size_t)nq * n1), Bd((size_t)nq * n1, 0.0);
  for (int q = 0; q < nq; ++q)
    for (int i = 0; i < n1; ++i) {
      double l = 1.0;
      for (int m = 0; m < n1; ++m)
        if (m != i) l *= (xq[q] - xg[m]) / (xg[i] - xg[m]);
      B[(size_t)q * n1 + i] = l;
    }
  // l_i' has degree p - 1, so it equals its interpolant through the GLL nodes: Bd = B D
  for (int q = 0; q < nq; ++q)
    for (int i = 0; i < n1; ++i) {
      double a = 0.0;
      for (int m = 0; m < n1; ++m) a += B[(size_t)q * n1 + m] * D[(size_t)m * n1 + i];
      Bd[(size_t)q * n1 + i] = a;
    }
  // Gauss-point metrics from the nodal Jacobian (its entries have degree <= p per direction,
  // so the degree-p interpolant through the GLL nodes reproduces them)
  const int nqd = dim == 3 ? nq * nq : nq;
  const int ncomp = dim == 3 ? 5 : 2;
  const int64_t ms = (int64_t)c.n_eh * nqd, hs = (int64_t)c.n_eh * c.nh;
  std::vector<double> met((size_t)ncomp * ms);
  double lo = 1e300, hi = 0.0;
  const double gam = std::pow((double)p / (2.0 * p + 1.0), dim - 1);
  for (int64_t e = 0; e < c.n_eh; ++e) {
    double dq_min = 1e300, dq_max = 0.0, dn_min = 1e300, dn_max = 0.0;
    for (int t = 0; t < c.nh; ++t) {
      const double dn = c.h_hm[(size_t)(dim == 3 ? 4 : 1) * hs + e * c.nh + t];
      dn_min = std::min(dn_min, dn);
      dn_max = std::max(dn_max, dn);
    }
    for (int k = 0; k < nqd; ++k) {
      double det;
      const size_t o = (size_t)e * nqd + k;
      if (dim == 3) {
        const int qy = k / nq, qx = k - qy * nq;
        double J[4] = {0, 0, 0, 0};   // xxi, xet, yxi, yet
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i) {
            const double wgt = B[(size_t)qy * n1 + j] * B[(size_t)qx * n1 + i];
            const size_t no = (size_t)e * c.nh + j * n1 + i;
            for (int a = 0; a < 4; ++a) J[a] += wgt * c.h_hm[(size_t)(5 + a) * hs + no];
          }
        det = J[0] * J[3] - J[1] * J[2];
        if (!(det > 0.0)) return "surface quadrature: non-positive Jacobian at a Gauss point";
        met[0 * ms + o] = J[3] / det;
        met[1 * ms + o] = -J[1] / det;
        met[2 * ms + o] = -J[2] / det;
        met[3 * ms + o] = J[0] / det;
        met[4 * ms + o] = wq[qy] * wq[qx] * det;
      } else {
        double xx = 0.0;
        for (int i = 0; i < n1; ++i) xx += B[(size_t)k * n1 + i] * c.h_hm[(size_t)1 * hs + e * c.nh + i];
        det = xx;
        if (!(det > 0.0)) return "surface quadrature: non-positive Jacobian at a Gauss point";
        met[0 * ms + o] = 1.0 / xx;
        met[1 * ms + o] = wq[k] * xx;
      }
      dq_min = std::min(dq_min, det);
      dq_max = std::max(dq_max, det);
    }
    lo = std::min(lo, gam * dq_min / dn_max);
    hi = std::max(hi, dq_max / dn_min);
  }
  sq_free(c);
  auto up = [](double **d, const std::vector<double> &h) {
    if (hipMalloc(d, h.size() * sizeof(double)) != hipSuccess) return false;
    return hipMemcpy(*d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
  };
  if (!up(&c.d_sq_B, B) || !up(&c.d_sq_Bd, Bd) || !up(&c.d_sq_met, met)) return "surface quadrature: allocation";
  double **vecs[] = {&c.d_sq_b, &c.d_sq_x, &c.d_sq_r, &c.d_sq_d, &c.d_sq_ad};
  for (double **v : vecs)
    if (hipMalloc(v, 2 * c.n_s * sizeof(double)) != hipSuccess) return "surface quadrature: allocation";
  if (hipMalloc(&c.d_sq_scr, 3 * c.n_s * sizeof(double)) != hipSuccess) return "surface quadrature: allocation";
  c.sq_lo = lo;
  c.sq_hi = hi;
  const double kappa = hi / lo;
  const double rho = (std::sqrt(kappa) - 1.0) / (std::sqrt(kappa) + 1.0);
  c.sq_iters = rho <= 0.0 ? 1 : (int)std::ceil(std::log(2.0 / 1e-15) / std::log(1.0 / rho));
  c.sq_nq = nq;
  return nullptr;
}

}  // namespace fnpf
