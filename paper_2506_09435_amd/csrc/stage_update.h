// ERK4 stage combination for one surface node (Sec. 3.2), shared by the fused lumped RHS kernel
// and the stage kernel of the consistent free-surface form; after the last stage, the relaxation
// zones (Sec. 3.3).
#pragma once

#include "fnpf_internal.h"

namespace fnpf {

__device__ __forceinline__ void stage_update(const RkStageArgs &a, int64_t hn, double ke, double kp) {
  if (a.stage < 0) {
    a.out_e[hn] = ke;
    a.out_p[hn] = kp;
    return;
  }
  const double ae = (a.stage == 0 ? 0.0 : a.acc_e[hn]) + a.bdt * ke;
  const double ap = (a.stage == 0 ? 0.0 : a.acc_p[hn]) + a.bdt * kp;
  if (a.stage < 3) {
    a.acc_e[hn] = ae;
    a.acc_p[hn] = ap;
    a.out_e[hn] = a.eta0[hn] + a.cdt * ke;
    a.out_p[hn] = a.phi0[hn] + a.cdt * kp;
    return;
  }
  double ne = a.eta0[hn] + ae;
  double np = a.phi0[hn] + ap;
  if (a.cr) {
    const double c = a.cr[hn];
    ne = (1.0 - c) * ne + c * (a.rc * a.ec[hn] + a.rs * a.es[hn]);
    np = (1.0 - c) * np + c * (a.rc * a.pc[hn] + a.rs * a.ps[hn]);
  }
  a.out_e[hn] = ne;
  a.out_p[hn] = np;
}

}  // namespace fnpf
