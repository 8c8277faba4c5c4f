// Step 4 of the ADMM (Section 3.1, eq. constrains with the tolerances of the
// same section) and the adaptive penalty update (Section 4.1, eq. varying
// algorithm), run by the last workgroup of the local pass on the device.
#pragma once
#include "pass_common.hpp"

namespace acm {

// Step 4 and the penalty update, run by the last workgroup of the local pass.
__device__ __forceinline__ void stokes_finalize(StokesCtl* ctl, const double* __restrict__ gpart, int ngreen,
                                const double* __restrict__ lpart, int nlocal, int64_t ntot,
                                double* hist, double* red) {
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int j = threadIdx.x; j < ngreen; j += blockDim.x) {
    acc[0] += gpart[j * 3 + 0];
    acc[1] += gpart[j * 3 + 1];
    acc[2] += gpart[j * 3 + 2];
  }
  for (int j = threadIdx.x; j < nlocal; j += blockDim.x) {
    acc[3] += lpart[j * 4 + 0];
    acc[4] += lpart[j * 4 + 1];
    acc[5] += lpart[j * 4 + 2];
    acc[6] += lpart[j * 4 + 3];
  }
  block_sum<7>(acc, red);
  if (threadIdx.x != 0) return;
  const double inv_n = 1.0 / (double)ntot;
  const double s_div = acc[0] * inv_n, s_ddiv = acc[1] * inv_n, s_q = acc[2] * inv_n;
  const double s_su2 = acc[3], s_sd = acc[4], s_a2 = acc[5], s_du = acc[6];
  const double al = ctl->psi[0], be = ctl->psi[1], bb = ctl->psi[2];
  const double cc = bb / (bb + al);
  const double one_m_cc = al / (bb + al);
  const double nsu = sqrt(s_su2);
  double rp[3] = {cc * nsu, sqrt(s_div), one_m_cc * nsu};
  double rd[3] = {al * sqrt(s_sd), be * sqrt(s_ddiv), bb * sqrt(s_du)};
  double mu[3] = {sqrt(s_a2), sqrt(s_q), sqrt(s_a2)};
  const double eps = ctl->eps;
  bool ok = true, finite = true;
  for (int k = 0; k < 3; ++k) {
    const double tp = ctl->sqrt_n[k] * eps + eps * fmax(rp[k], mu[k]);
    const double td = ctl->sqrt_n[k] * eps + eps * mu[k];
    ctl->rp[k] = rp[k];
    ctl->rd[k] = rd[k];
    ctl->tp[k] = tp;
    ctl->td[k] = td;
    ctl->mu[k] = mu[k];
    if (!(rp[k] <= tp && rd[k] <= td)) ok = false;
    if (!isfinite(rp[k]) || !isfinite(rd[k])) finite = false;
  }
  const int64_t it = ctl->iter + 1;
  ctl->iter = it;
  if (hist != nullptr && ctl->hist_cap > 0) {
    double* hrec = hist + ((it - 1) % ctl->hist_cap) * kHistDoubles;
    for (int k = 0; k < 3; ++k) {
      hrec[k] = rp[k];
      hrec[3 + k] = rd[k];
      hrec[6 + k] = ctl->tp[k];
      hrec[9 + k] = ctl->td[k];
      hrec[12 + k] = ctl->psi[k];
    }
  }
  ctl->c_prev = cc;
  if (!finite) {
    ctl->done = 1;
    ctl->status = -5;
  } else if (ok) {
    ctl->done = 1;
    ctl->status = 0;
  } else if (it >= ctl->max_iter) {
    ctl->done = 1;
    ctl->status = 1;
  } else if (ctl->adaptive) {
    for (int k = 0; k < 3; ++k) {
      if (rp[k] > ctl->tau[k] * rd[k])
        ctl->psi[k] = ctl->phi[k] * ctl->psi[k];
      else if (rd[k] > ctl->tau[k] * rp[k])
        ctl->psi[k] = fmax(ctl->psi[k] / ctl->phi[k], ctl->psi_min[k]);
    }
  }
  ctl->counter = 0u;
}

}  // namespace acm
