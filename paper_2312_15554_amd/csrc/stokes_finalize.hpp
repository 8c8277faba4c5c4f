// Step 4 of the ADMM (Section 3.1, eq. constrains with the tolerances of the
// same section) and the adaptive penalty update (Section 4.1, eq. varying
// algorithm), computed on the device from the partial sums of the passes.
#pragma once
#include "pass_common.hpp"

namespace acm {

// Totals of the green partials (3 per tile: |div u|^2, |div u - div u_prev|^2,
// |q|^2, Parseval-weighted) and the local partials (4 per workgroup: |H u|^2,
// |H (ut - ut_prev)|^2, |a|^2, |u - u_prev|^2) in a fixed order, so every
// workgroup that forms them gets the same bits.  The whole workgroup calls
// it; the totals are valid in thread 0.  `red` holds 7 * 16 doubles.
// U: tuples of each kind per thread whose loads are issued together, green
// and local ones in the same round, before any is added.
template <int U = 2>
__device__ __forceinline__ void stokes_sum_partials(const double* __restrict__ gpart, int ngreen,
                                                    const double* __restrict__ lpart, int nlocal,
                                                    double (&acc)[7], double* red) {
  const gmem<double>* gp = as_global(gpart);
  const gmem<double>* lp = as_global(lpart);
  for (int k = 0; k < 7; ++k) acc[k] = 0.0;
  const int nmax = ngreen > nlocal ? ngreen : nlocal;
  for (int j0 = threadIdx.x; j0 < nmax; j0 += U * blockDim.x) {
    double vg[U][3], vl[U][4];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int j = j0 + k * blockDim.x;
      const bool ig = j < ngreen, il = j < nlocal;
#pragma unroll
      for (int c = 0; c < 3; ++c) vg[k][c] = ig ? gp[j * 3 + c] : 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) vl[k][c] = il ? lp[j * 4 + c] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[c] += vg[k][c];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[3 + c] += vl[k][c];
    }
  }
  block_sum<7>(acc, red);
}

// Totals of the records of the two-launch slab local pass (7 per workgroup:
// its share of the green partials, then its 4 local partials), in a fixed
// order; valid in thread 0.  `red` holds 7 * 16 doubles.
template <int U>
__device__ __forceinline__ void stokes_sum_records(const double* __restrict__ rec, int nrec,
                                                   double (&acc)[7], double* red) {
  const gmem<double>* rp = as_global(rec);
  for (int k = 0; k < 7; ++k) acc[k] = 0.0;
  for (int j0 = threadIdx.x; j0 < nrec; j0 += U * blockDim.x) {
    double v[U][7];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int j = j0 + k * blockDim.x;
#pragma unroll
      for (int c = 0; c < 7; ++c) v[k][c] = j < nrec ? rp[j * 7 + c] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < U; ++k)
#pragma unroll
      for (int c = 0; c < 7; ++c) acc[c] += v[k][c];
  }
  block_sum<7>(acc, red);
}

// Step 4 and the penalty update: the state `nx` that follows `cur` given the
// totals.  Pure function of its inputs (one thread calls it).
__device__ __forceinline__ void stokes_step4(const StokesCtl* __restrict__ ctl,
                                             const StokesState& cur, const double (&tot)[7],
                                             int64_t ntot, StokesState& nx) {
  const double inv_n = 1.0 / (double)ntot;
  const double s_div = tot[0] * inv_n, s_ddiv = tot[1] * inv_n, s_q = tot[2] * inv_n;
  const double s_su2 = tot[3], s_sd = tot[4], s_a2 = tot[5], s_du = tot[6];
  const double al = cur.psi[0], be = cur.psi[1], bb = cur.psi[2];
  const double cc = bb / (bb + al);
  const double one_m_cc = al / (bb + al);
  const double nsu = sqrt(s_su2);
  const double rp[3] = {cc * nsu, sqrt(s_div), one_m_cc * nsu};
  const double rd[3] = {al * sqrt(s_sd), be * sqrt(s_ddiv), bb * sqrt(s_du)};
  const double mu[3] = {sqrt(s_a2), sqrt(s_q), sqrt(s_a2)};
  const double eps = ctl->eps;
  bool ok = true, finite = true;
  for (int k = 0; k < 3; ++k) {
    const double tp = ctl->sqrt_n[k] * eps + eps * fmax(rp[k], mu[k]);
    const double td = ctl->sqrt_n[k] * eps + eps * mu[k];
    nx.rp[k] = rp[k];
    nx.rd[k] = rd[k];
    nx.tp[k] = tp;
    nx.td[k] = td;
    nx.mu[k] = mu[k];
    nx.psi[k] = cur.psi[k];
    if (!(rp[k] <= tp && rd[k] <= td)) ok = false;
    if (!isfinite(rp[k]) || !isfinite(rd[k])) finite = false;
  }
  nx.iter = cur.iter + 1;
  nx.c_prev = cc;
  nx.done = 0;
  nx.status = 1;
  // divergence: a non-finite residual, or the sum of the six grown a
  // millionfold over its smallest value so far
  const double rsum = rp[0] + rp[1] + rp[2] + rd[0] + rd[1] + rd[2];
  nx.s_min = fmin(cur.s_min, rsum);
  if (nx.iter > 5 && rsum > 1e6 * nx.s_min) finite = false;
  if (!finite) {
    nx.done = 1;
    nx.status = -5;
  } else if (ok) {
    nx.done = 1;
    nx.status = 0;
  } else if (nx.iter >= ctl->max_iter) {
    nx.done = 1;
    nx.status = 1;
  } else if (ctl->adaptive) {
    for (int k = 0; k < 3; ++k) {
      if (rp[k] > ctl->tau[k] * rd[k])
        nx.psi[k] = ctl->phi[k] * cur.psi[k];
      else if (rd[k] > ctl->tau[k] * rp[k])
        nx.psi[k] = fmax(cur.psi[k] / ctl->phi[k], ctl->psi_min[k]);
    }
  }
  // the local pass formed X with this b: valid as long as b is kept.  The
  // increment form starts after the first kIncrAfter iterations: in the
  // increment form the rounding of each solve stays in u (it is never formed
  // again from a and q), so the large early increments are left to the
  // paper's form
  nx.incr = (ctl->incr_enabled && !nx.done && nx.psi[2] == cur.psi[2] && nx.iter >= kIncrAfter)
                ? 1 : 0;
}

// One record of the residual history ring: rp, rd, tp, td and the penalties
// the iteration used.
__device__ __forceinline__ void stokes_history(const StokesCtl* ctl, const StokesState& cur,
                                               const StokesState& nx, double* hist) {
  if (hist == nullptr || ctl->hist_cap <= 0) return;
  double* hrec = hist + ((nx.iter - 1) % ctl->hist_cap) * kHistDoubles;
  for (int k = 0; k < 3; ++k) {
    hrec[k] = nx.rp[k];
    hrec[3 + k] = nx.rd[k];
    hrec[6 + k] = nx.tp[k];
    hrec[9 + k] = nx.td[k];
    hrec[12 + k] = cur.psi[k];
  }
}

// Last-workgroup form (row passes, single-launch slab pass): sums, Step 4,
// writes slot par ^ 1 and the history, and re-arms the arrival counter.
__device__ __forceinline__ void stokes_finalize(StokesCtl* ctl, int par,
                                                const double* __restrict__ gpart, int ngreen,
                                                const double* __restrict__ lpart, int nlocal,
                                                int64_t ntot, double* hist, double* red) {
  double acc[7];
  stokes_sum_partials(gpart, ngreen, lpart, nlocal, acc, red);
  if (threadIdx.x != 0) return;
  const StokesState cur = ctl->st[par];
  StokesState nx;
  stokes_step4(ctl, cur, acc, ntot, nx);
  stokes_history(ctl, cur, nx, hist);
  ctl->st[par ^ 1] = nx;
  ctl->counter = 0u;
}

}  // namespace acm
