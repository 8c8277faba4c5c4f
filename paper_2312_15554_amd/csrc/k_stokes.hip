// Fused passes of the ADMM iteration for unit-cell Stokes flow (Section 3.1,
// Steps 1-4, with the adaptive penalties of Section 4.1).
//
// State kept on the device per voxel: u (= u^n, the previous velocity) and a.
// Steps 2 and 3 imply, exactly, that after one iteration a = 0 and ut = u in
// the pore while a = lambda and ut = b/(b+alpha) u in the solid (given
// a^0 = lambda^0 supported in the solid and u^0 = 0 there).  So ut and lambda
// are never stored; q lives only as its spectrum q-hat.
//
// One iteration n:
//   green  (last axis): r-hat + N g delta_k0 - i s q-hat -> Step 1 solved per
//           mode with M = (nu L + b) I + beta s s^T (Sherman-Morrison), Step 3
//           for q-hat, Parseval sums for |div u|, |div u - div u_prev|, |q|.
//   [y inverse in 3D]
//   local  (x rows): inverse x transform gives u^{n+1}; Steps 2-3 pointwise;
//           sums for the residuals; the last workgroup runs Step 4 and the
//           penalty update (eq. varying algorithm).
//   rhs    (x rows): r = b^{n+1} ut^{n+1} - a^{n+1}, forward x transform.
//   [y forward in 3D]
#include <algorithm>

#include "slab_common.hpp"
#include "stokes_finalize.hpp"

namespace acm {

struct GreenGeom {
  int dim;
  int nx, xh;
  int plane;   // pencils along the last axis
  int64_t nspec;
  int64_t ntot;
};

// Component c of the right-hand side of Step 1 at one mode (eq. FFT step1):
//   form 1: r-hat - i s_c q-hat (+ N g_c at k = 0: `g0`);
//   increment form: X-hat + i beta s_c div-hat, where X is the change of the
//   real-space part since the last solve and i beta s div-hat = -i s (q-hat -
//   q-hat_prev) + i (beta - beta_prev) s div-hat is the change of the
//   pressure term plus the change of beta s s^T applied to the last u-hat.
// Every green kernel calls this with the same operands, and the fused
// multiply-adds are explicit, so the kernels round the same way.
template <typename T>
__device__ __forceinline__ cplx<T> step1_rhs(cplx<T> r, T s, const cplx<T>& q, const cplx<T>& dp,
                                             T beta, bool incr, T g0) {
  if (incr) {
    const T bs = beta * s;
    r.x = fma(-bs, dp.y, r.x);
    r.y = fma(bs, dp.x, r.y);
  } else {
    r.x = fma(s, q.y, r.x) + g0;
    r.y = fma(-s, q.x, r.y);
  }
  return r;
}

template <typename T, int L, int NC, int VAR, int SPL>
__global__ __launch_bounds__((ColCfg<T, L, NC, VAR, SPL>::NT)) void k_stokes_green(
    StokesCellArgs one, const StokesCellArgs* __restrict__ many, GreenGeom gg, int par,
    const cplx<T>* __restrict__ tw_g, const T* __restrict__ sx, const T* __restrict__ lx,
    const T* __restrict__ sy, const T* __restrict__ ly, const T* __restrict__ sz,
    const T* __restrict__ lz) {
  using C = ColCfg<T, L, NC, VAR, SPL>;
  const StokesCellArgs ca = many ? many[blockIdx.z] : one;
  gmem<cplx<T>>* __restrict__ spec = as_global(reinterpret_cast<cplx<T>*>(ca.spec));
  gmem<cplx<T>>* __restrict__ qhat = as_global(reinterpret_cast<cplx<T>*>(ca.qhat));
  gmem<cplx<T>>* __restrict__ dhat = as_global(reinterpret_cast<cplx<T>*>(ca.dhat));
  gmem<double>* __restrict__ partials = as_global(ca.part);
  const StokesCtl* __restrict__ ctl = ca.ctl;
  constexpr int PS = L * C::TX;  // LDS pencil-set stride per field
  extern __shared__ __align__(16) char smem_raw[];
  __shared__ double red[3 * 16];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  if (stokes_skip(ctl)) return;
  const cplx<T>* tw = twiddles_to_lds<T, C::NT, Plan<L>::tw_total>(lds + NC * PS, tw_g);
  const T beta = (T)ctl->st[par].psi[1];
  const T bpen = (T)ctl->st[par].psi[2];
  const T nu = (T)ctl->nu;
  const bool incr = ctl->st[par].incr != 0;
  const int P = gg.plane;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int f0 = tile * C::TX;

  gather_to_lds<cplx<T>, C::NT, NC * PS>(lds, NC * PS, [&](int e) {
    const int c = e / PS, rem = e - c * PS;
    const int i = rem / C::TX, col = rem - i * C::TX;
    const int f = f0 + col;
    cplx<T> v = cmake<T>(T(0), T(0));
    if (f < P) v = spec[c * gg.nspec + (int64_t)i * P + f];
    return v;
  });
  // q-hat and the previous div-hat of this thread's modes, fetched before the
  // forward transform so that their latency overlaps it
  constexpr int MPT = (PS + C::NT - 1) / C::NT;
  cplx<T> qpre[MPT], dpre[MPT];
#pragma unroll
  for (int r = 0; r < MPT; ++r) {
    const int e = threadIdx.x + r * C::NT;
    const int i = e / C::TX, col = e - i * C::TX;
    const int f = f0 + col;
    if (e < PS && f < P) {
      qpre[r] = qhat[(int64_t)i * P + f];
      dpre[r] = dhat[(int64_t)i * P + f];
    }
  }
  __syncthreads();
  // transform threads: (field, t, column) with SPL, else (t, column) over all fields
  const int fc = SPL ? threadIdx.x / (C::TPP * C::TX) : 0;
  const int tr = SPL ? threadIdx.x % (C::TPP * C::TX) : threadIdx.x;
  const int t = tr / C::TX, colt = tr % C::TX;
  const bool act = fc < NC && t < C::TPP && f0 + colt < P;
  cplx<T>* const pen = lds + (act ? fc : 0) * PS + colt;
  if constexpr (SPL)
    PencilFFT<T, L, 1, -1>::run_lds(t, act, pen, PS, C::TX, tw);
  else
    PencilFFT<T, L, NC, -1>::run_lds(t, act, pen, PS, C::TX, tw);
  __syncthreads();

  double acc[3] = {0.0, 0.0, 0.0};
  const T inv_ntot = T(1.0 / (double)gg.ntot);
#pragma unroll
  for (int r = 0; r < MPT; ++r) {
    const int e = threadIdx.x + r * C::NT;
    if (e >= PS) continue;
    const int i = e / C::TX, col = e - i * C::TX;
    const int f = f0 + col;
    if (f >= P) continue;
    int kx, ky, kz;
    if (NC == 3) {
      kx = f % gg.xh;
      ky = f / gg.xh;
      kz = i;
    } else {
      kx = f;
      ky = i;
      kz = 0;
    }
    T s[NC];
    s[0] = sx[kx];
    s[1] = sy[ky];
    T Lk = lx[kx] + ly[ky];
    if constexpr (NC == 3) {
      s[2] = sz[kz];
      Lk += lz[kz];
    }
    const double w = (kx == 0 || 2 * kx == gg.nx) ? 1.0 : 2.0;
    const int64_t mi = (int64_t)i * P + f;
    const cplx<T> q = qpre[r];
    const cplx<T> dp = dpre[r];
    cplx<T> R[NC];
    const bool k0 = (kx == 0 && ky == 0 && kz == 0);
#pragma unroll
    for (int c = 0; c < NC; ++c)
      R[c] = step1_rhs<T>(lds[c * PS + e], s[c], q, dp, beta, incr,
                          k0 ? (T)((double)gg.ntot * ctl->g[c]) : T(0));
    const T c0 = nu * Lk + bpen;
    cplx<T> sr = cmake<T>(T(0), T(0));
    T ss = T(0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      sr.x += s[c] * R[c].x;
      sr.y += s[c] * R[c].y;
      ss += s[c] * s[c];
    }
    const T den = c0 + beta * ss;
    const T inv_den = T(1) / den;
    const cplx<T> coef = cscale(sr, beta * inv_den);
    const T inv_c0 = T(1) / c0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      cplx<T> uc = cmake<T>((R[c].x - s[c] * coef.x) * inv_c0, (R[c].y - s[c] * coef.y) * inv_c0);
      lds[c * PS + e] = cscale(uc, inv_ntot);
    }
    // div u-hat = i s . u-hat = i (s . R) / den (its change in increment form)
    const cplx<T> di = cmake<T>(-sr.y * inv_den, sr.x * inv_den);
    const cplx<T> dl = incr ? cmake<T>(dp.x + di.x, dp.y + di.y) : di;
    const cplx<T> qn = cmake<T>(q.x - beta * dl.x, q.y - beta * dl.y);
    qhat[mi] = qn;
    dhat[mi] = dl;
    const double ddx = incr ? (double)di.x : (double)dl.x - (double)dp.x;
    const double ddy = incr ? (double)di.y : (double)dl.y - (double)dp.y;
    acc[0] += w * ((double)dl.x * dl.x + (double)dl.y * dl.y);
    acc[1] += w * (ddx * ddx + ddy * ddy);
    acc[2] += w * ((double)qn.x * qn.x + (double)qn.y * qn.y);
  }
  __syncthreads();
  if constexpr (SPL)
    PencilFFT<T, L, 1, 1>::run_lds(t, act, pen, PS, C::TX, tw);
  else
    PencilFFT<T, L, NC, 1>::run_lds(t, act, pen, PS, C::TX, tw);
  __syncthreads();
  scatter_from_lds<cplx<T>, C::NT, NC * PS>(lds, NC * PS, [&](int e, const cplx<T>& v) {
    const int c = e / PS, rem = e - c * PS;
    const int i = rem / C::TX, col = rem - i * C::TX;
    const int f = f0 + col;
    if (f < P) spec[c * gg.nspec + (int64_t)i * P + f] = v;
  });
  block_sum<3>(acc, red);
  if (threadIdx.x == 0) {
    partials[tile * 3 + 0] = acc[0];
    partials[tile * 3 + 1] = acc[1];
    partials[tile * 3 + 2] = acc[2];
  }
}

template <typename T, int M>
__global__ __launch_bounds__((RowCfg<T, M>::NT)) void k_stokes_local(
    StokesCellArgs one, const StokesCellArgs* __restrict__ many, int par, int ngreen, int nrows,
    int64_t ntot, int64_t nspec, const cplx<T>* __restrict__ tw, const cplx<T>* __restrict__ rtw) {
  using C = RowCfg<T, M>;
  const StokesCellArgs ca = many ? many[blockIdx.z] : one;
  const cplx<T>* __restrict__ spec = reinterpret_cast<const cplx<T>*>(ca.spec);
  T* __restrict__ u = reinterpret_cast<T*>(ca.u);
  T* __restrict__ a = reinterpret_cast<T*>(ca.a);
  const uint8_t* __restrict__ H = ca.H;
  const double* __restrict__ gpart = ca.part;
  double* __restrict__ lpart = ca.lpart;
  StokesCtl* ctl = ca.ctl;
  double* hist = ca.hist;
  constexpr int NX = 2 * M;
  extern __shared__ __align__(16) char smem_raw[];
  __shared__ double red[7 * 16];
  __shared__ int s_last;
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  T* ldsr = reinterpret_cast<T*>(smem_raw);
  if (stokes_skip(ctl)) return;
  const StokesState& S = ctl->st[par];
  const double al = S.psi[0], bb = S.psi[2];
  const T cc = (T)(bb / (bb + al));
  const T cp = (T)S.c_prev;
  const T ka = (T)(bb * al / (bb + al));
  const int field = blockIdx.y;
  const int row0 = blockIdx.x * C::RB;
  const int nr = min(C::RB, nrows - row0);
  const gmem<cplx<T>>* src = as_global(spec + field * nspec + (int64_t)row0 * (M + 1));
  gather_to_lds<cplx<T>, C::NT, C::RB * (M + 1)>(lds, nr * (M + 1), [&](int v) { return src[v]; });
  __syncthreads();
  const int row = threadIdx.x / C::TPP, t = threadIdx.x % C::TPP;
  rows_c2r_lds<T, M>(lds, 0, row, t, row < nr, tw, rtw);

  const int64_t off = field * ntot + (int64_t)row0 * NX;
  gmem<T>* ur = as_global(u + off);
  gmem<T>* ar = as_global(a + off);
  const gmem<uint8_t>* hr = as_global(H + (int64_t)row0 * NX);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int v = threadIdx.x; v < nr * NX; v += C::NT) {
    const int r = v / NX, x = v - r * NX;
    const T un = ldsr[r * 2 * C::RP + x];
    const T up = ur[v];
    const T du = un - up;
    acc[3] += (double)du * du;
    ur[v] = un;
    if (hr[v]) {
      const T an = ar[v] + ka * un;
      ar[v] = an;
      const T dd = cc * un - cp * up;
      acc[0] += (double)un * un;
      acc[1] += (double)dd * dd;
      acc[2] += (double)an * an;
    }
  }
  block_sum<4>(acc, red);
  const int nblk = gridDim.x * gridDim.y;
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  if (threadIdx.x == 0) {
    lpart[bid * 4 + 0] = acc[0];
    lpart[bid * 4 + 1] = acc[1];
    lpart[bid * 4 + 2] = acc[2];
    lpart[bid * 4 + 3] = acc[3];
    __threadfence();
    const unsigned prev = atomicAdd(&ctl->counter, 1u);
    s_last = (prev == (unsigned)(nblk - 1)) ? 1 : 0;
  }
  __syncthreads();
  if (s_last) {
    __threadfence();
    stokes_finalize(ctl, par, gpart, ngreen, lpart, nblk, ntot, hist, red);
  }
}

template <typename T, int M>
__global__ __launch_bounds__((RowCfg<T, M>::NT)) void k_stokes_rhs(
    StokesCellArgs one, const StokesCellArgs* __restrict__ many, int slot, int nrows, int64_t ntot,
    int64_t nspec, const cplx<T>* __restrict__ tw, const cplx<T>* __restrict__ rtw) {
  using C = RowCfg<T, M>;
  const StokesCellArgs ca = many ? many[blockIdx.z] : one;
  cplx<T>* __restrict__ spec = reinterpret_cast<cplx<T>*>(ca.spec);
  const T* __restrict__ u = reinterpret_cast<const T*>(ca.u);
  const T* __restrict__ a = reinterpret_cast<const T*>(ca.a);
  const uint8_t* __restrict__ H = ca.H;
  const StokesCtl* __restrict__ ctl = ca.ctl;
  constexpr int NX = 2 * M;
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  T* ldsr = reinterpret_cast<T*>(smem_raw);
  if (stokes_skip(ctl)) return;
  const StokesState& S = ctl->st[slot];
  const T bb = (T)S.psi[2];
  const T bcp = (T)(S.psi[2] * S.c_prev);
  const int field = blockIdx.y;
  const int row0 = blockIdx.x * C::RB;
  const int nr = min(C::RB, nrows - row0);
  const int64_t off = field * ntot + (int64_t)row0 * NX;
  const gmem<T>* ur = as_global(u + off);
  const gmem<T>* ar = as_global(a + off);
  const gmem<uint8_t>* hr = as_global(H + (int64_t)row0 * NX);
  for (int v = threadIdx.x; v < nr * NX; v += C::NT) {
    const int r = v / NX, x = v - r * NX;
    const T un = ur[v];
    ldsr[r * 2 * C::RP + x] = hr[v] ? (bcp * un - ar[v]) : (bb * un);
  }
  __syncthreads();
  const int row = threadIdx.x / C::TPP, t = threadIdx.x % C::TPP;
  rows_r2c_lds<T, M>(lds, 0, row, t, row < nr, tw, rtw);
  gmem<cplx<T>>* dst = as_global(spec + field * nspec + (int64_t)row0 * (M + 1));
  scatter_from_lds<cplx<T>, C::NT, C::RB * (M + 1)>(lds, nr * (M + 1),
                                                    [&](int v, const cplx<T>& x) { dst[v] = x; });
}


// ------------------------------------------------------------ row-step pass
// x-row form of the fused local pass, for cells whose xy-slab does not fit in
// LDS (and 2D cells on request): a persistent grid walks the row blocks of one
// field; for each block it loads the half-spectrum rows, takes them back to
// real space (u^{n+1}, or its change in increment form), applies Steps 2-3,
// forms the next Step 1's real-space input with the b of this iteration (r, or
// X in increment form), forward-transforms it and stores it over the rows it
// loaded.  One 7-value record per workgroup (its share of the green partials,
// then its 4 partial sums) goes to the Step 4 kernel; no cross-workgroup
// traffic, no fences.
template <typename T, int M>
__global__ __launch_bounds__((RowCfg<T, M>::NT)) void k_rows_step(
    StokesCellArgs ca, int par, int ngreen, int nfield, int nrows, int64_t ntot, int64_t nspec,
    const cplx<T>* __restrict__ tw, const cplx<T>* __restrict__ rtw) {
  using C = RowCfg<T, M>;
  using V = typename Vec4<T>::type;
  constexpr int NX = 2 * M;
  constexpr int QR = NX / 4;  // quads per row
  cplx<T>* __restrict__ spec = reinterpret_cast<cplx<T>*>(ca.spec);
  T* __restrict__ u = reinterpret_cast<T*>(ca.u);
  T* __restrict__ a = reinterpret_cast<T*>(ca.a);
  const uint8_t* __restrict__ H = ca.H;
  const double* __restrict__ gpart = ca.part;
  const StokesCtl* ctl = ca.ctl;
  extern __shared__ __align__(16) char smem_raw[];
  __shared__ double red[4 * 16];
  constexpr int kShare = 8;
  __shared__ double gsh[3 * kShare];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  T* ldsr = reinterpret_cast<T*>(smem_raw);
  if (stokes_skip(ctl)) return;
  const StokesState& cur = ctl->st[par];
  const double al = cur.psi[0], bb = cur.psi[2];
  const double ccd = bb / (bb + al);
  const T cc = (T)ccd;
  const T cp = (T)cur.c_prev;
  const T ka = (T)(bb * al / (bb + al));
  const T rb = (T)bb;
  const T rbc = (T)(bb * ccd);
  const T rbcp = (T)(bb * cur.c_prev);
  const bool incr = cur.incr != 0;
  // X only where Step 4 may pass it on (see k_slab_local)
  const bool xform = ctl->incr_enabled != 0 && cur.iter + 1 >= kIncrAfter;
  const int nblk = gridDim.x, bid = blockIdx.x;
  if (threadIdx.x < kShare) {
    const int g0 = (int)((int64_t)ngreen * bid / nblk), g1 = (int)((int64_t)ngreen * (bid + 1) / nblk);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int j = g0 + (int)threadIdx.x; j < g1; j += kShare) {
      s0 += gpart[j * 3 + 0];
      s1 += gpart[j * 3 + 1];
      s2 += gpart[j * 3 + 2];
    }
    gsh[threadIdx.x * 3 + 0] = s0;
    gsh[threadIdx.x * 3 + 1] = s1;
    gsh[threadIdx.x * 3 + 2] = s2;
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // the twiddles of the row transforms, read by every stage of every row
  // block, copied once into LDS after the rows (made visible by the first
  // barrier of the loop)
  constexpr int TWN = Plan<M>::tw_total + M + 1;
  cplx<T>* const ltw = lds + C::RB * C::RP;
  batched_copy<cplx<T>, C::NT, TWN>(
      TWN, [&](int e) { return e < Plan<M>::tw_total ? tw[e] : rtw[e - Plan<M>::tw_total]; },
      [&](int e, const cplx<T>& v) { ltw[e] = v; });
  const cplx<T>* const twl = ltw;
  const cplx<T>* const rtwl = ltw + Plan<M>::tw_total;
  // work list: (field, row block) pairs, field-major
  const int nrb = (nrows + C::RB - 1) / C::RB;
  const int row = threadIdx.x / C::TPP, t = threadIdx.x % C::TPP;
  for (int w = blockIdx.x; w < nfield * nrb; w += gridDim.x) {
    const int field = w / nrb, b = w - field * nrb;
    const int row0 = b * C::RB;
    const int nr = min(C::RB, nrows - row0);
    cplx<T>* rows = spec + field * nspec + (int64_t)row0 * (M + 1);
    static_assert(C::RP == M + 1, "rows are copied as one contiguous block");
    gather_to_lds<cplx<T>, C::NT, C::RB * (M + 1)>(lds, nr * (M + 1),
                                                   [&](int v) { return rows[v]; });
    __syncthreads();
    rows_c2r_lds<T, M>(lds, 0, row, t, row < nr, twl, rtwl);
    const int64_t off = field * ntot + (int64_t)row0 * NX;
    V* uq = reinterpret_cast<V*>(u + off);
    V* aq = reinterpret_cast<V*>(a + off);
    const uint32_t* hq = reinterpret_cast<const uint32_t*>(H + (int64_t)row0 * NX);
    for (int q = threadIdx.x; q < nr * QR; q += C::NT) {
      const int r = q / QR, x = 4 * (q - r * QR);
      // a is exactly zero in the pore, so it is loaded unconditionally
      const V upj = uq[q];
      const uint32_t hwj = hq[q];
      V aoj = aq[q];
      T* cell = ldsr + r * 2 * C::RP + x;
      V un = lds_ld4<V>(cell);
      if (incr) {
        un.x += upj.x;
        un.y += upj.y;
        un.z += upj.z;
        un.w += upj.w;
      }
      const T unv[4] = {un.x, un.y, un.z, un.w};
      const T upv[4] = {upj.x, upj.y, upj.z, upj.w};
      T dav[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double du = (double)unv[e] - (double)upv[e];
        acc[3] += du * du;
      }
      uq[q] = un;
      if (hwj) {
        T aov[4] = {aoj.x, aoj.y, aoj.z, aoj.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if ((hwj >> (8 * e)) & 0xffu) {
            const T an = aov[e] + ka * unv[e];
            dav[e] = an - aov[e];
            aov[e] = an;
            const T dd = cc * unv[e] - cp * upv[e];
            acc[0] += (double)unv[e] * unv[e];
            acc[1] += (double)dd * dd;
            acc[2] += (double)an * an;
          }
        }
        aoj.x = aov[0];
        aoj.y = aov[1];
        aoj.z = aov[2];
        aoj.w = aov[3];
        aq[q] = aoj;
      }
      V r4;
      if (xform) {
        r4.x = ((hwj & 0xffu) ? rbc * un.x - rbcp * upj.x : rb * (un.x - upj.x)) - dav[0];
        r4.y = ((hwj & 0xff00u) ? rbc * un.y - rbcp * upj.y : rb * (un.y - upj.y)) - dav[1];
        r4.z = ((hwj & 0xff0000u) ? rbc * un.z - rbcp * upj.z : rb * (un.z - upj.z)) - dav[2];
        r4.w = ((hwj & 0xff000000u) ? rbc * un.w - rbcp * upj.w : rb * (un.w - upj.w)) - dav[3];
      } else {
        r4.x = ((hwj & 0xffu) ? rbc : rb) * un.x - aoj.x;
        r4.y = ((hwj & 0xff00u) ? rbc : rb) * un.y - aoj.y;
        r4.z = ((hwj & 0xff0000u) ? rbc : rb) * un.z - aoj.z;
        r4.w = ((hwj & 0xff000000u) ? rbc : rb) * un.w - aoj.w;
      }
      lds_st4(cell, r4);
    }
    __syncthreads();
    rows_r2c_lds<T, M>(lds, 0, row, t, row < nr, twl, rtwl);
    for (int v = threadIdx.x; v < nr * (M + 1); v += C::NT) {
      const int r = v / (M + 1), k = v - r * (M + 1);
      rows[v] = lds[r * C::RP + k];
    }
    __syncthreads();
  }
  block_sum<4>(acc, red);
  if (threadIdx.x == 0) {
    double gs[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < kShare; ++k)
      for (int c = 0; c < 3; ++c) gs[c] += gsh[k * 3 + c];
    for (int c = 0; c < 3; ++c) ca.lpart[bid * 7 + c] = gs[c];
    for (int c = 0; c < 4; ++c) ca.lpart[bid * 7 + 3 + c] = acc[c];
  }
}

// After the Step 4 kernel: when Step 4 changed b, r = b' ut' - a' is formed
// again from the stored u, a and H with the new penalties (and Step 1 of the
// next iteration is in the paper's form); otherwise the rows already hold the
// next right-hand side and every workgroup exits at once.
template <typename T, int M>
__global__ __launch_bounds__((RowCfg<T, M>::NT)) void k_rows_rhs_cond(
    StokesCellArgs ca, int par, int nfield, int nrows, int64_t ntot, int64_t nspec,
    const cplx<T>* __restrict__ tw, const cplx<T>* __restrict__ rtw) {
  using C = RowCfg<T, M>;
  constexpr int NX = 2 * M;
  cplx<T>* __restrict__ spec = reinterpret_cast<cplx<T>*>(ca.spec);
  const T* __restrict__ u = reinterpret_cast<const T*>(ca.u);
  const T* __restrict__ a = reinterpret_cast<const T*>(ca.a);
  const uint8_t* __restrict__ H = ca.H;
  const StokesCtl* __restrict__ ctl = ca.ctl;
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  T* ldsr = reinterpret_cast<T*>(smem_raw);
  if (ctl->hold) return;
  const StokesState& nx = ctl->st[par ^ 1];
  if (nx.done || nx.psi[2] == ctl->st[par].psi[2]) return;
  const T bb = (T)nx.psi[2];
  const T bcp = (T)(nx.psi[2] * nx.c_prev);
  const int nrb = (nrows + C::RB - 1) / C::RB;
  const int row = threadIdx.x / C::TPP, t = threadIdx.x % C::TPP;
  for (int w = blockIdx.x; w < nfield * nrb; w += gridDim.x) {
    const int field = w / nrb, b = w - field * nrb;
    const int row0 = b * C::RB;
    const int nr = min(C::RB, nrows - row0);
    const int64_t off = field * ntot + (int64_t)row0 * NX;
    for (int v = threadIdx.x; v < nr * NX; v += C::NT) {
      const int r = v / NX, x = v - r * NX;
      const T un = u[off + v];
      ldsr[r * 2 * C::RP + x] = H[(int64_t)row0 * NX + v] ? (bcp * un - a[off + v]) : (bb * un);
    }
    __syncthreads();
    rows_r2c_lds<T, M>(lds, 0, row, t, row < nr, tw, rtw);
    cplx<T>* dst = spec + field * nspec + (int64_t)row0 * (M + 1);
    for (int v = threadIdx.x; v < nr * (M + 1); v += C::NT) {
      const int r = v / (M + 1), k = v - r * (M + 1);
      dst[v] = lds[r * C::RP + k];
    }
    __syncthreads();
  }
}

// Register-resident variant of the green pass (lengths whose plan allows the
// register FFT): every thread loads the pencil elements it owns straight from
// global memory, the forward transform, the per-mode operator and the inverse
// transform run on registers (LDS only between transform stages), and the
// results are stored straight back.
template <typename T, int L, int NC, int VAR>
__global__ __launch_bounds__((ColCfg<T, L, NC, VAR>::NT)) void k_stokes_green_reg(
    StokesCellArgs one, const StokesCellArgs* __restrict__ many, GreenGeom gg, int par,
    const cplx<T>* __restrict__ tw, const T* __restrict__ sx, const T* __restrict__ lx,
    const T* __restrict__ sy, const T* __restrict__ ly, const T* __restrict__ sz,
    const T* __restrict__ lz) {
  using C = ColCfg<T, L, NC, VAR>;
  constexpr int PS = L * C::TX;
  constexpr int TPP = C::TPP;
  constexpr int EPT = L / TPP;
  const StokesCellArgs ca = many ? many[blockIdx.z] : one;
  gmem<cplx<T>>* __restrict__ spec = as_global(reinterpret_cast<cplx<T>*>(ca.spec));
  gmem<cplx<T>>* __restrict__ qhat = as_global(reinterpret_cast<cplx<T>*>(ca.qhat));
  gmem<cplx<T>>* __restrict__ dhat = as_global(reinterpret_cast<cplx<T>*>(ca.dhat));
  gmem<double>* __restrict__ partials = as_global(ca.part);
  const StokesCtl* __restrict__ ctl = ca.ctl;
  extern __shared__ __align__(16) char smem_raw[];
  __shared__ double red[3 * 16];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  if (stokes_skip(ctl)) return;
  const T beta = (T)ctl->st[par].psi[1];
  const T bpen = (T)ctl->st[par].psi[2];
  const T nu = (T)ctl->nu;
  const bool incr = ctl->st[par].incr != 0;
  const int P = gg.plane;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int f0 = tile * C::TX;
  const int t = threadIdx.x / C::TX, col = threadIdx.x % C::TX;
  const int f = f0 + col;
  const bool act = t < TPP && f < P;

  const cplx<T>* twl = twiddles_to_lds<T, C::NT, Plan<L>::tw_total>(lds + NC * PS, tw);
  // the column's modes and, per element, the symbols of the transformed axis
  // are loaded with the data, before the forward transform hides their latency
  int kx = f, ky = 0;
  if (NC == 3) {
    kx = f % gg.xh;
    ky = f / gg.xh;
  }
  const T* sl = NC == 3 ? sz : sy;  // symbols of the transformed axis
  const T* ll = NC == 3 ? lz : ly;
  cplx<T> v[NC][EPT], qv[EPT], dv[EPT];
  T sv[EPT], lv[EPT];
  T sx0 = T(0), sy0 = T(0), L01 = T(0);
  if (act) {
    sx0 = sx[kx];
    sy0 = sy[ky];
    L01 = lx[kx] + (NC == 3 ? ly[ky] : T(0));
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int64_t mi = (int64_t)(t + m * TPP) * P + f;
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c][m] = spec[c * gg.nspec + mi];
      qv[m] = qhat[mi];
      dv[m] = dhat[mi];
      sv[m] = sl[t + m * TPP];
      lv[m] = ll[t + m * TPP];
    }
  }
  RegFFT<T, L, NC, -1>::run(t, act, v, lds + col, PS, C::TX, twl);

  double acc[3] = {0.0, 0.0, 0.0};
  const T inv_ntot = T(1.0 / (double)gg.ntot);
  if (act) {
    const double w = (kx == 0 || 2 * kx == gg.nx) ? 1.0 : 2.0;
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int i = t + m * TPP;  // index along the transformed (last) axis
      const int kz = NC == 3 ? i : 0;
      if (NC != 3) ky = i;
      T s[NC];
      s[0] = sx0;
      T Lk;
      if constexpr (NC == 3) {
        s[1] = sy0;
        s[2] = sv[m];
        Lk = L01 + lv[m];
      } else {
        s[1] = sv[m];
        Lk = L01 + lv[m];
      }
      const cplx<T> q = qv[m];
      const cplx<T> dp = dv[m];
      const bool k0 = (kx == 0 && ky == 0 && kz == 0);
      cplx<T> R[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c)
        R[c] = step1_rhs<T>(v[c][m], s[c], q, dp, beta, incr,
                            k0 ? (T)((double)gg.ntot * ctl->g[c]) : T(0));
      const T c0 = nu * Lk + bpen;
      cplx<T> sr = cmake<T>(T(0), T(0));
      T ss = T(0);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        sr.x += s[c] * R[c].x;
        sr.y += s[c] * R[c].y;
        ss += s[c] * s[c];
      }
      const T inv_den = T(1) / (c0 + beta * ss);
      const cplx<T> coef = cscale(sr, beta * inv_den);
      const T inv_c0 = T(1) / c0;
#pragma unroll
      for (int c = 0; c < NC; ++c)
        v[c][m] = cscale(cmake<T>((R[c].x - s[c] * coef.x) * inv_c0, (R[c].y - s[c] * coef.y) * inv_c0),
                         inv_ntot);
      const cplx<T> di = cmake<T>(-sr.y * inv_den, sr.x * inv_den);
      const cplx<T> dl = incr ? cmake<T>(dp.x + di.x, dp.y + di.y) : di;
      const cplx<T> qn = cmake<T>(q.x - beta * dl.x, q.y - beta * dl.y);
      const int64_t mi = (int64_t)i * P + f;
      qhat[mi] = qn;
      dhat[mi] = dl;
      const double ddx = incr ? (double)di.x : (double)dl.x - (double)dp.x;
      const double ddy = incr ? (double)di.y : (double)dl.y - (double)dp.y;
      acc[0] += w * ((double)dl.x * dl.x + (double)dl.y * dl.y);
      acc[1] += w * (ddx * ddx + ddy * ddy);
      acc[2] += w * ((double)qn.x * qn.x + (double)qn.y * qn.y);
    }
  }
  __syncthreads();  // the forward transform's last LDS reads are complete
  RegFFT<T, L, NC, 1>::run(t, act, v, lds + col, PS, C::TX, twl);
  if (act) {
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      const int64_t mi = (int64_t)(t + m * TPP) * P + f;
#pragma unroll
      for (int c = 0; c < NC; ++c) spec[c * gg.nspec + mi] = v[c][m];
    }
  }
  block_sum<3>(acc, red);
  if (threadIdx.x == 0) {
    partials[tile * 3 + 0] = acc[0];
    partials[tile * 3 + 1] = acc[1];
    partials[tile * 3 + 2] = acc[2];
  }
}

// ------------------------------------------------------------------ launchers
template <int L, typename T, int VAR>
static int green_blocks_for(const Geom& g) {
  if (g.dim == 3)
    return (int)((g.plane + ColCfg<T, L, 3, VAR>::TX - 1) / ColCfg<T, L, 3, VAR>::TX);
  return (int)((g.plane + ColCfg<T, L, 2, VAR>::TX - 1) / ColCfg<T, L, 2, VAR>::TX);
}

template <int L, typename T>
static int green_blocks_var(const Geom& g, int variant) {
  // register-resident (3, 4) and field-split (5, 6) kernels use the tile
  // widths of variants 0 and 1
  if (variant == 3 || variant == 5) variant = 0;
  if (variant == 4 || variant == 6) variant = 1;
  if (variant == 1) return green_blocks_for<L, T, 1>(g);
  if (variant == 2) return green_blocks_for<L, T, 2>(g);
  return green_blocks_for<L, T, 0>(g);
}

int stokes_green_blocks(const Geom& g, int prec_bytes, int variant) {
  switch (g.last_n) {
#define CASE(LL)                                                                                \
  case LL:                                                                                      \
    return prec_bytes == 8 ? green_blocks_var<LL, double>(g, variant)                           \
                           : green_blocks_var<LL, float>(g, variant);
    ACM_COL_LENGTHS(CASE)
#undef CASE
    default:
      return -1;
  }
}

int stokes_local_blocks(const Geom& g, int prec_bytes) {
  switch (g.nx / 2) {
#define CASE(M)                                                                               \
  case M: {                                                                                   \
    const int rb = prec_bytes == 8 ? RowCfg<double, M>::RB : RowCfg<float, M>::RB;            \
    return (int)((g.nrows + rb - 1) / rb) * g.dim;                                            \
  }
    ACM_ROW_LENGTHS(CASE)
#undef CASE
    default:
      return -1;
  }
}

template <typename T, int LL, int NC, int VAR, bool REG, int SPL = 0>
static hipError_t green_launch(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                               const StokesCellArgs* many, int ncells, int par, int* nblocks,
                               hipStream_t s) {
  using C = ColCfg<T, LL, NC, VAR, SPL>;
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  const T* rt = tb.rtab;
  GreenGeom gg{g.dim, g.nx, g.xh, (int)g.plane, g.nspec, g.ntot};
  const cplx<T>* tw = ct + (g.dim == 3 ? tb.off.tw_z : tb.off.tw_y);
  const int nb = (int)((g.plane + C::TX - 1) / C::TX);
  if (nblocks) *nblocks = nb;
  if constexpr (REG)
    ACM_LAUNCH((k_stokes_green_reg<T, LL, NC, VAR>), dim3(nb, 1, ncells), dim3(C::NT),
                       C::LDS_BYTES + Plan<LL>::tw_total * (int)sizeof(cplx<T>), s, one, many, gg,
                       par, tw, rt + tb.off.sx, rt + tb.off.lx, rt + tb.off.sy, rt + tb.off.ly,
                       rt + tb.off.sz, rt + tb.off.lz);
  else
    ACM_LAUNCH((k_stokes_green<T, LL, NC, VAR, SPL>), dim3(nb, 1, ncells), dim3(C::NT),
                       C::LDS_BYTES + Plan<LL>::tw_total * (int)sizeof(cplx<T>), s, one, many, gg,
                       par, tw, rt + tb.off.sx, rt + tb.off.lx, rt + tb.off.sy, rt + tb.off.ly,
                       rt + tb.off.sz, rt + tb.off.lz);
  return hipGetLastError();
}

template <typename T, int LL, int NC>
static hipError_t green_var(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                            const StokesCellArgs* many, int ncells, int par, int variant,
                            int* nblocks, hipStream_t s) {
  constexpr bool reg_ok = RegPlanOk<LL>::value();
  if (variant == 3 || variant == 4) {
    if constexpr (reg_ok) {
      if (variant == 3) return green_launch<T, LL, NC, 0, true>(g, tb, one, many, ncells, par, nblocks, s);
      return green_launch<T, LL, NC, 1, true>(g, tb, one, many, ncells, par, nblocks, s);
    }
    variant -= 3;  // radix-3 plans: LDS-staged kernel of the same tile width
  }
  if (variant == 5) return green_launch<T, LL, NC, 0, false, 1>(g, tb, one, many, ncells, par, nblocks, s);
  if (variant == 6) return green_launch<T, LL, NC, 1, false, 1>(g, tb, one, many, ncells, par, nblocks, s);
  if (variant == 1) return green_launch<T, LL, NC, 1, false>(g, tb, one, many, ncells, par, nblocks, s);
  if (variant == 2) return green_launch<T, LL, NC, 2, false>(g, tb, one, many, ncells, par, nblocks, s);
  return green_launch<T, LL, NC, 0, false>(g, tb, one, many, ncells, par, nblocks, s);
}

template <typename T>
hipError_t launch_stokes_green(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                               const StokesCellArgs* many, int ncells, int par, int variant,
                               int* nblocks, hipStream_t s) {
  switch (g.last_n) {
#define CASE(LL)                                                                     \
  case LL:                                                                           \
    if (g.dim == 3) return green_var<T, LL, 3>(g, tb, one, many, ncells, par, variant, nblocks, s); \
    return green_var<T, LL, 2>(g, tb, one, many, ncells, par, variant, nblocks, s);
    ACM_COL_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_stokes_local(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                               const StokesCellArgs* many, int ncells, int par, int green_blocks,
                               hipStream_t s) {
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  switch (g.nx / 2) {
#define CASE(M)                                                                               \
  case M: {                                                                                   \
    using C = RowCfg<T, M>;                                                                   \
    dim3 grid((unsigned)((g.nrows + C::RB - 1) / C::RB), (unsigned)g.dim, (unsigned)ncells);  \
    ACM_LAUNCH((k_stokes_local<T, M>), grid, dim3(C::NT), C::LDS_BYTES, s, one, many, par,  \
                       green_blocks, (int)g.nrows, g.ntot, g.nspec, ct + tb.off.tw_x,         \
                       ct + tb.off.rtw);                                                      \
    return hipGetLastError();                                                                 \
  }
    ACM_ROW_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_stokes_rhs(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                             const StokesCellArgs* many, int ncells, int slot, hipStream_t s) {
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  switch (g.nx / 2) {
#define CASE(M)                                                                               \
  case M: {                                                                                   \
    using C = RowCfg<T, M>;                                                                   \
    dim3 grid((unsigned)((g.nrows + C::RB - 1) / C::RB), (unsigned)g.dim, (unsigned)ncells);  \
    ACM_LAUNCH((k_stokes_rhs<T, M>), grid, dim3(C::NT), C::LDS_BYTES, s, one, many, slot, \
                       (int)g.nrows, g.ntot, g.nspec, ct + tb.off.tw_x, ct + tb.off.rtw);     \
    return hipGetLastError();                                                                 \
  }
    ACM_ROW_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

// Row-step pass: a persistent grid of kRowsStepWG workgroups (what the
// device holds at once: 5 of the 256-thread workgroups per CU at the kernel's
// register count, on 256 CUs) walks the (field, row block) work list, so
// that the Step 4 kernel sums a bounded number of records.
constexpr int kRowsStepWG = 1280;
constexpr int kRowsRhsWG = 512;

int rows_step_blocks(const Geom& g, int prec_bytes) {
  switch (g.nx / 2) {
#define CASE(M)                                                                               \
  case M: {                                                                                   \
    const int rb = prec_bytes == 8 ? RowCfg<double, M>::RB : RowCfg<float, M>::RB;            \
    const int nrb = (int)((g.nrows + rb - 1) / rb);                                           \
    return std::min(nrb * g.dim, kRowsStepWG);                                                \
  }
    ACM_ROW_LENGTHS(CASE)
#undef CASE
    default:
      return -1;
  }
}

template <typename T>
hipError_t launch_rows_step(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                            int par, int green_blocks, hipStream_t s) {
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  const int nb = rows_step_blocks(g, (int)sizeof(T));
  if (nb <= 0) return hipErrorInvalidValue;
  switch (g.nx / 2) {
#define CASE(M)                                                                               \
  case M: {                                                                                   \
    using C = RowCfg<T, M>;                                                                   \
    constexpr int lds_bytes = C::LDS_BYTES + (Plan<M>::tw_total + M + 1) * (int)sizeof(cplx<T>); \
    ACM_LAUNCH((k_rows_step<T, M>), dim3((unsigned)nb), dim3(C::NT), lds_bytes, s, one,      \
               par, green_blocks, g.dim, (int)g.nrows, g.ntot, g.nspec, ct + tb.off.tw_x,     \
               ct + tb.off.rtw);                                                              \
    return hipGetLastError();                                                                 \
  }
    ACM_ROW_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_rows_rhs_cond(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                                int par, hipStream_t s) {
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  switch (g.nx / 2) {
#define CASE(M)                                                                               \
  case M: {                                                                                   \
    using C = RowCfg<T, M>;                                                                   \
    const int nrb = (int)((g.nrows + C::RB - 1) / C::RB);                                     \
    dim3 grid((unsigned)std::min(nrb * g.dim, kRowsRhsWG));                                   \
    ACM_LAUNCH((k_rows_rhs_cond<T, M>), grid, dim3(C::NT), C::LDS_BYTES, s, one, par, g.dim, \
               (int)g.nrows, g.ntot, g.nspec, ct + tb.off.tw_x, ct + tb.off.rtw);             \
    return hipGetLastError();                                                                 \
  }
    ACM_ROW_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

#define INST(T)                                                                                \
  template hipError_t launch_rows_step<T>(const Geom&, const DevTables<T>&,                    \
                                          const StokesCellArgs&, int, int, hipStream_t);       \
  template hipError_t launch_rows_rhs_cond<T>(const Geom&, const DevTables<T>&,                \
                                              const StokesCellArgs&, int, hipStream_t);        \
  template hipError_t launch_stokes_green<T>(const Geom&, const DevTables<T>&,                 \
                                             const StokesCellArgs&, const StokesCellArgs*, int, \
                                             int, int, int*, hipStream_t);                     \
  template hipError_t launch_stokes_local<T>(const Geom&, const DevTables<T>&,                 \
                                             const StokesCellArgs&, const StokesCellArgs*, int, \
                                             int, int, hipStream_t);                           \
  template hipError_t launch_stokes_rhs<T>(const Geom&, const DevTables<T>&,                   \
                                           const StokesCellArgs&, const StokesCellArgs*, int,   \
                                           int, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace acm
