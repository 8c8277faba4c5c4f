// Fused xy-slab passes of the ADMM iteration for 3D cells whose z-slab of one
// field fits in LDS (ny * (nx/2 + 2) complex values, up to 150 KB).  One
// workgroup owns one (field, z) slab:
//   slab_local: load the half-spectrum slab, inverse y transform (columns),
//               inverse x transform (rows) -> u^{n+1}, Steps 2-3 pointwise
//               (Section 3.1), FP64 partial sums; then r = b ut^{n+1} -
//               a^{n+1} with the b of this iteration, forward x and y
//               transforms, store the slab in place of the one it loaded.
//   slab_rhs:   every workgroup forms Step 4 and the penalty update from the
//               partial sums.  Only when that changes b (a few per cent of
//               the iterations) is r formed again with the new b from the
//               stored u, a and H and transformed; otherwise the pass ends.
// r depends on the penalties only through b and the c of the iteration just
// done (its solid coefficient is b c_prev), so the speculative r is exactly
// the one the rhs pass would form whenever b is kept.
// This replaces the separate x-row and y-column passes of the general path
// and saves one HBM round trip of the spectra per direction of transform.
#include "slab_common.hpp"
#include "stokes_finalize.hpp"

namespace acm {

// Bound on the polls of the fused pass's gate (each poll sleeps briefly): a
// wait that long means the workgroups were not all resident, and the pass
// then gives up (ctl->fault) instead of hanging.
constexpr uint32_t kGatePolls = 1u << 22;

// Local pass (FUSED = false), or local and rhs passes of one cell in one
// launch (FUSED = true, a single cell, every workgroup resident).
template <typename T, int NX, int NY, bool FUSED>
__global__ __launch_bounds__((SlabCfg<T, NX, NY>::NT))
__attribute__((amdgpu_waves_per_eu(FUSED ? SlabCfg<T, NX, NY>::WPE_ONE
                                          : SlabCfg<T, NX, NY>::WPE))) void k_slab_local(
    StokesCellArgs one, const StokesCellArgs* __restrict__ many, int par, int ngreen,
    int64_t ntot, int64_t nspec, const cplx<T>* __restrict__ twx_g,
    const cplx<T>* __restrict__ twy_g, const cplx<T>* __restrict__ rtw_g) {
  using S = SlabCfg<T, NX, NY>;
  const StokesCellArgs ca = many ? many[blockIdx.z] : one;
  cplx<T>* __restrict__ spec = reinterpret_cast<cplx<T>*>(ca.spec);
  T* __restrict__ u = reinterpret_cast<T*>(ca.u);
  T* __restrict__ a = reinterpret_cast<T*>(ca.a);
  const uint8_t* __restrict__ H = ca.H;
  const double* __restrict__ gpart = ca.part;
  double* __restrict__ lpart = ca.lpart;
  StokesCtl* ctl = ca.ctl;
  double* hist = ca.hist;
  using V = typename Vec4<T>::type;
  extern __shared__ __align__(32) char smem_raw[];
  __shared__ double red[4 * 16];
  __shared__ double red7[7 * 16];
  __shared__ int s_last, s_go;
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  T* ldsr = reinterpret_cast<T*>(smem_raw);
  if (stokes_skip(ctl)) return;
  const uint32_t gate0 = FUSED ? ctl->gate : 0u;  // read before this workgroup arrives
  // Two-launch form: this workgroup's share of the green partials of the
  // iteration (records [g0, g1)) goes into its own record, so that Step 4
  // sums one record per local workgroup.  kShare threads sum it (fixed order)
  // into LDS while the slab loads are in flight.
  constexpr int kShare = 8;
  __shared__ double gsh[3 * kShare];
  const StokesState& cur = ctl->st[par];
  const double al = cur.psi[0], bb = cur.psi[2];
  const double ccd = bb / (bb + al);
  const T cc = (T)ccd;
  const T cp = (T)cur.c_prev;
  const T ka = (T)(bb * al / (bb + al));
  // r of the next Step 1 if Step 4 keeps b (it changes b in a few per cent of
  // the iterations): the coefficients the rhs pass would use then, in the
  // same arithmetic (c_prev of the next state is ccd)
  const T rb = (T)bb;
  const T rbc = (T)(bb * ccd);
  // increment form: this iteration's transforms give the change of u, and the
  // next Step 1 gets the change of its right-hand side,
  //   X = b (ut^{n+1} - ut^n) - (a^{n+1} - a^n),
  // with ut = c u in the solid (c of the iteration that formed it) and the
  // change of a as stored
  const bool incr = cur.incr != 0;
  // X only where Step 4 may pass it on: the increment form starts after the
  // first kIncrAfter iterations (Step 4 of this iteration completes cur.iter + 1)
  const bool xform = !FUSED && ctl->incr_enabled != 0 && cur.iter + 1 >= kIncrAfter;
  const T rbcp = (T)(bb * cur.c_prev);
  const int z = blockIdx.x, field = blockIdx.y;

  const int64_t off = field * ntot + (int64_t)z * S::NV;
  gmem<V>* uq = as_global(reinterpret_cast<V*>(u + off));
  gmem<V>* aq = as_global(reinterpret_cast<V*>(a + off));
  const gmem<uint32_t>* hq = as_global(reinterpret_cast<const uint32_t*>(H + (int64_t)z * S::NV));
  // a is exactly zero in the pore (it is only ever written in the solid), so
  // it is loaded unconditionally: no load waits on the value of H.
  V up[S::QPT], ao[S::QPT];
  uint32_t hw[S::QPT];
#pragma unroll
  for (int j = 0; j < S::QPT; ++j) {
    const int q = threadIdx.x + j * S::NT;
    hw[j] = 0u;
    if (S::PF >= 1 && (S::FULL || q < S::NQ)) {
      up[j] = uq[q];
      hw[j] = hq[q];
      if constexpr (S::PF == 2) ao[j] = aq[q];
    }
  }

  cplx<T>* slab = spec + field * nspec + (int64_t)z * NY * S::XH;
  float4 stg[SlabCopy<T, NX, NY>::PT];
  slab_load_regs<T, NX, NY>(stg, slab);  // in flight during the partial sums below
  const SlabTw<T> tws = slab_twiddles<T, NX, NY>(lds, twx_g, twy_g, rtw_g);
  const cplx<T>*twx = tws.x, *twy = tws.y, *rtw = tws.r;
  if constexpr (!FUSED) {
    if (threadIdx.x < kShare) {
      const int nb = gridDim.x * gridDim.y, b = blockIdx.y * gridDim.x + blockIdx.x;
      const int g0 = (int)((int64_t)ngreen * b / nb), g1 = (int)((int64_t)ngreen * (b + 1) / nb);
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
  }
  slab_regs_to_lds<T, NX, NY>(lds, stg);
  __syncthreads();
  slab_cols_inverse<T, NX, NY>(lds, twy);
  if constexpr (S::PF == 1) {
    // a is issued here: its latency overlaps the row transforms, and fewer
    // registers stay live across the column transforms
#pragma unroll
    for (int j = 0; j < S::QPT; ++j) {
      const int q = threadIdx.x + j * S::NT;
      if (S::FULL || q < S::NQ) ao[j] = aq[q];
    }
  }
  slab_rows_inverse<T, NX, NY>(lds, twx, rtw);

  // Steps 2-3 on 4 consecutive voxels per quad.  The fused pass keeps the new
  // a and the solid flags of its quads for the rhs half (u stays in LDS).
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll S::UNR
  for (int j = 0; j < S::QPT; ++j) {
    const int q = threadIdx.x + j * S::NT;
    if (!S::FULL && q >= S::NQ) continue;
    const int v = 4 * q;
    const int y = v / NX, x = v - y * NX;
    V upj, aoj;
    uint32_t hwj;
    if constexpr (S::PF == 0) {
      upj = uq[q];
      hwj = hq[q];
      aoj = aq[q];
    } else {
      upj = up[j];
      hwj = hw[j];
      aoj = ao[j];
    }
    V un = lds_ld4<V>(ldsr + y * 2 * S::P2 + x);
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
    if constexpr (FUSED) {
      ao[j] = aoj;
      hw[j] = hwj;
    } else if (xform) {
      V r;
      r.x = ((hwj & 0xffu) ? rbc * un.x - rbcp * upj.x : rb * (un.x - upj.x)) - dav[0];
      r.y = ((hwj & 0xff00u) ? rbc * un.y - rbcp * upj.y : rb * (un.y - upj.y)) - dav[1];
      r.z = ((hwj & 0xff0000u) ? rbc * un.z - rbcp * upj.z : rb * (un.z - upj.z)) - dav[2];
      r.w = ((hwj & 0xff000000u) ? rbc * un.w - rbcp * upj.w : rb * (un.w - upj.w)) - dav[3];
      lds_st4(ldsr + y * 2 * S::P2 + x, r);
    } else {
      V r;
      r.x = ((hwj & 0xffu) ? rbc : rb) * un.x - aoj.x;
      r.y = ((hwj & 0xff00u) ? rbc : rb) * un.y - aoj.y;
      r.z = ((hwj & 0xff0000u) ? rbc : rb) * un.z - aoj.z;
      r.w = ((hwj & 0xff000000u) ? rbc : rb) * un.w - aoj.w;
      lds_st4(ldsr + y * 2 * S::P2 + x, r);
    }
  }
  const int nblk = gridDim.x * gridDim.y;
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  if constexpr (!FUSED) {
    // Step 4 is formed after the launch boundary (by the rhs pass or the next
    // green pass) from one record per workgroup: the green share, then these
    // partials.  No cross-workgroup traffic here.
    block_sum<4>(acc, red);
    if (threadIdx.x == 0) {
      double gs[3] = {0.0, 0.0, 0.0};
      for (int t = 0; t < kShare; ++t)
        for (int c = 0; c < 3; ++c) gs[c] += gsh[t * 3 + c];
      for (int c = 0; c < 3; ++c) lpart[bid * 7 + c] = gs[c];
      for (int c = 0; c < 4; ++c) lpart[bid * 7 + 3 + c] = acc[c];
    }
    // the speculative r of this slab, forward transformed in place of the
    // spectrum it was loaded from (only this workgroup touches that slab)
    __syncthreads();
    slab_forward_store<T, NX, NY>(lds, slab, twx, twy, rtw);
    return;
  }
  block_sum<4>(acc, red);
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
    stokes_finalize(ctl, par, gpart, ngreen, lpart, nblk, ntot, hist, red7);
  }
  if constexpr (FUSED) {
    // ---- device-wide gate: the last workgroup opens it after Step 4
    if (threadIdx.x == 0) {
      int go = 1;
      if (s_last) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&ctl->gate, gate0 + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        uint32_t polls = 0;
        while (__hip_atomic_load(&ctl->gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gate0) {
          __builtin_amdgcn_s_sleep(8);
          if (++polls == kGatePolls) {
            go = 0;
            break;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      StokesState* nx = &ctl->st[par ^ 1];
      if (!go) {
        __hip_atomic_store(&ctl->fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&nx->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if (__hip_atomic_load(&nx->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        go = 0;  // converged (or stopped) at this iteration: no next rhs
      }
      s_go = go;
    }
    __syncthreads();
    if (!s_go) return;
    // ---- rhs half: r = b^{n+1} ut^{n+1} - a^{n+1} on the slab in LDS
    const StokesState* nx = &ctl->st[par ^ 1];
    const double bnew = __hip_atomic_load(&nx->psi[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double cprev = __hip_atomic_load(&nx->c_prev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const T b1 = (T)bnew;
    const T bcp = (T)(bnew * cprev);
#pragma unroll
    for (int j = 0; j < S::QPT; ++j) {
      const int q = threadIdx.x + j * S::NT;
      if (!S::FULL && q >= S::NQ) continue;
      const int v = 4 * q;
      const int y = v / NX, x = v - y * NX;
      T* cell = ldsr + y * 2 * S::P2 + x;
      const V un = lds_ld4<V>(cell);
      V r;
      r.x = ((hw[j] & 0xffu) ? bcp : b1) * un.x - ao[j].x;
      r.y = ((hw[j] & 0xff00u) ? bcp : b1) * un.y - ao[j].y;
      r.z = ((hw[j] & 0xff0000u) ? bcp : b1) * un.z - ao[j].z;
      r.w = ((hw[j] & 0xff000000u) ? bcp : b1) * un.w - ao[j].w;
      lds_st4(cell, r);
    }
    __syncthreads();
    slab_forward_store<T, NX, NY>(lds, slab, twx, twy, rtw);
  }
}

template <typename T, int NX, int NY>
__global__ __launch_bounds__((SlabCfg<T, NX, NY>::NT))
__attribute__((amdgpu_waves_per_eu(SlabCfg<T, NX, NY>::WPE))) void k_slab_rhs(
    StokesCellArgs one, const StokesCellArgs* __restrict__ many, int par, int step4, int ngreen,
    int64_t ntot, int64_t nspec, const cplx<T>* __restrict__ twx_g,
    const cplx<T>* __restrict__ twy_g, const cplx<T>* __restrict__ rtw_g) {
  using S = SlabCfg<T, NX, NY>;
  const StokesCellArgs ca = many ? many[blockIdx.z] : one;
  cplx<T>* __restrict__ spec = reinterpret_cast<cplx<T>*>(ca.spec);
  const T* __restrict__ u = reinterpret_cast<const T*>(ca.u);
  const T* __restrict__ a = reinterpret_cast<const T*>(ca.a);
  const uint8_t* __restrict__ H = ca.H;
  StokesCtl* ctl = ca.ctl;
  using V = typename Vec4<T>::type;
  extern __shared__ __align__(32) char smem_raw[];
  __shared__ double red7[7 * 16];
  __shared__ double s_b, s_cp;
  __shared__ int s_stop, s_kept;
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  T* ldsr = reinterpret_cast<T*>(smem_raw);
  if (stokes_skip(ctl)) return;
  const SlabTw<T> tws = slab_twiddles<T, NX, NY>(lds, twx_g, twy_g, rtw_g);
  const cplx<T>*twx = tws.x, *twy = tws.y, *rtw = tws.r;
  const int z = blockIdx.x, field = blockIdx.y;
  const int64_t off = field * ntot + (int64_t)z * S::NV;
  const gmem<V>* uq = as_global(reinterpret_cast<const V*>(u + off));
  const gmem<V>* aq = as_global(reinterpret_cast<const V*>(a + off));
  const gmem<uint32_t>* hq = as_global(reinterpret_cast<const uint32_t*>(H + (int64_t)z * S::NV));
  // Step 4 of this iteration, formed from all partial sums by every
  // workgroup (same order, same bits); workgroup 0 of the cell stores the new
  // state in the other slot.  Without step4 the current slot is used as is.
  if (step4) {
    double tot[7];
    stokes_sum_records<S::SUM_U>(ca.lpart, gridDim.x * gridDim.y, tot, red7);
    if (threadIdx.x == 0) {
      const StokesState cur = ctl->st[par];
      StokesState nx;
      stokes_step4(ctl, cur, tot, ntot, nx);
      if (blockIdx.x == 0 && blockIdx.y == 0) {
        stokes_history(ctl, cur, nx, ca.hist);
        ctl->st[par ^ 1] = nx;
      }
      s_b = nx.psi[2];
      s_cp = nx.c_prev;
      s_stop = nx.done;
      s_kept = nx.psi[2] == cur.psi[2];
    }
  } else if (threadIdx.x == 0) {
    s_b = ctl->st[par].psi[2];
    s_cp = ctl->st[par].c_prev;
    s_stop = 0;
    s_kept = 0;
  }
  __syncthreads();
  // after a slab local pass (step4) the spectra already hold r unless Step 4
  // changed b
  if (s_stop || s_kept) return;
  const T bb = (T)s_b;
  const T bcp = (T)(s_b * s_cp);
  // a vanishes in the pore, so r = (H ? b c : b) u - a needs no branch on H
  // and every load of the loop can be issued at once.
#pragma unroll
  for (int j = 0; j < S::QPT; ++j) {
    const int q = threadIdx.x + j * S::NT;
    if (!S::FULL && q >= S::NQ) continue;
    const int v = 4 * q;
    const int y = v / NX, x = v - y * NX;
    const V uv = uq[q], av = aq[q];
    const uint32_t hw = hq[q];
    V r;
    r.x = ((hw & 0xffu) ? bcp : bb) * uv.x - av.x;
    r.y = ((hw & 0xff00u) ? bcp : bb) * uv.y - av.y;
    r.z = ((hw & 0xff0000u) ? bcp : bb) * uv.z - av.z;
    r.w = ((hw & 0xff000000u) ? bcp : bb) * uv.w - av.w;
    lds_st4(ldsr + y * 2 * S::P2 + x, r);
  }
  __syncthreads();
  slab_forward_store<T, NX, NY>(lds, spec + field * nspec + (int64_t)z * NY * S::XH, twx, twy, rtw);
}

// Step 4 in one workgroup (pass mode 4) of the slab passes' block size: the
// same sums as the rhs pass forms (same records, same order), so the same bits.
__global__ __launch_bounds__(1024) void k_slab_step4(StokesCellArgs one, int par, int nrec,
                                                     int64_t ntot, int set_hold) {
  __shared__ double red7[7 * 16];
  StokesCtl* ctl = one.ctl;
  // The kernel is a chain of latencies: everything it reads (the stop words,
  // this thread's records, the current state) is loaded before any of it is
  // used.  The sum is the one stokes_sum_records<2> forms.
  const int32_t skip = ctl->st[0].done | ctl->st[1].done | ctl->hold;
  double v[2][7];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int j = threadIdx.x + k * blockDim.x;
#pragma unroll
    for (int c = 0; c < 7; ++c) v[k][c] = j < nrec ? one.lpart[j * 7 + c] : 0.0;
  }
  StokesState cur;
  if (threadIdx.x == 0) cur = ctl->st[par];
  if (skip) return;
  double tot[7];
  if (nrec <= 2 * (int)blockDim.x) {
#pragma unroll
    for (int c = 0; c < 7; ++c) tot[c] = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int c = 0; c < 7; ++c) tot[c] += v[k][c];
    block_sum<7>(tot, red7);
  } else {
    stokes_sum_records<2>(one.lpart, nrec, tot, red7);
  }
  if (threadIdx.x == 0) {
    StokesState nx;
    stokes_step4(ctl, cur, tot, ntot, nx);
    stokes_history(ctl, cur, nx, one.hist);
    ctl->st[par ^ 1] = nx;
    if (set_hold && !nx.done && nx.psi[2] != cur.psi[2]) ctl->hold = 1 + (par ^ 1);
  }
}

// ------------------------------------------------------------------ launchers

template <typename T>
hipError_t launch_slab_step4(const Geom& g, const StokesCellArgs& one, int par, int nrec,
                             hipStream_t s) {
  int nt = 0;
  switch (g.nx) {
#define CASE(N)                  \
  case N:                        \
    nt = SlabCfg<T, N, N>::NT;   \
    break;
    ACM_SLAB_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  ACM_LAUNCH(k_slab_step4, dim3(1), dim3(nt), 0, s, one, par, nrec, g.ntot, 1);
  return hipGetLastError();
}

hipError_t launch_step4_nohold(const Geom& g, const StokesCellArgs& one, int par, int nrec,
                               hipStream_t s) {
  ACM_LAUNCH(k_slab_step4, dim3(1), dim3(1024), 0, s, one, par, nrec, g.ntot, 0);
  return hipGetLastError();
}

template <typename T>
bool slab_supported(const Geom& g) {
  if (g.dim != 3 || g.nx != g.ny) return false;
  switch (g.nx) {
#define CASE(N) \
  case N:       \
    return SlabCfg<T, N, N>::LDS_BYTES <= 150 * 1024;
    ACM_SLAB_LENGTHS(CASE)
#undef CASE
    default:
      return false;
  }
}

template <typename T>
int slab_local_blocks(const Geom& g) {
  return g.nz * g.dim;
}

template <typename T>
hipError_t launch_slab_local(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                             const StokesCellArgs* many, int ncells, int par, int green_blocks,
                             hipStream_t s) {
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  dim3 grid((unsigned)g.nz, (unsigned)g.dim, (unsigned)ncells);
  switch (g.nx) {
#define CASE(N)                                                                                \
  case N: {                                                                                    \
    using S = SlabCfg<T, N, N>;                                                                \
    ACM_LAUNCH((k_slab_local<T, N, N, false>), grid, dim3(S::NT), S::LDS_BYTES, s, one, many,  \
               par, green_blocks, g.ntot, g.nspec, ct + tb.off.tw_x, ct + tb.off.tw_y,         \
               ct + tb.off.rtw);                                                               \
    return hipGetLastError();                                                                  \
  }
    ACM_SLAB_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_slab_rhs(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                           const StokesCellArgs* many, int ncells, int par, int step4,
                           int green_blocks, hipStream_t s) {
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  dim3 grid((unsigned)g.nz, (unsigned)g.dim, (unsigned)ncells);
  switch (g.nx) {
#define CASE(N)                                                                                \
  case N: {                                                                                    \
    using S = SlabCfg<T, N, N>;                                                                \
    ACM_LAUNCH((k_slab_rhs<T, N, N>), grid, dim3(S::NT), S::LDS_BYTES, s, one, many, par,  \
               step4, green_blocks, g.ntot, g.nspec, ct + tb.off.tw_x, ct + tb.off.tw_y,       \
               ct + tb.off.rtw);                                                               \
    return hipGetLastError();                                                                  \
  }
    ACM_SLAB_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
int slab_fused_capacity(const Geom& g) {
  if (!slab_supported<T>(g)) return 0;
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  hipError_t e = hipErrorInvalidValue;
  switch (g.nx) {
#define CASE(N)                                                                                \
  case N: {                                                                                    \
    using S = SlabCfg<T, N, N>;                                                                \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(                                          \
        &per_cu, reinterpret_cast<const void*>(&k_slab_local<T, N, N, true>), S::NT,           \
        S::LDS_BYTES);                                                                         \
    break;                                                                                     \
  }
    ACM_SLAB_LENGTHS(CASE)
#undef CASE
    default:
      return 0;
  }
  if (e != hipSuccess) return 0;
  return per_cu * ncu;
}

template <typename T>
hipError_t launch_slab_fused(const Geom& g, const DevTables<T>& tb, const StokesCellArgs& one,
                             int par, int green_blocks, hipStream_t s) {
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  dim3 grid((unsigned)g.nz, (unsigned)g.dim, 1u);
  switch (g.nx) {
#define CASE(N)                                                                                \
  case N: {                                                                                    \
    using S = SlabCfg<T, N, N>;                                                                \
    ACM_LAUNCH((k_slab_local<T, N, N, true>), grid, dim3(S::NT), S::LDS_BYTES, s, one,  \
                       nullptr, par, green_blocks, g.ntot, g.nspec, ct + tb.off.tw_x,          \
                       ct + tb.off.tw_y, ct + tb.off.rtw);                                     \
    return hipGetLastError();                                                                  \
  }
    ACM_SLAB_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

#define INST(T)                                                                                \
  template bool slab_supported<T>(const Geom&);                                                \
  template int slab_fused_capacity<T>(const Geom&);                                            \
  template hipError_t launch_slab_fused<T>(const Geom&, const DevTables<T>&,                   \
                                           const StokesCellArgs&, int, int, hipStream_t);      \
  template int slab_local_blocks<T>(const Geom&);                                              \
  template hipError_t launch_slab_step4<T>(const Geom&, const StokesCellArgs&, int, int,       \
                                           hipStream_t);                                       \
  template hipError_t launch_slab_local<T>(const Geom&, const DevTables<T>&,                   \
                                           const StokesCellArgs&, const StokesCellArgs*, int,   \
                                           int, int, hipStream_t);                             \
  template hipError_t launch_slab_rhs<T>(const Geom&, const DevTables<T>&,                     \
                                         const StokesCellArgs&, const StokesCellArgs*, int,     \
                                         int, int, int, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace acm
