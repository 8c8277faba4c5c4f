// Fused passes of the Lippmann-Schwinger iteration for the penalised
// advection-diffusion cell problem (Section 3.2: eq. penalization, eq. iter,
// eq. fft_solute, eq. tol_solute; symbols of eq. fft_app).
//
// One iteration n (3D; in 2D the y passes disappear and "last axis" is y):
//   [y inverse of grad chi-hat]
//   local  (x rows, all fields of a row at once): grad chi^n in real space,
//           e = grad chi + g, tau = (A - A0) e, f = calF (1-H) - (B - B0) . e,
//           forward x transform of (tau, f).
//   [y forward of (tau, f)]
//   green  (last axis): F-hat = f-hat + i s . tau-hat, chi-hat update by the
//           comparison-medium symbol (plus 1/dt for a time step), Parseval
//           sums for r_1 = |chi^{n+1} - chi^n| and r_2 = |grad chi^{n+1} -
//           grad chi^n|, the last workgroup applies the stopping test, and
//           grad chi-hat = i s chi-hat is transformed back along the last axis.
#include "slab_common.hpp"

namespace acm {

struct TGreenGeom {
  int dim;
  int nx, xh;
  int ny, nz;
  int plane;
  int64_t nspec;
  int64_t ntot;
};

// Tile configuration of the green pass (see ColCfg): pencil-count variant and
// whether each field gets its own threads during the transforms (which takes
// it from 102 to 65.9 us per LS iteration at 128^3 FP32).  Half-width tiles
// (8 pencils): at 128^3 the 1,040 tiles all fit on the chip at once (five
// workgroups of 384 threads per CU), where 520 full-width tiles of 768
// threads leave 8 for a second round (24.7 against 27.0 us).
constexpr int kTGVar = 1;
constexpr int kTGSpl = 1;
template <typename T, int L, int NC>
using TGCfg = ColCfg<T, L, NC, kTGVar, kTGSpl>;

// Fields the green pass transforms forward: the row form brings tau-hat (D
// fields) and f-hat; the slab form (SL) brings S = G_x + G_y + f_z as three
// partial spectra (fields 0, 1, 4), summed on load, and tau_z (field 3; see
// k_transport_slab).
// Flux form (FL, row form only): the inputs are the spectra of the face
// fluxes tau_c = (A_f,c - A0)(D+_c chi + g_c) and of f, whose divergence takes
// the backward-difference symbol (1 - e^{-i theta_c})/h_c = l_c h_c/2 + i s_c;
// the outputs are the central gradient (advection) and the forward difference
// D+_c chi-hat = (i s_c - l_c h_c/2) chi-hat (2 D fields).
template <int D, bool SL>
constexpr int tg_inputs() { return SL ? 2 : D + 1; }
template <int D, bool SL, bool FL = false>
constexpr int tg_fields() { return FL ? 2 * D : (SL ? D : D + 1); }

// MODE 0: LS update.  MODE 1: only form grad chi-hat from chi-hat (set-up).
template <typename T, int L, int D, int MODE, bool SL, bool FL>
__global__ __launch_bounds__((TGCfg<T, L, tg_fields<D, SL, FL>()>::NT)) void k_transport_green(
    cplx<T>* __restrict__ spec, cplx<T>* __restrict__ chat, const cplx<T>* __restrict__ chat_m,
    double* __restrict__ partials, TransportCtl* ctl, TGreenGeom gg, int par, int judge,
    const cplx<T>* __restrict__ tw_g, const T* __restrict__ sx, const T* __restrict__ lx,
    const T* __restrict__ sy, const T* __restrict__ ly, const T* __restrict__ sz,
    const T* __restrict__ lz) {
  using C = TGCfg<T, L, tg_fields<D, SL, FL>()>;
  constexpr int PS = L * C::TX;
  constexpr int NIN = tg_inputs<D, SL>();
  constexpr int NOUT = FL ? 2 * D : D;
  extern __shared__ __align__(16) char smem_raw[];
  __shared__ double red[2 * 16];
  __shared__ int s_last;
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  if (MODE == 0 && transport_done(ctl)) return;
  const cplx<T>* tw =
      twiddles_to_lds<T, C::NT, Plan<L>::tw_total>(lds + tg_fields<D, SL, FL>() * PS, tw_g);
  const int P = gg.plane;
  // neighbouring tiles share the cache lines at their edges (a tile row is
  // half a line of FP32 complex): keep them on one XCD, whose L2 they share
  const int f0 = xcd_tile(blockIdx.x, gridDim.x) * C::TX;
  // transform threads: (field, t, column) when each field has its own threads
  const int fc = kTGSpl ? threadIdx.x / (C::TPP * C::TX) : 0;
  const int tr = kTGSpl ? threadIdx.x % (C::TPP * C::TX) : threadIdx.x;
  const int t = tr / C::TX, colt = tr % C::TX;
  const bool act = t < C::TPP && f0 + colt < P;

  if constexpr (MODE == 0) {
    gather_to_lds<cplx<T>, C::NT, NIN * PS>(lds, NIN * PS, [&](int e) {
      const int c = e / PS, rem = e - c * PS;
      const int i = rem / C::TX, col = rem - i * C::TX;
      const int f = f0 + col;
      cplx<T> v = cmake<T>(T(0), T(0));
      if (f < P) {
        const int64_t mi = (int64_t)i * P + f;
        if constexpr (SL) {
          if (c == 0) {  // S = G_x + G_y + f_z
            const cplx<T> a = spec[mi], b = spec[gg.nspec + mi], d = spec[4 * gg.nspec + mi];
            v = cmake<T>(a.x + b.x + d.x, a.y + b.y + d.y);
          } else {  // tau_z
            v = spec[3 * gg.nspec + mi];
          }
        } else {
          v = spec[c * gg.nspec + mi];
        }
      }
      return v;
    });
    __syncthreads();
    if constexpr (kTGSpl)
      PencilFFT<T, L, 1, -1>::run_lds(t, act && fc < NIN, lds + (fc < NIN ? fc : 0) * PS + colt, PS,
                                      C::TX, tw);
    else
      PencilFFT<T, L, NIN, -1>::run_lds(t, act, lds + colt, PS, C::TX, tw);
    __syncthreads();
  }

  double acc[2] = {0.0, 0.0};
  const T inv_ntot = T(1.0 / (double)gg.ntot);
  const T A0 = (T)ctl->A0;
  const T inv_dt = (T)ctl->inv_dt;
  const int steady = ctl->steady;
  T B0[3] = {(T)ctl->B0[0], (T)ctl->B0[1], (T)ctl->B0[2]};
  for (int e = threadIdx.x; e < PS; e += C::NT) {
    const int i = e / C::TX, col = e - i * C::TX;
    const int f = f0 + col;
    if (f >= P) continue;
    int kx, ky, kz;
    if (D == 3) {
      kx = f % gg.xh;
      ky = f / gg.xh;
      kz = i;
    } else {
      kx = f;
      ky = i;
      kz = 0;
    }
    T s[D];
    s[0] = sx[kx];
    s[1] = sy[ky];
    T Lk = lx[kx] + ly[ky];
    if constexpr (D == 3) {
      s[2] = sz[kz];
      Lk += lz[kz];
    }
    // l_c h_c / 2: real part of the backward-difference symbol (flux form)
    T lh[D];
    if constexpr (FL) {
      lh[0] = lx[kx] * T(0.5 / gg.nx);
      lh[1] = ly[ky] * T(0.5 / gg.ny);
      if constexpr (D == 3) lh[2] = lz[kz] * T(0.5 / gg.nz);
    }
    const int64_t mi = (int64_t)i * P + f;
    cplx<T> cn;
    if constexpr (MODE == 0) {
      const bool k0 = (kx == 0 && ky == 0 && kz == 0);
      // F-hat = f-hat + i s . tau-hat (slab form: S-hat + i s_z tau_z-hat, the
      // x and y terms being already in S as central differences)
      cplx<T> F;
      T bs = T(0);
#pragma unroll
      for (int c = 0; c < D; ++c) bs += B0[c] * s[c];
      if constexpr (SL) {
        F = lds[e];
        const cplx<T> tz = lds[PS + e];
        F.x -= s[D - 1] * tz.y;
        F.y += s[D - 1] * tz.x;
      } else {
        F = lds[D * PS + e];
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const cplx<T> tc = lds[c * PS + e];
          F.x -= s[c] * tc.y;
          F.y += s[c] * tc.x;
          if constexpr (FL) {
            F.x += lh[c] * tc.x;
            F.y += lh[c] * tc.y;
          }
        }
      }
      if (k0) {
        double b0g = 0.0;
        for (int c = 0; c < D; ++c) b0g += ctl->B0[c] * ctl->g[c];
        F.x -= (T)((double)gg.ntot * b0g);
      }
      const cplx<T> co = chat[mi];
      if (inv_dt != T(0)) {
        const cplx<T> cm = chat_m[mi];
        F.x += inv_dt * cm.x;
        F.y += inv_dt * cm.y;
      }
      // chi-hat = F / (1/dt + A0 L + i B0 . s)
      const T dr = inv_dt + A0 * Lk, di = bs;
      const T inv = T(1) / (dr * dr + di * di);
      cn = cmake<T>((F.x * dr + F.y * di) * inv, (F.y * dr - F.x * di) * inv);
      if (k0 && steady) cn = cmake<T>(T(0), T(0));
      chat[mi] = cn;
      const double w = (kx == 0 || 2 * kx == gg.nx) ? 1.0 : 2.0;
      const double ddx = (double)cn.x - co.x, ddy = (double)cn.y - co.y;
      double s2 = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) s2 += (double)s[c] * s[c];
      const double a2 = w * (ddx * ddx + ddy * ddy);
      acc[0] += a2;
      acc[1] += a2 * s2;
    } else {
      cn = chat[mi];
    }
    // grad chi-hat / N = i s chi-hat / N (and D+ chi-hat / N in the flux form)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      lds[c * PS + e] = cmake<T>(-s[c] * cn.y * inv_ntot, s[c] * cn.x * inv_ntot);
      if constexpr (FL)
        lds[(D + c) * PS + e] = cmake<T>((-s[c] * cn.y - lh[c] * cn.x) * inv_ntot,
                                         (s[c] * cn.x - lh[c] * cn.y) * inv_ntot);
    }
  }
  __syncthreads();
  if constexpr (kTGSpl)
    PencilFFT<T, L, 1, 1>::run_lds(t, act && fc < NOUT, lds + (fc < NOUT ? fc : 0) * PS + colt, PS,
                                   C::TX, tw);
  else
    PencilFFT<T, L, NOUT, 1>::run_lds(t, act, lds + colt, PS, C::TX, tw);
  __syncthreads();
  scatter_from_lds<cplx<T>, C::NT, NOUT * PS>(lds, NOUT * PS, [&](int e, const cplx<T>& v) {
    const int c = e / PS, rem = e - c * PS;
    const int i = rem / C::TX, col = rem - i * C::TX;
    const int f = f0 + col;
    if (f < P) spec[c * gg.nspec + (int64_t)i * P + f] = v;
  });
  if constexpr (MODE == 0) {
    block_sum<2>(acc, red);
    if (!judge) {
      // the next slab pass judges these partials after the launch boundary
      if (threadIdx.x == 0) {
        partials[blockIdx.x * 2 + 0] = acc[0];
        partials[blockIdx.x * 2 + 1] = acc[1];
      }
      return;
    }
    if (threadIdx.x == 0) {
      partials[blockIdx.x * 2 + 0] = acc[0];
      partials[blockIdx.x * 2 + 1] = acc[1];
      __threadfence();
      const unsigned prev = atomicAdd(&ctl->counter, 1u);
      s_last = (prev == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (s_last) {
      __threadfence();
      double tot[2] = {0.0, 0.0};
      for (int j = threadIdx.x; j < (int)gridDim.x; j += blockDim.x) {
        tot[0] += partials[j * 2 + 0];
        tot[1] += partials[j * 2 + 1];
      }
      block_sum<2>(tot, red);
      if (threadIdx.x == 0) {
        ctl->st[par ^ 1] = transport_judge(ctl, ctl->st[par], tot[0], tot[1], gg.ntot);
        ctl->counter = 0u;
      }
    }
  }
}

// FL: flux form.  The row brings the central gradient (fields 0..D-1) and the
// forward difference D+ chi (fields D..2D-1); tau_c is the flux through the
// face between x and x + h e_c, (A_f,c - A0)(D+_c chi + g_c), with A_f,c the
// harmonic mean of A on the two sides (H of the neighbour is read from
// memory: along y and z it lies in another row).
template <typename T, int M, int D, bool FL>
__global__ __launch_bounds__((RowCfgN<T, M, FL ? 2 * D : D + 1>::NT)) void k_transport_local(
    cplx<T>* __restrict__ spec, const T* __restrict__ u, const uint8_t* __restrict__ H,
    const TransportCtl* __restrict__ ctl, int nrows, int ny, int nz, int64_t ntot, int64_t nspec,
    const cplx<T>* __restrict__ tw, const cplx<T>* __restrict__ rtw) {
  using C = RowCfgN<T, M, FL ? 2 * D : D + 1>;
  constexpr int NIN = FL ? 2 * D : D;
  constexpr int NX = 2 * M;
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  T* ldsr = reinterpret_cast<T*>(smem_raw);
  if (transport_done(ctl)) return;
  const int row0 = blockIdx.x * C::RB;
  const int nr = min(C::RB, nrows - row0);
  for (int c = 0; c < NIN; ++c) {
    const cplx<T>* src = spec + c * nspec + (int64_t)row0 * (M + 1);
    gather_to_lds<cplx<T>, C::NT, C::RB * (M + 1)>(lds + c * C::FS, nr * (M + 1),
                                                   [&](int v) { return src[v]; });
  }
  __syncthreads();
  const int row = threadIdx.x / C::TPP, t = threadIdx.x % C::TPP;
  rows_c2r_lds<T, M, NIN>(lds, C::FS, row, t, row < nr, tw, rtw);

  const T g[3] = {(T)ctl->g[0], (T)ctl->g[1], (T)ctl->g[2]};
  const T B0[3] = {(T)ctl->B0[0], (T)ctl->B0[1], (T)ctl->B0[2]};
  const T A0 = (T)ctl->A0, Pe = (T)ctl->Pe, eta = (T)ctl->eta, dif = (T)ctl->diff;
  const T calF = (T)ctl->calF;
  const int64_t off = (int64_t)row0 * NX;
  for (int v = threadIdx.x; v < nr * NX; v += C::NT) {
    const int r = v / NX, x = v - r * NX;
    const int li = r * 2 * C::RP + x;
    const bool solid = H[off + v] != 0;
    const T Aa = solid ? eta : dif;
    T fval = solid ? T(0) : calF;
    if constexpr (FL) {
      // neighbours x + h e_c of this voxel (row R = z ny + y of the cell)
      const int R = row0 + r;
      const int y = R % ny, z = R / ny;
      int64_t nb[3];
      nb[0] = off + (int64_t)r * NX + (x + 1 == NX ? 0 : x + 1);
      nb[1] = ((int64_t)z * ny + (y + 1 == ny ? 0 : y + 1)) * NX + x;
      nb[2] = ((int64_t)(z + 1 == nz ? 0 : z + 1) * ny + y) * NX + x;
      T tau[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const T e = ldsr[2 * c * C::FS + li] + g[c];
        const T Bc = solid ? T(0) : Pe * u[c * ntot + off + v];
        fval -= (Bc - B0[c]) * e;
        const T An = H[nb[c]] != 0 ? eta : dif;
        const T Af = T(2) * Aa * An / (Aa + An);
        tau[c] = (Af - A0) * (ldsr[2 * (D + c) * C::FS + li] + g[c]);
      }
#pragma unroll
      for (int c = 0; c < D; ++c) ldsr[2 * c * C::FS + li] = tau[c];
    } else {
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const T e = ldsr[2 * c * C::FS + li] + g[c];
        const T Bc = solid ? T(0) : Pe * u[c * ntot + off + v];
        fval -= (Bc - B0[c]) * e;
        ldsr[2 * c * C::FS + li] = (Aa - A0) * e;
      }
    }
    ldsr[2 * D * C::FS + li] = fval;
  }
  __syncthreads();
  rows_r2c_lds<T, M, D + 1>(lds, C::FS, row, t, row < nr, tw, rtw);
  for (int c = 0; c <= D; ++c) {
    cplx<T>* dst = spec + c * nspec + (int64_t)row0 * (M + 1);
    scatter_from_lds<cplx<T>, C::NT, C::RB * (M + 1)>(lds + c * C::FS, nr * (M + 1),
                                                      [&](int v, const cplx<T>& x) { dst[v] = x; });
  }
}

// Local pass on xy-slabs (3D cubes whose slab fits in LDS): workgroup (z, c)
// takes the z-slab of d_c chi back to real space (column then row inverse
// transforms), forms e_c = d_c chi + g_c, tau_c = (A - A0) e_c and this field's
// share of f, f_c = calF (1-H) [c = 0 only] - (B_c - B0_c) e_c.  Since F =
// f + div tau, the x and y workgroups fold their divergence term in real
// space, G_c = f_c + D_c tau_c, and transform only G_c (into field c); the z
// workgroups transform f_z (field 4) and tau_z (field 3, whose derivative
// needs the z transform), one each, so that every workgroup does one inverse
// and one forward transform.  The green pass then transforms S = G_x + G_y +
// f_z and tau_z.  Compared with the row pass this saves the separate y passes
// and three of the seven forward transforms of the iteration.
//
// D_c is the central difference along x (c = 0) or y (c = 1) of the periodic
// slab, exactly the i s_c of the spectral derivative.  Each G_c is formed in
// one sweep with no value held across a barrier: along x the quads of a row
// sit on consecutive lanes of one row group (R <= RG lanes, RG a power of two
// dividing 64), so the neighbours' tau come by cross-lane exchange; along y
// each thread walks a strip of rows of one quad column, taking the tau of the
// two rows that bound its strip before the barrier after which strips are
// overwritten.
template <typename T, int N>
__global__ __launch_bounds__((SlabCfg<T, N, N>::NT))
__attribute__((amdgpu_waves_per_eu(SlabCfg<T, N, N>::WPE_ONE))) void k_transport_slab(
    cplx<T>* __restrict__ spec, const T* __restrict__ u, const uint8_t* __restrict__ H,
    TransportCtl* ctl, const double* __restrict__ partials, int ngreen, int par, int64_t ntot,
    int64_t nspec, const cplx<T>* __restrict__ twx_g, const cplx<T>* __restrict__ twy_g,
    const cplx<T>* __restrict__ rtw_g) {
  using S = SlabCfg<T, N, N>;
  using V = typename Vec4<T>::type;
  constexpr int R = N / 4;  // quads per row
  constexpr int RG = R <= 8 ? 8 : (R <= 16 ? 16 : (R <= 32 ? 32 : 64));
  static_assert(R <= RG && RG <= 64 && S::NT % RG == 0, "row groups must tile the workgroup");
  constexpr int NG = S::NT / RG;           // row groups per workgroup
  constexpr int PX = (N + NG - 1) / NG;    // sweeps of the x workgroup
  constexpr int RPS = (N + NG - 1) / NG;   // rows per strip of the y workgroup
  extern __shared__ __align__(32) char smem_raw[];
  __shared__ double red[2 * 16];
  __shared__ int s_stop;
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  T* ldsr = reinterpret_cast<T*>(smem_raw);
  if (transport_done(ctl)) return;
  // Stop test of the previous green pass, formed by every workgroup from all
  // its partial sums in the same order (same bits); workgroup 0 stores it.
  {
    const TransportState cur = ctl->st[par];
    double tot[2] = {0.0, 0.0};
    if (cur.pend) {
      // four partials per thread in flight at a time (one green tile each;
      // 1,040 tiles at 128^3): the sum is one memory round trip, not three
      constexpr int U = 4;
      for (int j0 = threadIdx.x; j0 < ngreen; j0 += U * S::NT) {
        double v[U][2];
#pragma unroll
        for (int k = 0; k < U; ++k) {
          const int j = j0 + k * S::NT;
          v[k][0] = j < ngreen ? partials[j * 2 + 0] : 0.0;
          v[k][1] = j < ngreen ? partials[j * 2 + 1] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
          tot[0] += v[k][0];
          tot[1] += v[k][1];
        }
      }
      block_sum<2>(tot, red);
    }
    if (threadIdx.x == 0) {
      TransportState nx = cur.pend ? transport_judge(ctl, cur, tot[0], tot[1], ntot) : cur;
      nx.pend = nx.done ? 0 : 1;  // the green pass of this iteration will run
      if (blockIdx.x == 0 && blockIdx.y == 0) ctl->st[par ^ 1] = nx;
      s_stop = nx.done;
    }
    __syncthreads();
    if (s_stop) return;
  }
  // workgroup kinds: c = 0, 1 (axis c, output G_c), 2 (axis z, output f_z),
  // 3 (axis z, output tau_z): four kinds of equal work (one inverse and one
  // forward slab transform each)
  const int z = blockIdx.x, c = blockIdx.y, ax = c < 2 ? c : 2;
  const int64_t soff = (int64_t)z * N * S::XH;
  const SlabTw<T> tws = slab_twiddles<T, N, N>(lds, twx_g, twy_g, rtw_g);
  const cplx<T>*twx = tws.x, *twy = tws.y, *rtw = tws.r;
  slab_load_lds<T, N, N>(lds, spec + ax * nspec + soff);
  __syncthreads();
  slab_cols_inverse<T, N, N>(lds, twy);
  slab_rows_inverse<T, N, N>(lds, twx, rtw);

  const T gc = (T)ctl->g[ax], B0c = (T)ctl->B0[ax];
  const T A0 = (T)ctl->A0, Pe = (T)ctl->Pe, eta = (T)ctl->eta, dif = (T)ctl->diff;
  const T calF = c == 0 ? (T)ctl->calF : T(0);
  const T hs = T(0.5 * (double)N);  // 1 / (2 h) with h = 1 / N
  const int64_t off = (int64_t)z * S::NV;
  const gmem<V>* uq = as_global(reinterpret_cast<const V*>(u + ax * ntot + off));
  const gmem<uint32_t>* hq = as_global(reinterpret_cast<const uint32_t*>(H + off));
  V zero;
  zero.x = zero.y = zero.z = zero.w = T(0);
  // tau and f of a quad from its d chi (ev), flow component (uv) and H bytes
  auto quad = [&](const V& ev, const V& uv, uint32_t hw, V& tau, V& f) {
    const T e4[4] = {ev.x + gc, ev.y + gc, ev.z + gc, ev.w + gc};
    const T u4[4] = {uv.x, uv.y, uv.z, uv.w};
    T t4[4], f4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const bool solid = ((hw >> (8 * k)) & 0xffu) != 0;
      const T Aa = solid ? eta : dif;
      const T Bc = solid ? T(0) : Pe * u4[k];
      f4[k] = (solid ? T(0) : calF) - (Bc - B0c) * e4[k];
      t4[k] = (Aa - A0) * e4[k];
    }
    tau.x = t4[0];
    tau.y = t4[1];
    tau.z = t4[2];
    tau.w = t4[3];
    f.x = f4[0];
    f.y = f4[1];
    f.z = f4[2];
    f.w = f4[3];
  };
  const int xq = threadIdx.x % RG, grp = threadIdx.x / RG;
  const bool xin = xq < R;
  if (c == 0) {
    // G_x = f_x + D_x tau_x, row group grp taking rows p NG + grp
    const int gb = (threadIdx.x & 63) & ~(RG - 1);  // first lane of the row group
    const int src_l = gb + (xq == 0 ? R - 1 : xq - 1), src_r = gb + (xq >= R - 1 ? 0 : xq + 1);
#pragma unroll
    for (int p = 0; p < PX; ++p) {
      const int y = p * NG + grp;
      const bool act = xin && y < N;
      V tau = zero, f = zero;
      T* cell = ldsr + (act ? y : 0) * 2 * S::P2 + 4 * (act ? xq : 0);
      if (act) {
        const int q = y * R + xq;
        quad(lds_ld4<V>(cell), uq[q], hq[q], tau, f);
      }
      const T left = __shfl(tau.w, src_l, 64), right = __shfl(tau.x, src_r, 64);
      if (act) {
        V G;
        G.x = f.x + hs * (tau.y - left);
        G.y = f.y + hs * (tau.z - tau.x);
        G.z = f.z + hs * (tau.w - tau.y);
        G.w = f.w + hs * (right - tau.z);
        lds_st4(cell, G);
      }
    }
  } else if (c == 1) {
    // G_y = f_y + D_y tau_y, each thread walking rows y0 .. y1-1 of quad
    // column xq with a window of three rows
    const int y0 = grp * RPS, y1 = min(N, y0 + RPS);
    const bool act = xin && y0 < N;
    V tlo = zero, thi = zero;
    if (act) {
      const int ylo = y0 == 0 ? N - 1 : y0 - 1, yhi = y1 == N ? 0 : y1;
      V f;
      quad(lds_ld4<V>(ldsr + ylo * 2 * S::P2 + 4 * xq), zero, hq[ylo * R + xq], tlo, f);
      quad(lds_ld4<V>(ldsr + yhi * 2 * S::P2 + 4 * xq), zero, hq[yhi * R + xq], thi, f);
    }
    __syncthreads();  // the bounding rows are read before any strip is overwritten
    if (act) {
      V tm = tlo, tc, fc;
      {
        const int q = y0 * R + xq;
        quad(lds_ld4<V>(ldsr + y0 * 2 * S::P2 + 4 * xq), uq[q], hq[q], tc, fc);
      }
#pragma unroll
      for (int k = 0; k < RPS; ++k) {
        const int y = y0 + k;
        if (y < y1) {
          V tn = thi, fn = zero;
          if (y + 1 < y1) {
            const int q = (y + 1) * R + xq;
            quad(lds_ld4<V>(ldsr + (y + 1) * 2 * S::P2 + 4 * xq), uq[q], hq[q], tn, fn);
          }
          V G;
          G.x = fc.x + hs * (tn.x - tm.x);
          G.y = fc.y + hs * (tn.y - tm.y);
          G.z = fc.z + hs * (tn.z - tm.z);
          G.w = fc.w + hs * (tn.w - tm.w);
          lds_st4(ldsr + y * 2 * S::P2 + 4 * xq, G);
          tm = tc;
          tc = tn;
          fc = fn;
        }
      }
    }
  } else {
    // f_z (c = 2) or tau_z (c = 3) in place
#pragma unroll
    for (int j = 0; j < S::QPT; ++j) {
      const int q = threadIdx.x + j * S::NT;
      if (!S::FULL && q >= S::NQ) continue;
      const int v = 4 * q;
      const int y = v / N, x = v - y * N;
      T* cell = ldsr + y * 2 * S::P2 + x;
      V tau, f, uv = zero;
      if (c == 2) uv = uq[q];
      quad(lds_ld4<V>(cell), uv, hq[q], tau, f);
      lds_st4(cell, c == 3 ? tau : f);
    }
  }
  __syncthreads();
  // G_x, G_y into the field this workgroup read; tau_z into field 3 and f_z
  // into field 4 (field 2 is read by both z workgroups of this slab)
  slab_forward_store<T, N, N>(lds, spec + (c < 2 ? c : (c == 3 ? 3 : 4)) * nspec + soff, twx, twy,
                              rtw);
}

// ------------------------------------------------------------------ launchers
template <typename T, int LL>
static int tg_blocks(const Geom& g, bool slab, bool flux) {
  int tx;
  if (g.dim == 3)
    tx = flux ? TGCfg<T, LL, tg_fields<3, false, true>()>::TX
              : (slab ? TGCfg<T, LL, tg_fields<3, true>()>::TX
                      : TGCfg<T, LL, tg_fields<3, false>()>::TX);
  else
    tx = flux ? TGCfg<T, LL, tg_fields<2, false, true>()>::TX : TGCfg<T, LL, tg_fields<2, false>()>::TX;
  return (int)((g.plane + tx - 1) / tx);
}

int transport_green_blocks(const Geom& g, int prec_bytes, bool slab, bool flux) {
  switch (g.last_n) {
#define CASE(LL) \
  case LL:       \
    return prec_bytes == 8 ? tg_blocks<double, LL>(g, slab, flux) : tg_blocks<float, LL>(g, slab, flux);
    ACM_COL_LENGTHS(CASE)
#undef CASE
    default:
      return -1;
  }
}

template <typename T>
hipError_t launch_transport_green(const Geom& g, const DevTables<T>& tb, int mode, void* spec,
                                  void* chat, const void* chat_m, double* partials,
                                  TransportCtl* ctl, int slab, int par, int judge,
                                  hipStream_t s, int flux) {
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  const T* rt = tb.rtab;
  if (flux && slab) return hipErrorInvalidValue;
  TGreenGeom gg{g.dim, g.nx, g.xh, g.ny, g.nz, (int)g.plane, g.nspec, g.ntot};
  const cplx<T>* tw = ct + (g.dim == 3 ? tb.off.tw_z : tb.off.tw_y);
  auto* sp = reinterpret_cast<cplx<T>*>(spec);
  auto* cp = reinterpret_cast<cplx<T>*>(chat);
  auto* cm = reinterpret_cast<const cplx<T>*>(chat_m);
#define LAUNCH_TG1(LL, DD, MM, SLB, FLX)                                                     \
  {                                                                                          \
    using C = TGCfg<T, LL, tg_fields<DD, SLB, FLX>()>;                                       \
    const int nb = (int)((g.plane + C::TX - 1) / C::TX);                                     \
    ACM_LAUNCH((k_transport_green<T, LL, DD, MM, SLB, FLX>), dim3(nb), dim3(C::NT),          \
                       C::LDS_BYTES + Plan<LL>::tw_total * (int)sizeof(cplx<T>), s, sp, cp, cm,  \
                       partials, ctl, gg, par, judge,                                          \
                       tw,                                                                   \
                       rt + tb.off.sx,                                                       \
                       rt + tb.off.lx, rt + tb.off.sy, rt + tb.off.ly, rt + tb.off.sz,       \
                       rt + tb.off.lz);                                                      \
  }
  switch (g.last_n) {
#define CASE(LL)                                                      \
  case LL:                                                            \
    if (g.dim == 3) {                                                 \
      if (mode == 0 && slab) LAUNCH_TG1(LL, 3, 0, true, false)        \
      else if (mode == 0 && flux) LAUNCH_TG1(LL, 3, 0, false, true)   \
      else if (mode == 0) LAUNCH_TG1(LL, 3, 0, false, false)          \
      else if (flux) LAUNCH_TG1(LL, 3, 1, false, true)                \
      else LAUNCH_TG1(LL, 3, 1, false, false)                         \
    } else {                                                          \
      if (mode == 0 && flux) LAUNCH_TG1(LL, 2, 0, false, true)        \
      else if (mode == 0) LAUNCH_TG1(LL, 2, 0, false, false)          \
      else if (flux) LAUNCH_TG1(LL, 2, 1, false, true)                \
      else LAUNCH_TG1(LL, 2, 1, false, false)                         \
    }                                                                 \
    return hipGetLastError();
    ACM_COL_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
#undef LAUNCH_TG1
}

template <typename T>
hipError_t launch_transport_local(const Geom& g, const DevTables<T>& tb, void* spec, const T* u,
                                  const uint8_t* H, const TransportCtl* ctl, hipStream_t s,
                                  int flux) {
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  auto* sp = reinterpret_cast<cplx<T>*>(spec);
#define LAUNCH_TL(MM, DD, FLX)                                                                \
  {                                                                                           \
    using C = RowCfgN<T, MM, FLX ? 2 * DD : DD + 1>;                                          \
    dim3 grid((unsigned)((g.nrows + C::RB - 1) / C::RB));                                     \
    ACM_LAUNCH((k_transport_local<T, MM, DD, FLX>), grid, dim3(C::NT), C::LDS_BYTES, s, sp,   \
               u, H, ctl, (int)g.nrows, g.ny, g.nz, g.ntot, g.nspec, ct + tb.off.tw_x,        \
               ct + tb.off.rtw);                                                              \
  }
  switch (g.nx / 2) {
#define CASE(MM)                    \
  case MM:                          \
    if (g.dim == 3 && flux)         \
      LAUNCH_TL(MM, 3, true)        \
    else if (g.dim == 3)            \
      LAUNCH_TL(MM, 3, false)       \
    else if (flux)                  \
      LAUNCH_TL(MM, 2, true)        \
    else                            \
      LAUNCH_TL(MM, 2, false)       \
    return hipGetLastError();
    ACM_ROW_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
#undef LAUNCH_TL
}

template <typename T>
hipError_t launch_transport_slab(const Geom& g, const DevTables<T>& tb, void* spec, const T* u,
                                 const uint8_t* H, TransportCtl* ctl, const double* partials,
                                 int ngreen, int par, hipStream_t s) {
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  auto* sp = reinterpret_cast<cplx<T>*>(spec);
  if (g.dim != 3 || g.nx != g.ny) return hipErrorInvalidValue;
  dim3 grid((unsigned)g.nz, 4u, 1u);
  switch (g.nx) {
#define CASE(NN)                                                                                \
  case NN: {                                                                                    \
    using S = SlabCfg<T, NN, NN>;                                                               \
    ACM_LAUNCH((k_transport_slab<T, NN>), grid, dim3(S::NT), S::LDS_BYTES, s, sp, u, H, ctl,    \
               partials, ngreen, par, g.ntot, g.nspec, ct + tb.off.tw_x, ct + tb.off.tw_y,      \
               ct + tb.off.rtw);                                                                \
    return hipGetLastError();                                                                   \
  }
    ACM_SLAB_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

#define INST(T)                                                                              \
  template hipError_t launch_transport_green<T>(const Geom&, const DevTables<T>&, int, void*, \
                                                void*, const void*, double*, TransportCtl*,  \
                                                int, int, int, hipStream_t, int);            \
  template hipError_t launch_transport_slab<T>(const Geom&, const DevTables<T>&, void*,       \
                                               const T*, const uint8_t*, TransportCtl*,      \
                                               const double*, int, int, hipStream_t);        \
  template hipError_t launch_transport_local<T>(const Geom&, const DevTables<T>&, void*,      \
                                                const T*, const uint8_t*,                    \
                                                const TransportCtl*, hipStream_t, int);
INST(float)
INST(double)
#undef INST

}  // namespace acm
