// Shared pieces of the fused xy-slab passes (Stokes and transport): the slab
// configuration (workgroup size, LDS pitch, occupancy target), the column
// transforms of a slab held in LDS, and the forward half (rows, columns,
// store) that turns a real slab into its half spectrum.
#pragma once
#include "pass_common.hpp"

namespace acm {

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  using type = float4;
};
template <>
struct Vec4<double> {
  using type = double4;
};


// 4 consecutive reals of an LDS row (8-byte aligned)
template <typename V, typename T>
__device__ __forceinline__ V lds_ld4(const T* p) {
  V v;
  v.x = p[0];
  v.y = p[1];
  v.z = p[2];
  v.w = p[3];
  return v;
}
template <typename V, typename T>
__device__ __forceinline__ void lds_st4(T* p, const V& v) {
  p[0] = v.x;
  p[1] = v.y;
  p[2] = v.z;
  p[3] = v.w;
}

template <typename T, int NX, int NY>
struct SlabCfg {
  static constexpr int M = NX / 2;
  static constexpr int XH = M + 1;
  // row pitch in complex values: odd, so the elements of a column (2 P2 dwords
  // apart) fall in different LDS banks for the column transforms
  static constexpr int P2 = XH;
  static constexpr int TPPY = Plan<NY>::TPP;
  static constexpr int TPPX = Plan<M>::TPP;
  // NT_EVEN: workgroup of TPPY * M/2 threads (XH columns in three rounds, the
  // last one column) instead of enough threads for two rounds; measured
  // faster at 128^2, where 512 threads leave room for two workgroups per CU.
  // PF: state loads issued before the slab load (2: u, H and a; 1: u and H,
  // a after the column transforms; 0: each quad's state is loaded in the
  // pointwise loop, which keeps the fewest registers live; measured fastest).
  // UNR: unroll of the pointwise loop (with PF = 0 its loads sit in it).
  static constexpr bool NT_EVEN = (NX == 128);
  static constexpr int PF = 0;
  static constexpr int NT0 = NT_EVEN ? ((TPPY * (M / 2) + 63) / 64) * 64
                                     : ((TPPY * ((XH + 1) / 2) + 63) / 64) * 64;
  static constexpr int NT = NT0 < 64 ? 64 : (NT0 > 1024 ? 1024 : NT0);
  static constexpr int GY = NT / TPPY;  // column groups per round
  static constexpr int GX = NT / TPPX;  // row groups per round
  // PACK: the DC and Nyquist columns (k = 0 and M), whose y transforms are
  // Hermitian in the inverse direction and real in the forward one, share
  // one complex column transform (column 0 carries X_0 + i X_M) where that
  // saves a round of column transforms (XH = M + 1 columns in rounds of GY:
  // at 128^2, 64 columns in two rounds instead of 65 in three).
  static constexpr bool PACK = (XH - 1 + GY - 1) / GY < (XH + GY - 1) / GY;
  static constexpr int XC = PACK ? XH - 1 : XH;  // columns transformed
  // the slab, then the twiddles of the x rows, the y columns and the
  // real-pair step of the row transforms
  static constexpr int TWX = Plan<M>::tw_total, TWY = Plan<NY>::tw_total, TWR = M + 1;
  static constexpr int SLAB_BYTES = NY * P2 * (int)sizeof(cplx<T>);
  static constexpr int LDS_BYTES = SLAB_BYTES + (TWX + TWY + TWR) * (int)sizeof(cplx<T>);
  static constexpr int NV = NX * NY;                     // voxels per slab
  static constexpr int NQ = NV / 4;                       // quads per slab
  static constexpr int QPT = (NQ + NT - 1) / NT;          // quads per thread
  static constexpr bool FULL = (NQ % NT) == 0;
  static constexpr int UNR = QPT;
  // loads in flight per thread when the rhs pass sums the partials (its state
  // loads are already in registers then)
  static constexpr int SUM_U = 2;
  // Waves per SIMD that let as many workgroups reside per CU as LDS allows
  // (CDNA: 4 SIMDs and 160 KB of LDS per CU; at most 4 workgroups counted):
  // the minimum occupancy requested from the register allocator.
  static constexpr int BLK_LDS = (160 * 1024) / (LDS_BYTES + 1024);
  static constexpr int WPE = cmax(1, cmin(8, (cmin(BLK_LDS, 4) * (NT / 64) + 3) / 4));
  // the single-launch pass keeps more state in registers: two workgroups
  static constexpr int WPE_ONE = cmax(1, cmin(8, (cmin(BLK_LDS, 2) * (NT / 64) + 3) / 4));
};

// Geometry of the contiguous copies of a whole half-spectrum slab (NY * XH
// complex values; in LDS its pitch P2 equals XH) in 16-byte vectors.
template <typename T, int NX, int NY>
struct SlabCopy {
  using S = SlabCfg<T, NX, NY>;
  static constexpr int BYTES = NY * S::XH * (int)sizeof(cplx<T>);
  static_assert(BYTES % 16 == 0, "slab size must be a multiple of 16 bytes");
  static constexpr int NV = BYTES / 16;
  static constexpr int PT = (NV + S::NT - 1) / S::NT;
  static constexpr bool EVEN = (NV % S::NT) == 0;
};

// Load the half-spectrum slab `src` into LDS with 16-byte accesses, every
// load of a thread issued before the first LDS write: the slab arrives in one
// memory round trip rather than one per element (a loop that stores each
// loaded value to LDS waits on every load in turn).  In two halves, so that
// a kernel can do other work while the loads are in flight:
// slab_load_regs issues them (into b), slab_regs_to_lds writes them.
template <typename T, int NX, int NY, int PT>
__device__ __forceinline__ void slab_load_regs(float4 (&b)[PT], const cplx<T>* __restrict__ src) {
  using C = SlabCopy<T, NX, NY>;
  static_assert(PT == C::PT, "register stage of the slab's size");
  constexpr int NT = SlabCfg<T, NX, NY>::NT;
  const gmem<float4>* s = as_global(reinterpret_cast<const float4*>(src));
  // every load is unconditional (the tail re-reads the last vector), so
  // none waits inside a branch for the loads before it
#pragma unroll
  for (int j = 0; j < C::PT; ++j) {
    const int i = threadIdx.x + j * NT;
    b[j] = s[(C::EVEN || i < C::NV) ? i : C::NV - 1];
  }
}
template <typename T, int NX, int NY, int PT>
__device__ __forceinline__ void slab_regs_to_lds(cplx<T>* lds, const float4 (&b)[PT]) {
  using C = SlabCopy<T, NX, NY>;
  static_assert(PT == C::PT, "register stage of the slab's size");
  constexpr int NT = SlabCfg<T, NX, NY>::NT;
  float4* d = reinterpret_cast<float4*>(lds);
#pragma unroll
  for (int j = 0; j < C::PT; ++j) {
    const int i = threadIdx.x + j * NT;
    if (C::EVEN || i < C::NV) d[i] = b[j];
  }
}
template <typename T, int NX, int NY>
__device__ __forceinline__ void slab_load_lds(cplx<T>* lds, const cplx<T>* __restrict__ src) {
  float4 b[SlabCopy<T, NX, NY>::PT];
  slab_load_regs<T, NX, NY>(b, src);
  slab_regs_to_lds<T, NX, NY>(lds, b);
}

// The twiddle tables of a slab pass, copied into LDS after the slab.  Every
// butterfly stage of every column or row round reads its twiddles; from
// global memory each stage waited on their loads, from LDS they arrive with
// the stage's data (and lanes at the same pencil position read the same
// address).  The copy needs a barrier before the first transform.
template <typename T>
struct SlabTw {
  const cplx<T>* x;
  const cplx<T>* y;
  const cplx<T>* r;
};
template <typename T, int NX, int NY>
__device__ __forceinline__ SlabTw<T> slab_twiddles(cplx<T>* lds, const cplx<T>* __restrict__ twx,
                                                   const cplx<T>* __restrict__ twy,
                                                   const cplx<T>* __restrict__ rtw) {
  using S = SlabCfg<T, NX, NY>;
  constexpr int NTW = S::TWX + S::TWY + S::TWR;
  cplx<T>* t = lds + NY * S::P2;
  batched_copy<cplx<T>, S::NT, NTW>(
      NTW,
      [&](int e) {
        return e < S::TWX ? twx[e] : (e < S::TWX + S::TWY ? twy[e - S::TWX] : rtw[e - S::TWX - S::TWY]);
      },
      [&](int e, const cplx<T>& v) { t[e] = v; });
  return SlabTw<T>{t, t + S::TWX, t + S::TWX + S::TWY};
}

// Store the half-spectrum slab held in LDS (contiguous, pitch XH) to `dst`
// with 16-byte accesses, the LDS reads of a chunk of U vectors issued
// together (LDS latency is short: small chunks keep few registers live).
template <typename T, int NX, int NY, int U = 4>
__device__ __forceinline__ void slab_store_lds(cplx<T>* __restrict__ dst, const cplx<T>* lds) {
  using St = SlabCopy<T, NX, NY>;
  constexpr int NT = SlabCfg<T, NX, NY>::NT;
  const float4* s = reinterpret_cast<const float4*>(lds);
  gmem<float4>* d = as_global(reinterpret_cast<float4*>(dst));
#pragma unroll
  for (int j0 = 0; j0 < St::PT; j0 += U) {
    float4 b[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int i = threadIdx.x + (j0 + k) * NT;
      b[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (j0 + k < St::PT && (St::EVEN || i < St::NV)) b[k] = s[i];
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int i = threadIdx.x + (j0 + k) * NT;
      if (j0 + k < St::PT && (St::EVEN || i < St::NV)) d[i] = b[k];
    }
  }
}

// y transform of the XC columns of the slab held in LDS ([y][k], pitch P2).
template <typename T, int NX, int NY, int SIGN>
__device__ __forceinline__ void slab_cols(cplx<T>* lds, const cplx<T>* __restrict__ tw) {
  using S = SlabCfg<T, NX, NY>;
  // column index fastest across the lanes: every lane of a wave is at the
  // same point of its pencil, so each LDS access of every stage touches
  // consecutive complex values (no bank conflicts) and the twiddles are
  // uniform across the wave
  const int grp = threadIdx.x % S::GY, t = threadIdx.x / S::GY;
#pragma unroll 1
  for (int c0 = 0; c0 < S::XC; c0 += S::GY) {
    const int col = c0 + grp;
    const bool act = t < S::TPPY && col < S::XC;
    PencilFFT<T, NY, 1, SIGN>::run_lds(t, act, lds + (act ? col : 0), 0, S::P2, tw);
    __syncthreads();
  }
}

// Inverse y transforms of a half-spectrum slab in LDS (after a barrier that
// follows its load).  With PACK, column 0 first takes X_0 + i X_M: both
// columns are Hermitian in y, so their inverse transforms are real and come
// out as the real and imaginary parts of column 0, which is how the row
// transforms then read them.
template <typename T, int NX, int NY>
__device__ __forceinline__ void slab_cols_inverse(cplx<T>* lds, const cplx<T>* __restrict__ twy) {
  using S = SlabCfg<T, NX, NY>;
  if constexpr (S::PACK) {
    for (int y = threadIdx.x; y < NY; y += S::NT) {
      cplx<T>* r = lds + y * S::P2;
      const cplx<T> a = r[0], b = r[S::M];
      r[0] = cmake<T>(a.x - b.y, a.y + b.x);
    }
    __syncthreads();
  }
  slab_cols<T, NX, NY, +1>(lds, twy);
}

// Forward y transforms of the slab in LDS after the row transforms.  With
// PACK, column 0 holds z = X_0 + i X_M of two real columns; their transforms
// are (Z_k + conj Z_-k) / 2 and (Z_k - conj Z_-k) / 2i, written to columns 0
// and M.  Ends with a barrier.
template <typename T, int NX, int NY>
__device__ __forceinline__ void slab_cols_forward(cplx<T>* lds, const cplx<T>* __restrict__ twy) {
  using S = SlabCfg<T, NX, NY>;
  slab_cols<T, NX, NY, -1>(lds, twy);
  if constexpr (S::PACK) {
    for (int k = threadIdx.x; k <= NY / 2; k += S::NT) {
      const int km = k == 0 ? 0 : NY - k;
      cplx<T>* rk = lds + k * S::P2;
      cplx<T>* rm = lds + km * S::P2;
      const cplx<T> zk = rk[0], zm = rm[0];
      const cplx<T> e = cmake<T>(T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y));  // (Z_k + conj Z_-k)/2
      const cplx<T> o = cmake<T>(T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x));  // (Z_k - conj Z_-k)/2i
      rk[0] = e;
      rk[S::M] = o;
      rm[0] = cconj(e);
      rm[S::M] = cconj(o);
    }
    __syncthreads();
  }
}

// x transforms of the NY rows of a slab in LDS (row index fastest across the
// lanes: rows are an odd number of banks apart, so every stage is
// conflict-free).  Inverse: half spectra to real rows; forward: the reverse.
template <typename T, int NX, int NY>
__device__ __forceinline__ void slab_rows_inverse(cplx<T>* lds, const cplx<T>* __restrict__ twx,
                                                  const cplx<T>* __restrict__ rtw) {
  using S = SlabCfg<T, NX, NY>;
  const int grp = threadIdx.x % S::GX, t = threadIdx.x / S::GX;
#pragma unroll 1
  for (int r0 = 0; r0 < NY; r0 += S::GX) {
    const int row = r0 + grp;
    const bool act = t < S::TPPX && row < NY;
    rows_c2r_lds<T, S::M, 1, S::P2, S::PACK>(lds, 0, act ? row : 0, t, act, twx, rtw);
  }
}
template <typename T, int NX, int NY>
__device__ __forceinline__ void slab_rows_forward(cplx<T>* lds, const cplx<T>* __restrict__ twx,
                                                  const cplx<T>* __restrict__ rtw) {
  using S = SlabCfg<T, NX, NY>;
  const int grp = threadIdx.x % S::GX, t = threadIdx.x / S::GX;
#pragma unroll 1
  for (int r0 = 0; r0 < NY; r0 += S::GX) {
    const int row = r0 + grp;
    const bool act = t < S::TPPX && row < NY;
    rows_r2c_lds<T, S::M, 1, S::P2, S::PACK>(lds, 0, act ? row : 0, t, act, twx, rtw);
  }
}

// Forward half of the rhs pass on a real slab held in LDS (rows of pitch
// 2 P2 reals): x transforms of the rows, y transforms of the columns, store.
template <typename T, int NX, int NY>
__device__ __forceinline__ void slab_forward_store(cplx<T>* lds, cplx<T>* __restrict__ dst,
                                                   const cplx<T>* __restrict__ twx,
                                                   const cplx<T>* __restrict__ twy,
                                                   const cplx<T>* __restrict__ rtw) {
  slab_rows_forward<T, NX, NY>(lds, twx, rtw);
  slab_cols_forward<T, NX, NY>(lds, twy);
  slab_store_lds<T, NX, NY>(dst, lds);
}

// Load the half-spectrum slab `src` ([y][k], k < XH) into LDS and take it back
// to real space: inverse y transforms of the columns, then inverse x
// transforms of the rows.  Row y of the result starts at real offset
// y * 2 * P2.  Ends with a barrier.


// Square slab lengths compiled for the fused passes.
#define ACM_SLAB_LENGTHS(X) X(32) X(48) X(64) X(96) X(128)

}  // namespace acm
