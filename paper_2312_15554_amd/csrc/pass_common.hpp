// Device helpers shared by every pass kernel: real<->half-complex transforms of
// x rows held in LDS, and the column (strided pencil) tile mapping used by the
// y and z passes.
#pragma once
#include <hip/hip_ext.h>

#include "acm_internal.hpp"
#include "fft_core.hpp"

namespace acm {

// Kernel launch used by every pass: in the profiling mode (launch_events()
// armed) the dispatch itself records its start and end; otherwise a plain
// launch.
#define ACM_LAUNCH(KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                                      \
  do {                                                                                           \
    ::acm::LaunchEvents& le_ = ::acm::launch_events();                                           \
    if (le_.start) {                                                                             \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, le_.start, le_.stop, 0,          \
                            __VA_ARGS__);                                                        \
      le_ = ::acm::LaunchEvents{};                                                               \
    } else {                                                                                     \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);                      \
    }                                                                                            \
  } while (0)

// Supported lengths.  Row kernels take the complex half length M = nx/2,
// column kernels the full axis length.
#define ACM_ROW_LENGTHS(X) X(4) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(256) X(512)
#define ACM_COL_LENGTHS(X) X(8) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(512) X(1024)

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

// Global-memory view of a pointer.  A pointer read from memory at run time
// (the per-cell argument array of batched launches) is generic to the
// compiler, which then emits flat accesses: slower to issue, and waiting on
// them also waits on every LDS access in flight.  Kernels index the arrays
// of a cell through this view.  (The host pass, which only parses kernel
// bodies, sees the plain type: it has no address space 1 for class types.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gmem = __attribute__((address_space(1))) T;
#else
template <typename T>
using gmem = T;
#endif
template <typename T>
__device__ __forceinline__ gmem<T>* as_global(T* p) {
  return (gmem<T>*)p;
}

// Workgroup-wide copy of n <= MAXN elements by NT threads: put(e, ld(e))
// for every e < n, each thread issuing all of its loads before its first
// put.  Copying into LDS this way brings the block in one memory round trip:
// a loop that writes each loaded element to LDS before loading the next
// waits on every load in turn, which leaves a workgroup idle for most of its
// load phase.
template <typename E, int NT, int MAXN, typename F, typename P>
__device__ __forceinline__ void batched_copy(int n, F ld, P put) {
  constexpr int PT = (MAXN + NT - 1) / NT;
  E b[PT];
#pragma unroll
  for (int j = 0; j < PT; ++j) {
    const int e = (int)threadIdx.x + j * NT;
    b[j] = E{};  // defined on every path: a conditional first write puts b in scratch memory
    if (e < n) b[j] = ld(e);
  }
#pragma unroll
  for (int j = 0; j < PT; ++j) {
    const int e = (int)threadIdx.x + j * NT;
    if (e < n) put(e, b[j]);
  }
}

// lds[e] = ld(e) for e < n <= MAXN (batched_copy into LDS).
template <typename E, int NT, int MAXN, typename F>
__device__ __forceinline__ void gather_to_lds(E* lds, int n, F ld) {
  batched_copy<E, NT, MAXN>(n, ld, [&](int e, const E& v) { lds[e] = v; });
}

// Copy the N twiddles of a pencil transform into LDS at dst; the stages then
// read them there rather than waiting on global loads.  Visible after the
// next barrier (the transforms read twiddles from their second stage on,
// after the barrier that ends the first).
template <typename T, int NT, int N>
__device__ __forceinline__ const cplx<T>* twiddles_to_lds(cplx<T>* dst,
                                                          const cplx<T>* __restrict__ tw) {
  batched_copy<cplx<T>, NT, N>(
      N, [&](int e) { return tw[e]; }, [&](int e, const cplx<T>& v) { dst[e] = v; });
  return dst;
}

// The reverse: st(e, lds[e]) for e < n <= MAXN, the LDS reads of U elements
// per thread issued together.
template <typename E, int NT, int MAXN, int U = 4, typename F>
__device__ __forceinline__ void scatter_from_lds(const E* lds, int n, F st) {
  constexpr int PT = (MAXN + NT - 1) / NT;
#pragma unroll
  for (int j0 = 0; j0 < PT; j0 += U) {
    E b[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int e = (int)threadIdx.x + (j0 + k) * NT;
      b[k] = E{};
      if (j0 + k < PT && e < n) b[k] = lds[e];
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int e = (int)threadIdx.x + (j0 + k) * NT;
      if (j0 + k < PT && e < n) st(e, b[k]);
    }
  }
}

// --------------------------------------------------------------------- rows
// A workgroup holds RB consecutive x rows of one field, each with pitch RP
// complex values.  TPP threads cooperate on one row.
template <typename T, int M>
struct RowCfg {
  static constexpr int TPP = Plan<M>::TPP;
  static constexpr int RP = M + 1;
  static constexpr int RB_THREADS = cmax(1, 256 / TPP);
  static constexpr int RB_LDS = cmax(1, (40 * 1024) / (RP * (int)sizeof(cplx<T>)));
  static constexpr int RB = cmin(RB_THREADS, RB_LDS);
  // block size padded to whole wavefronts; threads past TPP*RB stay idle
  static constexpr int NT = ((TPP * RB + 63) / 64) * 64;
  static constexpr int LDS_BYTES = RB * RP * (int)sizeof(cplx<T>);
};

// Row pitch RP (complex values) defaults to M + 1.
// Multi-field row blocks: NF fields, field f's rows start at lds + f*fstride.
template <typename T, int M, int NF>
struct RowCfgN {
  static constexpr int TPP = Plan<M>::TPP;
  static constexpr int RP = M + 1;
  static constexpr int RB_THREADS = cmax(1, 256 / TPP);
  static constexpr int RB_LDS = cmax(1, (48 * 1024) / (NF * RP * (int)sizeof(cplx<T>)));
  static constexpr int RB = cmin(RB_THREADS, RB_LDS);
  static constexpr int NT = ((TPP * RB + 63) / 64) * 64;
  static constexpr int FS = RB * RP;  // complex values per field block
  static constexpr int LDS_BYTES = NF * FS * (int)sizeof(cplx<T>);
};

// Turn half spectra X[0..M] of row `row` of NF fields into real rows x[0..2M)
// in place (imaginary parts of X[0] and X[M] are ignored) (the row then reads as T[2M]).  The inverse is unnormalised along
// x, so the real row equals nx * (inverse DFT of X).  Ends with a barrier.
// PK: the row holds its (real) DC and Nyquist values packed in X[0] as
// (X_0, X_M), and X[M] is not read.
template <typename T, int M, int NF = 1, int RP = M + 1, bool PK = false>
__device__ __forceinline__ void rows_c2r_lds(cplx<T>* lds, int fstride, int row, int t,
                                             bool active, const cplx<T>* __restrict__ tw,
                                             const cplx<T>* __restrict__ rtw) {
  constexpr int TPP = Plan<M>::TPP;
  if (active) {
    for (int k = t; k <= M / 2; k += TPP) {
      const cplx<T> wk = rtw[k];
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) {
        cplx<T>* r = lds + fi * fstride + row * RP;
        if (k == 0) {
          // DC and Nyquist bins of a real row are real: their imaginary parts
          // are ignored (the usual inverse real transform)
          const T x0 = r[0].x, xm = PK ? r[0].y : r[M].x;
          r[0] = cmake<T>(x0 + xm, x0 - xm);
        } else if (2 * k == M) {
          r[k] = cscale(cconj(r[k]), T(2));
        } else {
          cplx<T> xk = r[k], xm = r[M - k];
          cplx<T> S = cadd(xk, cconj(xm));
          cplx<T> D = csub(xk, cconj(xm));
          cplx<T> P = cmulc(D, wk);  // D * conj(W^k)
          r[k] = cmake<T>(S.x - P.y, S.y + P.x);
          r[M - k] = cmake<T>(S.x + P.y, P.x - S.y);  // conj(S) + i conj(P)
        }
      }
    }
  }
  __syncthreads();
  PencilFFT<T, M, NF, +1>::run_lds(t, active, lds + row * RP, fstride, 1, tw);
  __syncthreads();
}

// Turn real rows x[0..2M) (stored as M complex) of NF fields into half spectra
// X[0..M] in place (forward, unnormalised).  Ends with a barrier.
// PK: the real DC and Nyquist values go packed into X[0] as (X_0, X_M), and
// X[M] is not written.
template <typename T, int M, int NF = 1, int RP = M + 1, bool PK = false>
__device__ __forceinline__ void rows_r2c_lds(cplx<T>* lds, int fstride, int row, int t,
                                             bool active, const cplx<T>* __restrict__ tw,
                                             const cplx<T>* __restrict__ rtw) {
  constexpr int TPP = Plan<M>::TPP;
  PencilFFT<T, M, NF, -1>::run_lds(t, active, lds + row * RP, fstride, 1, tw);
  __syncthreads();
  if (active) {
    for (int k = t; k <= M / 2; k += TPP) {
      const cplx<T> wk = rtw[k];
#pragma unroll
      for (int fi = 0; fi < NF; ++fi) {
        cplx<T>* r = lds + fi * fstride + row * RP;
        if (k == 0) {
          cplx<T> z = r[0];
          if constexpr (PK) {
            r[0] = cmake<T>(z.x + z.y, z.x - z.y);
          } else {
            r[0] = cmake<T>(z.x + z.y, T(0));
            r[M] = cmake<T>(z.x - z.y, T(0));
          }
        } else if (2 * k == M) {
          r[k] = cconj(r[k]);
        } else {
          cplx<T> zk = r[k], zm = r[M - k];
          cplx<T> E = cscale(cadd(zk, cconj(zm)), T(0.5));
          cplx<T> D = csub(zk, cconj(zm));
          cplx<T> O = cmake<T>(T(0.5) * D.y, T(-0.5) * D.x);
          cplx<T> WO = cmul(wk, O);
          r[k] = cadd(E, WO);
          r[M - k] = cconj(csub(E, WO));
        }
      }
    }
  }
  __syncthreads();
}

// ------------------------------------------------------------------ columns
// Pencils along an axis of stride `as`; pencil f in [0, ncols) starts at
// (f / inner) * outer + (f % inner).  A workgroup holds TX consecutive pencils
// of NCOMP fields in LDS as [field][i][col] (col fastest).
struct ColMap {
  int inner;
  int outer;
  int as;
  int ncols;
};

// Block -> tile map that keeps runs of consecutive tiles on one XCD (blocks
// are dealt to the 8 XCDs round-robin): neighbouring tiles then share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  const int full = (nb / 8) * 8;
  if (bid >= full) return bid;
  return (bid % 8) * (nb / 8) + bid / 8;
}

__device__ __forceinline__ int col_base(const ColMap& m, int f) {
  return (f / m.inner) * m.outer + (f % m.inner);
}

// VAR selects the tile width for the autotuner: 0 = default (about 256
// threads), 1 = half of it, 2 = twice it (each capped by LDS).  SPL = 1 gives
// every field its own threads during the transforms (NCOMP times as many
// threads, each transforming one pencil: fewer registers per thread).
template <typename T, int L, int NCOMP, int VAR = 0, int SPL = 0>
struct ColCfg {
  static constexpr int TPP = Plan<L>::TPP;
  static constexpr int TX_BASE = cmax(1, 256 / TPP);
  static constexpr int TX_THREADS = cmax(1, VAR == 1 ? TX_BASE / 2
                                            : (VAR == 2 ? cmin(TX_BASE * 2, 1024 / TPP) : TX_BASE));
  static constexpr int TX_LDS = cmax(1, ((VAR == 2 ? 100 : 56) * 1024) / (NCOMP * L * (int)sizeof(cplx<T>)));
  static constexpr int TX = cmin(TX_THREADS, TX_LDS);
  // block size padded to whole wavefronts; threads with t >= TPP stay idle
  static constexpr int NT = (((SPL ? NCOMP : 1) * TPP * TX + 63) / 64) * 64;
  static_assert(NT <= 1024, "workgroup too large");
  static constexpr int LDS_BYTES = NCOMP * L * TX * (int)sizeof(cplx<T>);
};

}  // namespace acm
