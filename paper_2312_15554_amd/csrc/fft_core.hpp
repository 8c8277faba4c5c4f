// Device-side building blocks: complex arithmetic, compile-time mixed-radix
// plans and a Stockham autosort FFT over pencils held in LDS.
//
// Pencil FFT (length L = 2^a 3^b): stages of radix 8/4/2 followed by radix 3.
// Stage s with radix R and sub-length Ns (product of the earlier radices):
// butterfly j in [0, L/R) reads elements j + r L/R, multiplies element r by
// w^(r k) with k = j mod Ns and w = exp(sign 2 pi i / (Ns R)), applies the
// radix-R DFT and writes outputs to (j div Ns) Ns R + k + r Ns.  After the last
// stage the pencil holds its DFT in natural order (no bit reversal pass).
// Twiddles come from an FP64-computed table stored in the working precision.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace acm {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmake(T a, T b) {
  cplx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return cmake<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return cmake<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return cmake<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return cmake<T>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return cmake<T>(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) { return cmake<T>(a.x * s, a.y * s); }
// multiply by sign*i
template <int SIGN, typename T>
__device__ __forceinline__ cplx<T> cmul_i(cplx<T> a) {
  return SIGN > 0 ? cmake<T>(-a.y, a.x) : cmake<T>(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// Compile-time radix plan
// ---------------------------------------------------------------------------
struct RadixPlan {
  int n;
  int nst;
  int r[12];
  int ns[12];
  int tw[12];  // offset of the stage's twiddles in the table
  int tw_total;
  bool ok;
};

constexpr RadixPlan make_plan(int L) {
  RadixPlan p{};
  p.n = L;
  int m = L;
  int threes = 0;
  while (m % 3 == 0) {
    m /= 3;
    ++threes;
  }
  int k = 0;
  while (m % 8 == 0 && m > 0) {
    p.r[k++] = 8;
    m /= 8;
  }
  if (m % 4 == 0) {
    p.r[k++] = 4;
    m /= 4;
  }
  if (m % 2 == 0) {
    p.r[k++] = 2;
    m /= 2;
  }
  for (int t = 0; t < threes; ++t) p.r[k++] = 3;
  p.ok = (m == 1) && k > 0;
  p.nst = k;
  int ns = 1, off = 0;
  for (int s = 0; s < k; ++s) {
    p.ns[s] = ns;
    p.tw[s] = off;
    off += ns * (p.r[s] - 1);
    ns *= p.r[s];
  }
  p.tw_total = off;
  return p;
}

template <int L>
struct Plan {
  static constexpr RadixPlan P = make_plan(L);
  static_assert(P.ok, "FFT length must be 2^a 3^b");
  static constexpr int nst = P.nst;
  static constexpr int TPP = L / P.r[0];  // threads per pencil
  static constexpr int radix(int s) { return P.r[s]; }
  static constexpr int ns(int s) { return P.ns[s]; }
  static constexpr int twoff(int s) { return P.tw[s]; }
  static constexpr int tw_total = P.tw_total;
  static constexpr int max_elems() {
    int m = 0;
    for (int s = 0; s < P.nst; ++s) {
      int nb = L / P.r[s];
      int per = (nb + TPP - 1) / TPP;
      if (per * P.r[s] > m) m = per * P.r[s];
    }
    return m;
  }
};

// ---------------------------------------------------------------------------
// Small DFTs (in registers). SIGN = -1 forward, +1 inverse.
// ---------------------------------------------------------------------------
template <int R, int SIGN, typename T>
struct Dft;

template <int SIGN, typename T>
struct Dft<2, SIGN, T> {
  __device__ __forceinline__ static void run(cplx<T>* v) {
    cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int SIGN, typename T>
struct Dft<3, SIGN, T> {
  __device__ __forceinline__ static void run(cplx<T>* v) {
    const T c1 = T(-0.5);
    const T s1 = T(SIGN) * T(0.86602540378443864676372317075293618);
    cplx<T> a = v[0], b = v[1], c = v[2];
    cplx<T> t = cadd(b, c);
    cplx<T> d = csub(b, c);
    v[0] = cadd(a, t);
    cplx<T> m = cmake<T>(a.x + c1 * t.x, a.y + c1 * t.y);
    // i*s1*d = (-s1 d.y, s1 d.x)
    cplx<T> n = cmake<T>(-s1 * d.y, s1 * d.x);
    v[1] = cadd(m, n);
    v[2] = csub(m, n);
  }
};

template <int SIGN, typename T>
struct Dft<4, SIGN, T> {
  __device__ __forceinline__ static void run(cplx<T>* v) {
    cplx<T> a0 = cadd(v[0], v[2]);
    cplx<T> a1 = csub(v[0], v[2]);
    cplx<T> b0 = cadd(v[1], v[3]);
    cplx<T> b1 = cmul_i<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, b1);
    v[3] = csub(a1, b1);
  }
};

template <int SIGN, typename T>
struct Dft<8, SIGN, T> {
  __device__ __forceinline__ static void run(cplx<T>* v) {
    const T r2 = T(0.70710678118654752440084436210484904);
    // split even/odd radix-4
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, SIGN, T>::run(e);
    Dft<4, SIGN, T>::run(o);
    // twiddles w8^k, w8 = exp(SIGN*i*pi/4)
    cplx<T> o1 = cmake<T>(r2 * (o[1].x - T(SIGN) * o[1].y), r2 * (o[1].y + T(SIGN) * o[1].x));
    cplx<T> o2 = cmul_i<SIGN>(o[2]);
    cplx<T> o3 = cmake<T>(r2 * (-o[3].x - T(SIGN) * o[3].y), r2 * (-o[3].y + T(SIGN) * o[3].x));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// ---------------------------------------------------------------------------
// Pencil FFT over NP pencils per thread group, stages exchanged through LDS.
//
// Thread t in [0, TPP) of a group of TPP threads works on NP pencils.  Pencil
// p's element i lives at lds[p*pstride + i*estride].  The whole workgroup must
// call run() together (it contains workgroup barriers); threads that own no
// pencil pass active = false but still hit every barrier.
// The first stage may read through `load(p, i)` instead of LDS and the last
// stage may write through `store(p, i, v)` instead of LDS.
// ---------------------------------------------------------------------------
template <typename T, int L, int NP, int SIGN>
struct PencilFFT {
  using PL = Plan<L>;
  static constexpr int TPP = PL::TPP;

  struct LdsLoad {
    const cplx<T>* lds;
    int pstride, estride;
    __device__ __forceinline__ cplx<T> operator()(int p, int i) const { return lds[p * pstride + i * estride]; }
  };
  struct LdsStore {
    cplx<T>* lds;
    int pstride, estride;
    __device__ __forceinline__ void operator()(int p, int i, cplx<T> v) const { lds[p * pstride + i * estride] = v; }
  };

  template <int S, class LoadF, class StoreF>
  __device__ __forceinline__ static void stage(int t, bool active, cplx<T>* lds, int pstride, int estride,
                               const cplx<T>* __restrict__ tw, const LoadF& load, const StoreF& store) {
    constexpr int R = PL::radix(S);
    constexpr int NS = PL::ns(S);
    constexpr int NB = L / R;
    constexpr int PER = (NB + TPP - 1) / TPP;
    constexpr bool FIRST = (S == 0);
    constexpr bool LAST = (S == PL::nst - 1);
    cplx<T> v[NP][PER][R];
    if (active) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int j = t + q * TPP;
        if ((NB % TPP == 0) || j < NB) {
          const int k = j % NS;
#pragma unroll
          for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
              cplx<T> x;
              if constexpr (FIRST)
                x = load(p, j + r * NB);
              else
                x = lds[p * pstride + (j + r * NB) * estride];
              v[p][q][r] = x;
            }
          }
          if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
              cplx<T> w = tw[PL::twoff(S) + k * (R - 1) + (r - 1)];
              if (SIGN > 0) w.y = -w.y;
#pragma unroll
              for (int p = 0; p < NP; ++p) v[p][q][r] = cmul(v[p][q][r], w);
            }
          }
#pragma unroll
          for (int p = 0; p < NP; ++p) Dft<R, SIGN, T>::run(v[p][q]);
        }
      }
    }
    if constexpr (!LAST || true) __syncthreads();
    if (active) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int j = t + q * TPP;
        if ((NB % TPP == 0) || j < NB) {
          const int k = j % NS;
          const int base = (j / NS) * NS * R + k;
#pragma unroll
          for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
              if constexpr (LAST)
                store(p, base + r * NS, v[p][q][r]);
              else
                lds[p * pstride + (base + r * NS) * estride] = v[p][q][r];
            }
          }
        }
      }
    }
    if constexpr (!LAST) {
      __syncthreads();
      stage<S + 1>(t, active, lds, pstride, estride, tw, load, store);
    }
  }

  // Generic entry: first stage reads via load, last stage writes via store,
  // intermediate stages use the LDS pencils.
  template <class LoadF, class StoreF>
  __device__ __forceinline__ static void run(int t, bool active, cplx<T>* lds, int pstride, int estride,
                             const cplx<T>* __restrict__ tw, const LoadF& load, const StoreF& store) {
    stage<0>(t, active, lds, pstride, estride, tw, load, store);
  }

  // In-place on LDS pencils.
  __device__ __forceinline__ static void run_lds(int t, bool active, cplx<T>* lds, int pstride, int estride,
                                 const cplx<T>* __restrict__ tw) {
    LdsLoad ld{lds, pstride, estride};
    LdsStore st{lds, pstride, estride};
    stage<0>(t, active, lds, pstride, estride, tw, ld, st);
  }
};


// ---------------------------------------------------------------------------
// Register-resident pencil FFT.  Thread t of a pencil group (TPP threads)
// holds the EPT = L / TPP elements i = t + m TPP (m in [0, EPT)) of each of
// NP pencils in v[p][m] before AND after the transform: the first stage reads
// exactly that set (its radix is EPT) and the last stage writes exactly that
// set back, so data enter and leave through registers and LDS is only used to
// exchange between stages.  Valid when every stage's butterfly count is a
// multiple of TPP (all plans without a radix-3 stage).
// ---------------------------------------------------------------------------
template <int L>
struct RegPlanOk {
  static constexpr bool value() {
    for (int s = 0; s < Plan<L>::nst; ++s)
      if ((L / Plan<L>::radix(s)) % Plan<L>::TPP != 0) return false;
    return true;
  }
};

template <typename T, int L, int NP, int SIGN>
struct RegFFT {
  using PL = Plan<L>;
  static constexpr int TPP = PL::TPP;
  static constexpr int EPT = L / TPP;
  static_assert(RegPlanOk<L>::value(), "register FFT needs TPP | L/R for every stage");

  // LDS exchange buffer: pencil p element i at lds[p*pstride + i*estride].
  template <int S>
  __device__ __forceinline__ static void stage(int t, bool active, cplx<T> (&v)[NP][EPT], cplx<T>* lds,
                               int pstride, int estride, const cplx<T>* __restrict__ tw) {
    constexpr int R = PL::radix(S);
    constexpr int NS = PL::ns(S);
    constexpr int NB = L / R;
    constexpr int PER = NB / TPP;
    constexpr bool FIRST = (S == 0);
    constexpr bool LAST = (S == PL::nst - 1);
    cplx<T> w[NP][PER][R];
    if (active) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int j = t + q * TPP;
        const int k = j % NS;
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if constexpr (FIRST)
              w[p][q][r] = v[p][r];  // element t + r TPP
            else
              w[p][q][r] = lds[p * pstride + (j + r * NB) * estride];
          }
        if constexpr (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            cplx<T> tt = tw[PL::twoff(S) + k * (R - 1) + (r - 1)];
            if (SIGN > 0) tt.y = -tt.y;
#pragma unroll
            for (int p = 0; p < NP; ++p) w[p][q][r] = cmul(w[p][q][r], tt);
          }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) Dft<R, SIGN, T>::run(w[p][q]);
      }
    }
    if constexpr (LAST) {
      // outputs at j + r NB = t + (q + r PER) TPP: the natural set again
      if (active) {
#pragma unroll
        for (int q = 0; q < PER; ++q)
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int p = 0; p < NP; ++p) v[p][q + r * PER] = w[p][q][r];
      }
    } else {
      if constexpr (!FIRST) __syncthreads();  // everyone has read the buffer
      if (active) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          const int j = t + q * TPP;
          const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
          for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int r = 0; r < R; ++r) lds[p * pstride + (base + r * NS) * estride] = w[p][q][r];
        }
      }
      __syncthreads();
      stage<S + 1>(t, active, v, lds, pstride, estride, tw);
    }
  }

  // The whole workgroup calls run() together; it contains workgroup barriers
  // (and ends with none: the caller synchronises before reusing `lds`).
  __device__ __forceinline__ static void run(int t, bool active, cplx<T> (&v)[NP][EPT], cplx<T>* lds,
                             int pstride, int estride, const cplx<T>* __restrict__ tw) {
    stage<0>(t, active, v, lds, pstride, estride, tw);
  }
};

// Workgroup-wide FP64 sum of NV values per thread.  Returns the totals in
// thread 0 (valid only there).  `red` must hold NV * (blockDim/64) doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    v[k] = x;
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * nw + wave] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[k * nw + w];
      v[k] = s;
    }
  }
  __syncthreads();
}

}  // namespace acm
