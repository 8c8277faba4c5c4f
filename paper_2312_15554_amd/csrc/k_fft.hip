// Plain multi-dimensional FFT passes (no physics): real x rows <-> half
// spectra, and complex transforms along y or z.  Used to set up and read out
// the solvers and exposed through the C ABI for testing.
#include "pass_common.hpp"

namespace acm {

bool fft_length_supported(int n) {
  switch (n) {
#define CASE(L) case L:
    ACM_COL_LENGTHS(CASE)
#undef CASE
    return true;
    default:
      return false;
  }
}

template <typename T, int M>
__global__ __launch_bounds__((RowCfg<T, M>::NT)) void k_rows_r2c(const T* __restrict__ in,
                                                               cplx<T>* __restrict__ out,
                                                               int nrows, int64_t ntot,
                                                               int64_t nspec,
                                                               const cplx<T>* __restrict__ tw,
                                                               const cplx<T>* __restrict__ rtw) {
  using C = RowCfg<T, M>;
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  T* ldsr = reinterpret_cast<T*>(smem_raw);
  const int field = blockIdx.y;
  const int row0 = blockIdx.x * C::RB;
  const int nr = min(C::RB, nrows - row0);
  const gmem<T>* src = as_global(in + field * ntot + (int64_t)row0 * (2 * M));
  batched_copy<T, C::NT, C::RB * 2 * M>(
      nr * 2 * M, [&](int v) { return src[v]; },
      [&](int v, T x) {
        const int r = v / (2 * M);
        ldsr[r * 2 * C::RP + (v - r * 2 * M)] = x;
      });
  __syncthreads();
  const int row = threadIdx.x / C::TPP, t = threadIdx.x % C::TPP;
  rows_r2c_lds<T, M>(lds, 0, row, t, row < nr, tw, rtw);
  gmem<cplx<T>>* dst = as_global(out + field * nspec + (int64_t)row0 * (M + 1));
  scatter_from_lds<cplx<T>, C::NT, C::RB * (M + 1)>(lds, nr * (M + 1),
                                                    [&](int v, const cplx<T>& x) { dst[v] = x; });
}

template <typename T, int M>
__global__ __launch_bounds__((RowCfg<T, M>::NT)) void k_rows_c2r(const cplx<T>* __restrict__ in,
                                                               T* __restrict__ out, int nrows,
                                                               int64_t ntot, int64_t nspec,
                                                               T scale,
                                                               const cplx<T>* __restrict__ tw,
                                                               const cplx<T>* __restrict__ rtw) {
  using C = RowCfg<T, M>;
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  T* ldsr = reinterpret_cast<T*>(smem_raw);
  const int field = blockIdx.y;
  const int row0 = blockIdx.x * C::RB;
  const int nr = min(C::RB, nrows - row0);
  const gmem<cplx<T>>* src = as_global(in + field * nspec + (int64_t)row0 * (M + 1));
  gather_to_lds<cplx<T>, C::NT, C::RB * (M + 1)>(lds, nr * (M + 1), [&](int v) { return src[v]; });
  __syncthreads();
  const int row = threadIdx.x / C::TPP, t = threadIdx.x % C::TPP;
  rows_c2r_lds<T, M>(lds, 0, row, t, row < nr, tw, rtw);
  T* dst = out + field * ntot + (int64_t)row0 * (2 * M);
  for (int v = threadIdx.x; v < nr * 2 * M; v += C::NT) {
    const int r = v / (2 * M), x = v - r * (2 * M);
    dst[v] = ldsr[r * 2 * C::RP + x] * scale;
  }
}

// Column tiles: lengths of 256 and more take the wider tile (16 columns of
// FP32: whole 128-byte lines per row of the tile).
template <int L>
constexpr int cols_var() {
  return L >= 256 ? 2 : 0;
}

template <typename T, int L, int SIGN>
__global__ __launch_bounds__((ColCfg<T, L, 1, cols_var<L>()>::NT)) void k_cols(
    ColCellArgs one, const ColCellArgs* __restrict__ many, int64_t field_stride, ColMap m,
    const cplx<T>* __restrict__ tw) {
  using C = ColCfg<T, L, 1, cols_var<L>()>;
  const ColCellArgs ca = many ? many[blockIdx.z] : one;
  if ((ca.skip != nullptr && *ca.skip) || (ca.skip2 != nullptr && *ca.skip2)) return;
  cplx<T>* data = reinterpret_cast<cplx<T>*>(ca.data);
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  gmem<cplx<T>>* base = as_global(data + blockIdx.y * field_stride);
  // neighbouring tiles share the cache lines at their edges (rows of the half
  // spectrum are xh = nx/2 + 1 values apart): keep them on one XCD
  const int f0 = xcd_tile(blockIdx.x, gridDim.x) * C::TX;
  gather_to_lds<cplx<T>, C::NT, L * C::TX>(lds, L * C::TX, [&](int e) {
    const int i = e / C::TX, col = e - i * C::TX;
    const int f = f0 + col;
    cplx<T> v = cmake<T>(T(0), T(0));
    if (f < m.ncols) v = base[col_base(m, f) + i * m.as];
    return v;
  });
  __syncthreads();
  const int t = threadIdx.x / C::TX, col = threadIdx.x % C::TX;
  PencilFFT<T, L, 1, SIGN>::run_lds(t, t < C::TPP && f0 + col < m.ncols, lds + col, 0, C::TX, tw);
  __syncthreads();
  scatter_from_lds<cplx<T>, C::NT, L * C::TX>(lds, L * C::TX, [&](int e, const cplx<T>& v) {
    const int i = e / C::TX, col = e - i * C::TX;
    const int f = f0 + col;
    if (f < m.ncols) base[col_base(m, f) + i * m.as] = v;
  });
}

// Register-resident column transform (lengths whose plan allows the register
// FFT): each thread loads the elements t + m TPP of its column straight from
// global memory, the stages run on registers with LDS only between them, and
// the results go straight back.
template <typename T, int L, int SIGN>
__global__ __launch_bounds__((ColCfg<T, L, 1, cols_var<L>()>::NT)) void k_cols_reg(
    ColCellArgs one, const ColCellArgs* __restrict__ many, int64_t field_stride, ColMap m,
    const cplx<T>* __restrict__ tw) {
  using C = ColCfg<T, L, 1, cols_var<L>()>;
  constexpr int TPP = C::TPP;
  constexpr int EPT = L / TPP;
  constexpr int PS = L * C::TX;
  const ColCellArgs ca = many ? many[blockIdx.z] : one;
  if ((ca.skip != nullptr && *ca.skip) || (ca.skip2 != nullptr && *ca.skip2)) return;
  cplx<T>* data = reinterpret_cast<cplx<T>*>(ca.data);
  extern __shared__ __align__(16) char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  gmem<cplx<T>>* base = as_global(data + blockIdx.y * field_stride);
  const int f0 = xcd_tile(blockIdx.x, gridDim.x) * C::TX;
  const int t = threadIdx.x / C::TX, col = threadIdx.x % C::TX;
  const int f = f0 + col;
  const bool act = t < TPP && f < m.ncols;
  const int cb = act ? col_base(m, f) : 0;
  const cplx<T>* twl = twiddles_to_lds<T, C::NT, Plan<L>::tw_total>(lds + PS, tw);
  cplx<T> v[1][EPT];
  if (act) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) v[0][k] = base[cb + (t + k * TPP) * m.as];
  }
  RegFFT<T, L, 1, SIGN>::run(t, act, v, lds + col, PS, C::TX, twl);
  if (act) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) base[cb + (t + k * TPP) * m.as] = v[0][k];
  }
}

template <typename T>
hipError_t launch_rows_r2c(const Geom& g, const DevTables<T>& tb, int nfields, const T* in,
                           void* out, hipStream_t s) {
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  switch (g.nx / 2) {
#define CASE(M)                                                                            \
  case M: {                                                                                \
    using C = RowCfg<T, M>;                                                                \
    dim3 grid((unsigned)((g.nrows + C::RB - 1) / C::RB), (unsigned)nfields);               \
    ACM_LAUNCH((k_rows_r2c<T, M>), grid, dim3(C::NT), C::LDS_BYTES, s, in,          \
                       reinterpret_cast<cplx<T>*>(out), (int)g.nrows, g.ntot, g.nspec,      \
                       ct + tb.off.tw_x, ct + tb.off.rtw);                                  \
    return hipGetLastError();                                                              \
  }
    ACM_ROW_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_rows_c2r(const Geom& g, const DevTables<T>& tb, int nfields, const void* in,
                           T* out, double scale, hipStream_t s) {
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  switch (g.nx / 2) {
#define CASE(M)                                                                            \
  case M: {                                                                                \
    using C = RowCfg<T, M>;                                                                \
    dim3 grid((unsigned)((g.nrows + C::RB - 1) / C::RB), (unsigned)nfields);               \
    ACM_LAUNCH((k_rows_c2r<T, M>), grid, dim3(C::NT), C::LDS_BYTES, s,              \
                       reinterpret_cast<const cplx<T>*>(in), out, (int)g.nrows, g.ntot,     \
                       g.nspec, (T)scale, ct + tb.off.tw_x, ct + tb.off.rtw);               \
    return hipGetLastError();                                                              \
  }
    ACM_ROW_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
static hipError_t cols_impl(const Geom& g, const DevTables<T>& tb, int axis, int sign,
                            int nfields, const ColCellArgs& one, const ColCellArgs* many,
                            int ncells, hipStream_t s) {
  const cplx<T>* ct = reinterpret_cast<const cplx<T>*>(tb.ctab);
  ColMap m;
  int L;
  const cplx<T>* tw;
  if (axis == 1) {
    L = g.ny;
    m.inner = g.xh;
    m.outer = g.ny * g.xh;
    m.as = g.xh;
    m.ncols = g.nz * g.xh;
    tw = ct + tb.off.tw_y;
  } else if (axis == 2 && g.dim == 3) {
    L = g.nz;
    m.inner = g.ny * g.xh;
    m.outer = 0;
    m.as = g.ny * g.xh;
    m.ncols = g.ny * g.xh;
    tw = ct + tb.off.tw_z;
  } else {
    return hipErrorInvalidValue;
  }
  switch (L) {
#define CASE(LL)                                                                            \
  case LL: {                                                                                \
    using C = ColCfg<T, LL, 1, cols_var<LL>()>;                                             \
    dim3 grid((unsigned)((m.ncols + C::TX - 1) / C::TX), (unsigned)nfields,                 \
              (unsigned)ncells);                                                            \
    if constexpr (RegPlanOk<LL>::value()) {                                                 \
      constexpr int lds_reg = C::LDS_BYTES + Plan<LL>::tw_total * (int)sizeof(cplx<T>);     \
      if (sign < 0)                                                                         \
        ACM_LAUNCH((k_cols_reg<T, LL, -1>), grid, dim3(C::NT), lds_reg, s, one, many,       \
                   g.nspec, m, tw);                                                         \
      else                                                                                  \
        ACM_LAUNCH((k_cols_reg<T, LL, 1>), grid, dim3(C::NT), lds_reg, s, one, many,        \
                   g.nspec, m, tw);                                                         \
    } else {                                                                                \
      if (sign < 0)                                                                         \
        ACM_LAUNCH((k_cols<T, LL, -1>), grid, dim3(C::NT), C::LDS_BYTES, s, one, many,      \
                   g.nspec, m, tw);                                                         \
      else                                                                                  \
        ACM_LAUNCH((k_cols<T, LL, 1>), grid, dim3(C::NT), C::LDS_BYTES, s, one, many,       \
                   g.nspec, m, tw);                                                         \
    }                                                                                       \
    return hipGetLastError();                                                               \
  }
    ACM_COL_LENGTHS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_cols(const Geom& g, const DevTables<T>& tb, int axis, int sign, int nfields,
                       void* data, hipStream_t s, const int32_t* skip, const int32_t* skip2) {
  ColCellArgs one{data, skip, skip2};
  return cols_impl<T>(g, tb, axis, sign, nfields, one, nullptr, 1, s);
}

template <typename T>
hipError_t launch_cols_batched(const Geom& g, const DevTables<T>& tb, int axis, int sign,
                               int nfields, const ColCellArgs* cells, int ncells, hipStream_t s) {
  ColCellArgs one{nullptr, nullptr, nullptr};
  return cols_impl<T>(g, tb, axis, sign, nfields, one, cells, ncells, s);
}

#define INST(T)                                                                              \
  template hipError_t launch_rows_r2c<T>(const Geom&, const DevTables<T>&, int, const T*,    \
                                         void*, hipStream_t);                                \
  template hipError_t launch_rows_c2r<T>(const Geom&, const DevTables<T>&, int, const void*, \
                                         T*, double, hipStream_t);                           \
  template hipError_t launch_cols<T>(const Geom&, const DevTables<T>&, int, int, int, void*, \
                                     hipStream_t, const int32_t*, const int32_t*);           \
  template hipError_t launch_cols_batched<T>(const Geom&, const DevTables<T>&, int, int, int, \
                                             const ColCellArgs*, int, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace acm
