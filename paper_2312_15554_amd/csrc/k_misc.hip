// FP64 volume averages behind the effective properties (Section 2, eq. K and
// eq. D) and the pore-averaged velocity used by the transport problem.
// Each kernel writes per-block partial sums; the host adds the partials in a
// fixed order, so results are bitwise reproducible.
#include "pass_common.hpp"

namespace acm {

constexpr int kRedBlocks = 512;
constexpr int kRedThreads = 256;

// sums[0] = sum_pore 1, sums[1+c] = sum_pore u_c, sums[1+d+c] = sum_Y u_c
template <typename T, int D>
__global__ __launch_bounds__(kRedThreads) void k_flow_sums(const T* __restrict__ u,
                                                            const uint8_t* __restrict__ H,
                                                            int64_t ntot,
                                                            double* __restrict__ part) {
  __shared__ double red[(1 + 2 * D) * 4];
  double acc[1 + 2 * D];
#pragma unroll
  for (int k = 0; k < 1 + 2 * D; ++k) acc[k] = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; v < ntot;
       v += (int64_t)gridDim.x * kRedThreads) {
    const bool pore = H[v] == 0;
    if (pore) acc[0] += 1.0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const double x = (double)u[c * ntot + v];
      if (pore) acc[1 + c] += x;
      acc[1 + D + c] += x;
    }
  }
  block_sum<1 + 2 * D>(acc, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 1 + 2 * D; ++k) part[blockIdx.x * (1 + 2 * D) + k] = acc[k];
}

// For one chi (and the flow u it was computed with):
// sums[0] = sum_Y chi, sums[1] = sum_pore chi, sums[2+c] = sum_pore u_c chi,
// sums[2+D+c] = sum_pore (grad_c chi)_c  (central difference, periodic)
template <typename T, int D>
__global__ __launch_bounds__(kRedThreads) void k_chi_sums(const T* __restrict__ chi,
                                                           const T* __restrict__ u,
                                                           const uint8_t* __restrict__ H, int nx,
                                                           int ny, int nz,
                                                           double* __restrict__ part) {
  constexpr int NS = 2 + 2 * D;
  __shared__ double red[NS * 4];
  double acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0.0;
  const int64_t ntot = (int64_t)nx * ny * nz;
  for (int64_t v = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; v < ntot;
       v += (int64_t)gridDim.x * kRedThreads) {
    const double c0 = (double)chi[v];
    acc[0] += c0;
    if (H[v] != 0) continue;
    acc[1] += c0;
    const int x = (int)(v % nx);
    const int64_t yz = v / nx;
    const int y = (int)(yz % ny);
    const int z = (int)(yz / ny);
#pragma unroll
    for (int c = 0; c < D; ++c) acc[2 + c] += (double)u[c * ntot + v] * c0;
    {
      const int xp = x + 1 == nx ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
      const int64_t row = v - x;
      acc[2 + D + 0] += 0.5 * nx * ((double)chi[row + xp] - (double)chi[row + xm]);
    }
    {
      const int yp = y + 1 == ny ? 0 : y + 1, ym = y == 0 ? ny - 1 : y - 1;
      const int64_t b = ((int64_t)z * ny) * nx + x;
      acc[2 + D + 1] += 0.5 * ny * ((double)chi[b + (int64_t)yp * nx] - (double)chi[b + (int64_t)ym * nx]);
    }
    if constexpr (D == 3) {
      const int zp = z + 1 == nz ? 0 : z + 1, zm = z == 0 ? nz - 1 : z - 1;
      const int64_t b = (int64_t)y * nx + x;
      const int64_t pl = (int64_t)ny * nx;
      acc[2 + D + 2] += 0.5 * nz * ((double)chi[b + zp * pl] - (double)chi[b + zm * pl]);
    }
  }
  block_sum<NS>(acc, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < NS; ++k) part[blockIdx.x * NS + k] = acc[k];
}

template <typename T>
hipError_t launch_flow_sums(const Geom& g, const T* u, const uint8_t* H, double* part, int* nsums,
                            hipStream_t s) {
  const int nb = (int)std::min<int64_t>(kRedBlocks, (g.ntot + kRedThreads - 1) / kRedThreads);
  if (g.dim == 3) {
    hipLaunchKernelGGL((k_flow_sums<T, 3>), dim3(nb), dim3(kRedThreads), 0, s, u, H, g.ntot, part);
    *nsums = 7;
  } else {
    hipLaunchKernelGGL((k_flow_sums<T, 2>), dim3(nb), dim3(kRedThreads), 0, s, u, H, g.ntot, part);
    *nsums = 5;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_chi_sums(const Geom& g, const T* chi, const T* u, const uint8_t* H,
                           double* part, int* nsums, hipStream_t s) {
  const int nb = (int)std::min<int64_t>(kRedBlocks, (g.ntot + kRedThreads - 1) / kRedThreads);
  if (g.dim == 3) {
    hipLaunchKernelGGL((k_chi_sums<T, 3>), dim3(nb), dim3(kRedThreads), 0, s, chi, u, H, g.nx,
                       g.ny, g.nz, part);
    *nsums = 8;
  } else {
    hipLaunchKernelGGL((k_chi_sums<T, 2>), dim3(nb), dim3(kRedThreads), 0, s, chi, u, H, g.nx,
                       g.ny, g.nz, part);
    *nsums = 6;
  }
  return hipGetLastError();
}

int reduction_blocks(const Geom& g) {
  return (int)std::min<int64_t>(kRedBlocks, (g.ntot + kRedThreads - 1) / kRedThreads);
}

#define INST(T)                                                                              \
  template hipError_t launch_flow_sums<T>(const Geom&, const T*, const uint8_t*, double*,    \
                                          int*, hipStream_t);                                \
  template hipError_t launch_chi_sums<T>(const Geom&, const T*, const T*, const uint8_t*,    \
                                         double*, int*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace acm
