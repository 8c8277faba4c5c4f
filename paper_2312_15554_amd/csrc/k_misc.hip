// FP64 volume averages behind the effective properties (Section 2, eq. K and
// eq. D) and the pore-averaged velocity used by the transport problem.
// Each kernel writes per-block partial sums; the host adds the partials in a
// fixed order, so results are bitwise reproducible.
#include "pass_common.hpp"

namespace acm {

constexpr int kRedBlocks = kReductionBlocksMax;
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


// Warm-start state (initial guess u_in, q_in): with u0 = (1-H) u_in,
//   a0 = lambda0 = H (g - grad_c q0 + nu Delta_h u0)   (the reaction the
//   fixed point carries in the solid), div = central divergence of u0.
// Real-space stencils: central first differences, compact second differences.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_warm_init(const T* __restrict__ u, const T* __restrict__ q,
                                                   const uint8_t* __restrict__ H, T* __restrict__ a,
                                                   T* __restrict__ div, int nx, int ny, int nz,
                                                   double nu, double g0, double g1, double g2) {
  const int64_t ntot = (int64_t)nx * ny * nz;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= ntot) return;
  const int x = (int)(v % nx);
  const int64_t yz = v / nx;
  const int y = (int)(yz % ny);
  const int z = (int)(yz / ny);
  const int n[3] = {nx, ny, nz};
  int64_t nb_p[3], nb_m[3];
  {
    const int xp = x + 1 == nx ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
    nb_p[0] = v - x + xp;
    nb_m[0] = v - x + xm;
    const int yp = y + 1 == ny ? 0 : y + 1, ym = y == 0 ? ny - 1 : y - 1;
    nb_p[1] = v + (int64_t)(yp - y) * nx;
    nb_m[1] = v + (int64_t)(ym - y) * nx;
    if (D == 3) {
      const int zp = z + 1 == nz ? 0 : z + 1, zm = z == 0 ? nz - 1 : z - 1;
      nb_p[2] = v + (int64_t)(zp - z) * nx * ny;
      nb_m[2] = v + (int64_t)(zm - z) * nx * ny;
    }
  }
  auto u0 = [&](int c, int64_t w) -> double { return H[w] ? 0.0 : (double)u[c * ntot + w]; };
  const double g[3] = {g0, g1, g2};
  double dv = 0.0;
  const bool solid = H[v] != 0;
  for (int c = 0; c < D; ++c) {
    dv += 0.5 * n[c] * (u0(c, nb_p[c]) - u0(c, nb_m[c]));
    double lap = 0.0;
    const double uc = u0(c, v);
    for (int j = 0; j < D; ++j)
      lap += (u0(c, nb_p[j]) - 2.0 * uc + u0(c, nb_m[j])) * (double)n[j] * n[j];
    const double gq = q ? 0.5 * n[c] * ((double)q[nb_p[c]] - (double)q[nb_m[c]]) : 0.0;
    a[c * ntot + v] = solid ? (T)(g[c] - gq + nu * lap) : T(0);
  }
  div[v] = (T)dv;
}

template <typename T>
__global__ __launch_bounds__(256) void k_mask_pore(T* __restrict__ u, const uint8_t* __restrict__ H,
                                                   int d, int64_t ntot) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= ntot || !H[v]) return;
  for (int c = 0; c < d; ++c) u[c * ntot + v] = T(0);
}

template <typename T>
hipError_t launch_warm_init(const Geom& g, const T* u, const T* q, const uint8_t* H, T* a, T* div,
                            double nu, const double* gp, hipStream_t s) {
  const unsigned nb = (unsigned)((g.ntot + 255) / 256);
  if (g.dim == 3)
    hipLaunchKernelGGL((k_warm_init<T, 3>), dim3(nb), dim3(256), 0, s, u, q, H, a, div, g.nx, g.ny,
                       g.nz, nu, gp[0], gp[1], gp[2]);
  else
    hipLaunchKernelGGL((k_warm_init<T, 2>), dim3(nb), dim3(256), 0, s, u, q, H, a, div, g.nx, g.ny,
                       g.nz, nu, gp[0], gp[1], 0.0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_mask_pore<T>), dim3(nb), dim3(256), 0, s, const_cast<T*>(u), H, g.dim, g.ntot);
  return hipGetLastError();
}

// Totals of nb per-block records of ns partial sums: record b is added to the
// running sum in block order, starting from 0.0 -- the additions the host makes
// when it adds the copied partials, in the same order, so the totals are the
// same bits either way.
__global__ __launch_bounds__(64) void k_sum_partials(const double* __restrict__ part, int nb,
                                                     int ns, double* __restrict__ out) {
  const int k = threadIdx.x;
  if (k >= ns) return;
  double acc = 0.0;
  for (int b = 0; b < nb; ++b) acc += part[(int64_t)b * ns + k];
  out[k] = acc;
}

hipError_t launch_sum_partials(const double* part, int nb, int ns, double* out, hipStream_t s) {
  if (ns < 1 || ns > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, part, nb, ns, out);
  return hipGetLastError();
}

int reduction_blocks(const Geom& g) {
  return (int)std::min<int64_t>(kRedBlocks, (g.ntot + kRedThreads - 1) / kRedThreads);
}

__global__ void k_noop(int) {}

hipError_t launch_noop(hipStream_t s) {
  ACM_LAUNCH(k_noop, dim3(1), dim3(64), 0, s, 0);
  return hipGetLastError();
}

#define INST(T)                                                                              \
  template hipError_t launch_flow_sums<T>(const Geom&, const T*, const uint8_t*, double*,    \
                                          int*, hipStream_t);                                \
  template hipError_t launch_chi_sums<T>(const Geom&, const T*, const T*, const uint8_t*,    \
                                         double*, int*, hipStream_t);                        \
  template hipError_t launch_warm_init<T>(const Geom&, const T*, const T*, const uint8_t*,   \
                                          T*, T*, double, const double*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace acm
