// Fourier-neural-operator warm start: forward, backward and Adam kernels.
//
// The network maps the solid indicator H of a cell to an initial guess
// (u_x, u_y, u_z, p) for the Stokes ADMM (Li et al., ICLR 2021, Fourier
// neural operator):
//   v0 = Pw H + Pb;  v_{l+1} = act_l(W_l v_l + b_l + K_l v_l);
//   K_l v = inverse real FFT of (R_l . forward real FFT of v) on the kept modes
//   (kx < m, ky and kz in [0, m) U [N-m, N));  act = GELU (tanh form) except
//   after the last layer;  out = Q2 GELU(Q1 v_L + c1) + c2.
// Weights are BF16 (rounded from FP32 master copies by the Adam kernel);
// activations, transforms and every accumulation are FP32, weight-gradient
// reductions are deterministic (per-block partials, then an ordered sum).
#include "pass_common.hpp"

namespace acm {

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint32_t r = ((u >> 16) & 1u) + 0x7fffu;  // round to nearest even
  return (uint16_t)((u + r) >> 16);
}
__device__ __forceinline__ float gelu_f(float x) {
  const float k = 0.7978845608028654f;
  return 0.5f * x * (1.f + tanhf(k * (x + 0.044715f * x * x * x)));
}
__device__ __forceinline__ float gelu_grad_f(float x) {
  const float k = 0.7978845608028654f;
  const float t = tanhf(k * (x + 0.044715f * x * x * x));
  return 0.5f * (1.f + t) + 0.5f * x * (1.f - t * t) * k * (1.f + 3.f * 0.044715f * x * x);
}

// ------------------------------------------------------------------- lift
__global__ __launch_bounds__(256) void k_fno_lift(const uint8_t* __restrict__ H,
                                                  const uint16_t* __restrict__ Pw,
                                                  const uint16_t* __restrict__ Pb,
                                                  float* __restrict__ v, int C, int64_t nvox,
                                                  int B) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (x >= nvox) return;
  const float h = H[(int64_t)b * nvox + x] ? 1.f : 0.f;
  for (int c = 0; c < C; ++c) v[((int64_t)b * C + c) * nvox + x] = bf2f(Pw[c]) * h + bf2f(Pb[c]);
}

// ----------------------------------------------------------- kept modes
// Gather the kept modes of every (b, c) half spectrum into a compact array
// [B*C][nm] and (optionally) clear the full spectrum afterwards is done by the
// host with a memset.
__global__ __launch_bounds__(256) void k_fno_gather(const float2* __restrict__ spec,
                                                    float2* __restrict__ out,
                                                    const int* __restrict__ midx, int nm,
                                                    int64_t nspec, int nfields) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (j >= nm || f >= nfields) return;
  out[(int64_t)f * nm + j] = spec[(int64_t)f * nspec + midx[j]];
}

// Y[b][o][m] = sum_i R[m][o][i] X[b][i][m] (conj(R) and sum over o when
// ADJ: Z[b][i][m] = sum_o conj(R[m][o][i]) X[b][o][m]); scattered into the
// (cleared) full spectrum at the kept-mode offsets.  A workgroup takes JT =
// 256 / C consecutive modes: their weights (C x C complex BF16 pairs per mode,
// contiguous) are staged in LDS with coalesced loads and a padded row, so that
// thread (c, jj) reads row c of R[m] (or column c for the adjoint) without
// bank conflicts and keeps it in registers while it runs through the batch;
// the activations of a chunk of batch members are staged beside them.
template <bool ADJ, int C>
__global__ __launch_bounds__(256) void k_fno_mix(const float2* __restrict__ Xm,
                                                 const uint16_t* __restrict__ R,
                                                 float2* __restrict__ spec,
                                                 const int* __restrict__ midx, int nm, int B,
                                                 int64_t nspec) {
  constexpr int JT = 256 / C, RS = C + 1, BT = 8;
  __shared__ uint32_t sR[JT * C * RS];
  __shared__ float2 sX[BT * C * JT];
  const int j0 = blockIdx.x * JT;
  const int nj = min(JT, nm - j0);
  const uint32_t* gR = reinterpret_cast<const uint32_t*>(R) + (int64_t)j0 * C * C;
  batched_copy<uint32_t, 256, JT * C * C>(
      nj * C * C, [&](int e) { return gR[e]; },
      [&](int e, const uint32_t& w) { sR[(e / C) * RS + e % C] = w; });
  const int c = threadIdx.x / JT, jj = threadIdx.x % JT;
  const bool live = jj < nj;
  const int64_t sidx = live ? midx[j0 + jj] : 0;
  __syncthreads();
  float rr[C], ri[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    // real part in the low half of the pair, imaginary in the high half
    const uint32_t w = ADJ ? sR[(jj * C + k) * RS + c] : sR[(jj * C + c) * RS + k];
    rr[k] = __uint_as_float(w << 16);
    ri[k] = __uint_as_float(w & 0xffff0000u);
  }
  for (int b0 = 0; b0 < B; b0 += BT) {
    const int nb = min(BT, B - b0);
    __syncthreads();
    // e = ((batch member in chunk) * C + channel) * JT + mode in tile
    batched_copy<float2, 256, BT * C * JT>(
        nb * C * JT,
        [&](int e) {
          const int jx = e % JT, bi = e / JT;
          float2 v = make_float2(0.f, 0.f);
          if (jx < nj) v = Xm[((int64_t)b0 * C + bi) * nm + j0 + jx];
          return v;
        },
        [&](int e, const float2& v) { sX[e] = v; });
    __syncthreads();
    if (!live) continue;
    for (int bb = 0; bb < nb; ++bb) {
      float ar = 0.f, ai = 0.f;
#pragma unroll
      for (int k = 0; k < C; ++k) {
        const float2 x = sX[(bb * C + k) * JT + jj];
        if (!ADJ) {
          ar += rr[k] * x.x - ri[k] * x.y;
          ai += rr[k] * x.y + ri[k] * x.x;
        } else {
          ar += rr[k] * x.x + ri[k] * x.y;
          ai += rr[k] * x.y - ri[k] * x.x;
        }
      }
      spec[((int64_t)(b0 + bb) * C + c) * nspec + sidx] = make_float2(ar, ai);
    }
  }
}

// dR[m][o][i] = sum_b (w_m / N) F[b][o][m] conj(X[b][i][m])  (float pairs).
// A workgroup takes JT = 256 / C consecutive modes, stages F and X of a chunk
// of batch members in LDS (coalesced along the modes; the row padded by one so
// that the threads of one mode read different banks) and writes the modes'
// C x C gradients as one contiguous run.
template <int C>
__global__ __launch_bounds__(256) void k_fno_dR(const float2* __restrict__ Fm,
                                                const float2* __restrict__ Xm,
                                                const float* __restrict__ mw,
                                                float* __restrict__ dR, int nm, int B,
                                                float inv_n) {
  constexpr int JT = 256 / C, JS = JT + 1, BT = 8, PER = JT * C * C / 256;
  __shared__ float2 sF[BT * C * JS], sX[BT * C * JS];
  __shared__ float smw[JT];
  const int j0 = blockIdx.x * JT;
  const int nj = min(JT, nm - j0);
  if (threadIdx.x < JT) smw[threadIdx.x] = threadIdx.x < nj ? mw[j0 + threadIdx.x] * inv_n : 0.f;
  float ar[PER], ai[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) ar[k] = ai[k] = 0.f;
  for (int b0 = 0; b0 < B; b0 += BT) {
    const int nb = min(BT, B - b0);
    __syncthreads();
    for (int e = threadIdx.x; e < nb * C * JT; e += 256) {
      const int jx = e % JT, bi = e / JT;  // bi = (batch member in chunk) * C + channel
      const int64_t g = ((int64_t)b0 * C + bi) * nm + j0 + jx;
      float2 fv = make_float2(0.f, 0.f), xv = fv;
      if (jx < nj) {
        fv = Fm[g];
        xv = Xm[g];
      }
      sF[bi * JS + jx] = fv;
      sX[bi * JS + jx] = xv;
    }
    __syncthreads();
    for (int bb = 0; bb < nb; ++bb) {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256;
        const int jj = e / (C * C), o = (e / C) % C, i = e % C;
        const float2 f = sF[(bb * C + o) * JS + jj];
        const float2 x = sX[(bb * C + i) * JS + jj];
        ar[k] += f.x * x.x + f.y * x.y;
        ai[k] += f.y * x.x - f.x * x.y;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + k * 256;
    const int jj = e / (C * C);
    if (jj < nj) {
      const float sc = smw[jj];
      const int64_t t = (int64_t)j0 * C * C + e;
      dR[2 * t] = ar[k] * sc;
      dR[2 * t + 1] = ai[k] * sc;
    }
  }
}

// --------------------------------------------------------- pointwise layer
// pre = W v + b + k;  vout = act(pre).  One thread per voxel; C <= 64.
template <int C>
__global__ __launch_bounds__(256) void k_fno_pointwise(const float* __restrict__ vin,
                                                       const float* __restrict__ k,
                                                       const uint16_t* __restrict__ W,
                                                       const uint16_t* __restrict__ bias,
                                                       float* __restrict__ pre,
                                                       float* __restrict__ vout, int64_t nvox,
                                                       int act) {
  __shared__ float sW[C * C];
  __shared__ float sb[C];
  for (int e = threadIdx.x; e < C * C; e += blockDim.x) sW[e] = bf2f(W[e]);
  for (int e = threadIdx.x; e < C; e += blockDim.x) sb[e] = bf2f(bias[e]);
  __syncthreads();
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (x >= nvox) return;
  const int64_t base = (int64_t)b * C * nvox + x;
  float v[C];
#pragma unroll
  for (int i = 0; i < C; ++i) v[i] = vin[base + i * nvox];
  for (int o = 0; o < C; ++o) {
    float acc = sb[o] + k[base + o * nvox];
#pragma unroll
    for (int i = 0; i < C; ++i) acc += sW[o * C + i] * v[i];
    if (pre) pre[base + o * nvox] = acc;
    vout[base + o * nvox] = act ? gelu_f(acc) : acc;
  }
}

// dpre = dv * act'(pre);  dvdir = W^T dpre.
template <int C>
__global__ __launch_bounds__(256) void k_fno_pointwise_bwd(const float* __restrict__ dv,
                                                           const float* __restrict__ pre,
                                                           const uint16_t* __restrict__ W,
                                                           float* __restrict__ dpre,
                                                           float* __restrict__ dvdir,
                                                           int64_t nvox, int act) {
  __shared__ float sW[C * C];
  for (int e = threadIdx.x; e < C * C; e += blockDim.x) sW[e] = bf2f(W[e]);
  __syncthreads();
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (x >= nvox) return;
  const int64_t base = (int64_t)b * C * nvox + x;
  float dp[C];
#pragma unroll
  for (int o = 0; o < C; ++o) {
    const float g = dv[base + o * nvox];
    dp[o] = act ? g * gelu_grad_f(pre[base + o * nvox]) : g;
    dpre[base + o * nvox] = dp[o];
  }
  for (int i = 0; i < C; ++i) {
    float acc = 0.f;
#pragma unroll
    for (int o = 0; o < C; ++o) acc += sW[o * C + i] * dp[o];
    dvdir[base + i * nvox] = acc;
  }
}

// ------------------------------------------- pointwise layer on matrix cores
// The 32-channel mix is a dense contraction, pre[o][x] = sum_i W[o][i] v[i][x]
// over 32 voxels per wave: v_mfma_f32_32x32x2_f32 takes W (32 x 2, lane l
// holding W[l % 32][2 s + l / 32] at step s) and v (2 x 32, lane l holding
// v[2 s + l / 32][x0 + l % 32]) and accumulates the 32 x 32 tile over 16
// steps in FP32, with the same operands (BF16-rounded weights, FP32
// activations) as the vector kernel.  Lane l then holds rows
// 8 (r / 4) + 4 (l / 32) + r % 4 of column l % 32 in its register r.
typedef float mfma_f32x16 __attribute__((ext_vector_type(16)));
constexpr int kMixTiles = 4;  // 32-voxel tiles per wave (the weights are loaded once)

__device__ __forceinline__ int mix_row(int r, int half) { return 8 * (r / 4) + 4 * half + (r % 4); }

__global__ __launch_bounds__(256) void k_fno_pointwise_mfma(const float* __restrict__ vin,
                                                            const float* __restrict__ k,
                                                            const uint16_t* __restrict__ W,
                                                            const uint16_t* __restrict__ bias,
                                                            float* __restrict__ pre,
                                                            float* __restrict__ vout, int64_t nvox,
                                                            int act) {
  constexpr int C = 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, half = lane >> 5;
  const int b = blockIdx.y;
  float wa[16], br[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) wa[s] = bf2f(W[col * C + 2 * s + half]);
#pragma unroll
  for (int r = 0; r < 16; ++r) br[r] = bf2f(bias[mix_row(r, half)]);
  const int64_t base = (int64_t)b * C * nvox;
  for (int tt = 0; tt < kMixTiles; ++tt) {
    const int64_t x0 = (((int64_t)blockIdx.x * 4 + wave) * kMixTiles + tt) * 32;
    if (x0 >= nvox) break;  // the same for the whole wave
    const int64_t x = x0 + col;
    const bool in = x < nvox;
    float bv[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) bv[s] = in ? vin[base + (int64_t)(2 * s + half) * nvox + x] : 0.f;
    mfma_f32x16 acc = {};
#pragma unroll
    for (int s = 0; s < 16; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wa[s], bv[s], acc, 0, 0, 0);
    if (in) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t off = base + (int64_t)mix_row(r, half) * nvox + x;
        const float v = acc[r] + br[r] + k[off];
        if (pre) pre[off] = v;
        vout[off] = act ? gelu_f(v) : v;
      }
    }
  }
}

// dpre = dv * act'(pre);  dvdir = W^T dpre, the contraction on matrix cores
// as above with W^T (lane l holding W[2 s + l / 32][l % 32] at step s) and
// dpre (formed in the lane that feeds it to the step).
__global__ __launch_bounds__(256) void k_fno_pointwise_bwd_mfma(const float* __restrict__ dv,
                                                                const float* __restrict__ pre,
                                                                const uint16_t* __restrict__ W,
                                                                float* __restrict__ dpre,
                                                                float* __restrict__ dvdir,
                                                                int64_t nvox, int act) {
  constexpr int C = 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, half = lane >> 5;
  const int b = blockIdx.y;
  float wa[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) wa[s] = bf2f(W[(2 * s + half) * C + col]);
  const int64_t base = (int64_t)b * C * nvox;
  for (int tt = 0; tt < kMixTiles; ++tt) {
    const int64_t x0 = (((int64_t)blockIdx.x * 4 + wave) * kMixTiles + tt) * 32;
    if (x0 >= nvox) break;
    const int64_t x = x0 + col;
    const bool in = x < nvox;
    float dp[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int64_t off = base + (int64_t)(2 * s + half) * nvox + x;
      float g = 0.f;
      if (in) {
        g = dv[off];
        if (act) g *= gelu_grad_f(pre[off]);
        dpre[off] = g;
      }
      dp[s] = g;
    }
    mfma_f32x16 acc = {};
#pragma unroll
    for (int s = 0; s < 16; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(wa[s], dp[s], acc, 0, 0, 0);
    if (in) {
#pragma unroll
      for (int r = 0; r < 16; ++r) dvdir[base + (int64_t)mix_row(r, half) * nvox + x] = acc[r];
    }
  }
}

// dv += other
__global__ __launch_bounds__(256) void k_fno_add(float* __restrict__ a, const float* __restrict__ b,
                                                 int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] += b[i];
}

// --------------------------------------------------------------- projection
// out[o] = sum_j Q2[o][j] GELU(sum_i Q1[j][i] v[i] + c1[j]) + c2[o]; optionally
// store h (Cp channels) for the backward pass.
template <int C>
__global__ __launch_bounds__(256) void k_fno_project(const float* __restrict__ v,
                                                     const uint16_t* __restrict__ Q1,
                                                     const uint16_t* __restrict__ c1,
                                                     const uint16_t* __restrict__ Q2,
                                                     const uint16_t* __restrict__ c2,
                                                     float* __restrict__ out, int Cp,
                                                     int64_t nvox) {
  extern __shared__ float sh[];
  float* sQ1 = sh;               // Cp*C
  float* sc1 = sQ1 + Cp * C;     // Cp
  float* sQ2 = sc1 + Cp;         // 4*Cp
  for (int e = threadIdx.x; e < Cp * C; e += blockDim.x) sQ1[e] = bf2f(Q1[e]);
  for (int e = threadIdx.x; e < Cp; e += blockDim.x) sc1[e] = bf2f(c1[e]);
  for (int e = threadIdx.x; e < 4 * Cp; e += blockDim.x) sQ2[e] = bf2f(Q2[e]);
  __syncthreads();
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (x >= nvox) return;
  float vv[C];
#pragma unroll
  for (int i = 0; i < C; ++i) vv[i] = v[((int64_t)b * C + i) * nvox + x];
  float o4[4] = {bf2f(c2[0]), bf2f(c2[1]), bf2f(c2[2]), bf2f(c2[3])};
  for (int j = 0; j < Cp; ++j) {
    float hp = sc1[j];
#pragma unroll
    for (int i = 0; i < C; ++i) hp += sQ1[j * C + i] * vv[i];
    const float h = gelu_f(hp);
#pragma unroll
    for (int o = 0; o < 4; ++o) o4[o] += sQ2[o * Cp + j] * h;
  }
#pragma unroll
  for (int o = 0; o < 4; ++o) out[((int64_t)b * 4 + o) * nvox + x] = o4[o];
}

// Backward of the projection: writes h and dh (Cp channels each, for the
// weight gradients) and dv = Q1^T dh.
template <int C>
__global__ __launch_bounds__(256) void k_fno_project_bwd(const float* __restrict__ v,
                                                         const float* __restrict__ dout,
                                                         const uint16_t* __restrict__ Q1,
                                                         const uint16_t* __restrict__ c1,
                                                         const uint16_t* __restrict__ Q2,
                                                         float* __restrict__ h_out,
                                                         float* __restrict__ dh_out,
                                                         float* __restrict__ dv, int Cp,
                                                         int64_t nvox) {
  extern __shared__ float sh[];
  float* sQ1 = sh;
  float* sc1 = sQ1 + Cp * C;
  float* sQ2 = sc1 + Cp;
  for (int e = threadIdx.x; e < Cp * C; e += blockDim.x) sQ1[e] = bf2f(Q1[e]);
  for (int e = threadIdx.x; e < Cp; e += blockDim.x) sc1[e] = bf2f(c1[e]);
  for (int e = threadIdx.x; e < 4 * Cp; e += blockDim.x) sQ2[e] = bf2f(Q2[e]);
  __syncthreads();
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (x >= nvox) return;
  float vv[C], dvv[C];
#pragma unroll
  for (int i = 0; i < C; ++i) {
    vv[i] = v[((int64_t)b * C + i) * nvox + x];
    dvv[i] = 0.f;
  }
  float d4[4];
#pragma unroll
  for (int o = 0; o < 4; ++o) d4[o] = dout[((int64_t)b * 4 + o) * nvox + x];
  for (int j = 0; j < Cp; ++j) {
    float hp = sc1[j];
#pragma unroll
    for (int i = 0; i < C; ++i) hp += sQ1[j * C + i] * vv[i];
    float g = 0.f;
#pragma unroll
    for (int o = 0; o < 4; ++o) g += sQ2[o * Cp + j] * d4[o];
    const float dh = g * gelu_grad_f(hp);
    h_out[((int64_t)b * Cp + j) * nvox + x] = gelu_f(hp);
    dh_out[((int64_t)b * Cp + j) * nvox + x] = dh;
#pragma unroll
    for (int i = 0; i < C; ++i) dvv[i] += sQ1[j * C + i] * dh;
  }
#pragma unroll
  for (int i = 0; i < C; ++i) dv[((int64_t)b * C + i) * nvox + x] = dvv[i];
}

// ----------------------------------------------------- outer-product sums
// part[blk][p*Q + q] = sum over this block's voxels (all b) of A[b][p][x] * Bm[b][q][x]
// (Bm == null: Bm = 1, giving sums of A; Bm_u8: a uint8 field as 0/1).
constexpr int kOuterTile = 64;
__global__ __launch_bounds__(256) void k_fno_outer(const float* __restrict__ A,
                                                   const float* __restrict__ Bm,
                                                   const uint8_t* __restrict__ Bu8, int P, int Q,
                                                   int64_t nvox, int B, int64_t chunk,
                                                   float* __restrict__ part) {
  extern __shared__ float sm[];
  float* sA = sm;                       // P * kOuterTile
  float* sB = sA + P * kOuterTile;      // Q * kOuterTile
  const int PQ = P * Q;
  constexpr int MAXE = 16;  // entries per thread: P*Q <= 16*256
  float acc[MAXE];
#pragma unroll
  for (int e = 0; e < MAXE; ++e) acc[e] = 0.f;
  const int64_t total = nvox * B;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < total ? beg + chunk : total;
  for (int64_t t0 = beg; t0 < end; t0 += kOuterTile) {
    __syncthreads();
    for (int e = threadIdx.x; e < (P + Q) * kOuterTile; e += blockDim.x) {
      const int r = e / kOuterTile, c = e - r * kOuterTile;
      const int64_t t = t0 + c;
      float val = 0.f;
      if (t < end) {
        const int64_t b = t / nvox, x = t - b * nvox;
        if (r < P) {
          val = A[(b * P + r) * nvox + x];
        } else {
          const int q = r - P;
          val = Bm ? Bm[(b * Q + q) * nvox + x] : (Bu8 ? (Bu8[b * nvox + x] ? 1.f : 0.f) : 1.f);
        }
      }
      sm[e] = val;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < MAXE; ++k) {
      const int e = threadIdx.x + k * 256;
      if (e < PQ) {
        const int p = e / Q, q = e - p * Q;
        float s = 0.f;
        for (int c = 0; c < kOuterTile; ++c) s += sA[p * kOuterTile + c] * sB[q * kOuterTile + c];
        acc[k] += s;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < MAXE; ++k) {
    const int e = threadIdx.x + k * 256;
    if (e < PQ) part[(int64_t)blockIdx.x * PQ + e] = acc[k];
  }
}

// The same sums on the matrix cores.  G = A B^T over the B nvox voxels of the
// batch is a dense contraction of two short matrices: a workgroup owns a group
// of GP x GQ output blocks of 32 x 32 and walks 64-voxel tiles of the batch
// (grid-stride, one batch member per tile since nvox is a multiple of 64).
// Each tile's 32 (GP + GQ) rows of A and B are staged in LDS with coalesced
// loads while the next tile's loads are in flight, and v_mfma_f32_32x32x2_f32
// contracts them: with four blocks in the group each wave owns one block and
// the whole tile; with fewer, the waves of a block split the tile's voxels and
// their partial blocks are added in a fixed order at the end.  Since the
// voxel index is only summed over, lane l takes voxel base + (l / 32) HALF + j
// of row l % 32 at step j, so that it reads its operands as float4 runs.
// Rows beyond P or Q are zero; BM selects B: 0 the matrix Bm, 1 the
// indicator of the uint8 field Bu8 in every row, 2 ones.
template <int GP, int GQ, int BM>
__global__ __launch_bounds__(256) void k_fno_outer_mfma(const float* __restrict__ A,
                                                        const float* __restrict__ Bm,
                                                        const uint8_t* __restrict__ Bu8, int P,
                                                        int Q, int64_t nvox, int64_t ntiles,
                                                        float* __restrict__ part) {
  constexpr int TK = kOuterTile, LS = TK + 4, TQ = TK / 4;
  constexpr int R = 32 * (GP + GQ);
  constexpr int NL = R * TQ / 256;  // float4 loads per thread and tile
  constexpr int NBG = GP * GQ, KP = 4 / NBG, HALF = TK / KP / 2;
  static_assert(R * TQ % 256 == 0 && 4 % NBG == 0, "outer tile shape");
  extern __shared__ __align__(16) float sm[];
  const int qgroups = (Q + 32 * GQ - 1) / (32 * GQ);
  const int p0 = (int)(blockIdx.y / qgroups) * GP * 32, q0 = (int)(blockIdx.y % qgroups) * GQ * 32;
  const gmem<const float>* gA = as_global(A);
  const gmem<const float>* gB = as_global(Bm);
  const gmem<const uint8_t>* gU = as_global(Bu8);

  float4 buf[NL];
  auto load = [&](int64_t tile) {
    const int64_t t0 = tile * TK;
    const int64_t b = t0 / nvox, x0 = t0 - b * nvox;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int e = threadIdx.x + j * 256;
      const int row = e / TQ, c = 4 * (e % TQ);
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (row < 32 * GP) {
        const int p = p0 + row;
        if (p < P) v = *(const gmem<const float4>*)(gA + (b * P + p) * nvox + x0 + c);
      } else {
        const int q = q0 + row - 32 * GP;
        if (q < Q) {
          if constexpr (BM == 0) {
            v = *(const gmem<const float4>*)(gB + (b * Q + q) * nvox + x0 + c);
          } else if constexpr (BM == 1) {
            const uchar4 m = *(const gmem<const uchar4>*)(gU + b * nvox + x0 + c);
            v = make_float4(m.x ? 1.f : 0.f, m.y ? 1.f : 0.f, m.z ? 1.f : 0.f, m.w ? 1.f : 0.f);
          } else {
            v = make_float4(1.f, 1.f, 1.f, 1.f);
          }
        }
      }
      buf[j] = v;
    }
  };

  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 31, h = l >> 5;
  const int bb = w % NBG, kp = w / NBG, bp = bb / GQ, bq = bb % GQ;
  const float* pa = sm + (bp * 32 + r) * LS + kp * 2 * HALF + h * HALF;
  const float* pb = sm + (32 * GP + bq * 32 + r) * LS + kp * 2 * HALF + h * HALF;
  mfma_f32x16 acc = {};
  int64_t tile = blockIdx.x;
  if (tile < ntiles) load(tile);
  for (; tile < ntiles; tile += gridDim.x) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int e = threadIdx.x + j * 256;
      *reinterpret_cast<float4*>(sm + (e / TQ) * LS + 4 * (e % TQ)) = buf[j];
    }
    __syncthreads();
    if (tile + gridDim.x < ntiles) load(tile + gridDim.x);
#pragma unroll
    for (int j = 0; j < HALF; j += 4) {
      const float4 a = *reinterpret_cast<const float4*>(pa + j);
      const float4 c = *reinterpret_cast<const float4*>(pb + j);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, c.x, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, c.y, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, c.z, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, c.w, acc, 0, 0, 0);
    }
  }
  __syncthreads();
  float* red = sm;  // 4 waves x 16 registers x 64 lanes
#pragma unroll
  for (int i = 0; i < 16; ++i) red[(w * 16 + i) * 64 + l] = acc[i];
  __syncthreads();
  if (w >= NBG) return;
  const int q = q0 + bq * 32 + r;
  float* dst = part + (int64_t)blockIdx.x * P * Q;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    float v = red[(w * 16 + i) * 64 + l];
#pragma unroll
    for (int k = 1; k < KP; ++k) v += red[((w + k * NBG) * 16 + i) * 64 + l];
    const int p = p0 + bp * 32 + mix_row(i, h);
    if (p < P && q < Q) dst[p * Q + q] = v;
  }
}

// out[e] = sum over blocks of part[blk][e], in double: each of the 16 waves
// of a workgroup sums a contiguous slice of the blocks for 64 entries, and the
// slices are added in order, so the result does not depend on timing.
constexpr int kSumWaves = 16;
__global__ __launch_bounds__(64 * kSumWaves) void k_fno_sum_parts(const float* __restrict__ part,
                                                                  int nblk, int n,
                                                                  float* __restrict__ out) {
  __shared__ double red[kSumWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  const int k0 = (int)((int64_t)nblk * w / kSumWaves);
  const int k1 = (int)((int64_t)nblk * (w + 1) / kSumWaves);
  double acc = 0.0;
  if (e < n) {
#pragma unroll 8
    for (int k = k0; k < k1; ++k) acc += part[(int64_t)k * n + e];
  }
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0 && e < n) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < kSumWaves; ++j) t += red[j][lane];
    out[e] = (float)t;
  }
}

// ------------------------------------------------------------------- Adam
__global__ __launch_bounds__(256) void k_fno_adam(float* __restrict__ p, uint16_t* __restrict__ pb,
                                                  const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v,
                                                  int64_t n, float lr, float b1, float b2,
                                                  float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  pb[i] = f2bf(pi);
}

__global__ __launch_bounds__(256) void k_fno_to_bf16(const float* __restrict__ p,
                                                     uint16_t* __restrict__ pb, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pb[i] = f2bf(p[i]);
}

// loss = sum (out - target)^2 / count ;  dout = 2 (out - target) / count
__global__ __launch_bounds__(256) void k_fno_mse(const float* __restrict__ out,
                                                 const float* __restrict__ tgt,
                                                 float* __restrict__ dout, int64_t n,
                                                 double inv_count, double* __restrict__ part) {
  __shared__ double red[4];
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)out[i] - (double)tgt[i];
    acc[0] += d * d;
    dout[i] = (float)(2.0 * d * inv_count);
  }
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc[0] * inv_count;
}

// ------------------------------------------------------------- host glue
struct FnoLaunch {
  hipStream_t s;
};

hipError_t fno_lift(const uint8_t* H, const uint16_t* Pw, const uint16_t* Pb, float* v, int C,
                    int64_t nvox, int B, hipStream_t s) {
  dim3 grid((unsigned)((nvox + 255) / 256), (unsigned)B);
  hipLaunchKernelGGL(k_fno_lift, grid, dim3(256), 0, s, H, Pw, Pb, v, C, nvox, B);
  return hipGetLastError();
}

hipError_t fno_gather(const void* spec, void* out, const int* midx, int nm, int64_t nspec,
                      int nfields, hipStream_t s) {
  dim3 grid((unsigned)((nm + 255) / 256), (unsigned)nfields);
  hipLaunchKernelGGL(k_fno_gather, grid, dim3(256), 0, s, (const float2*)spec, (float2*)out, midx,
                     nm, nspec, nfields);
  return hipGetLastError();
}

#define FNO_CHANNELS(X) X(4) X(8) X(16) X(32)

hipError_t fno_mix(const void* Xm, const uint16_t* R, void* spec, const int* midx, int nm, int C,
                   int B, int64_t nspec, bool adjoint, hipStream_t s) {
  switch (C) {
#define CASE(CC)                                                                              \
  case CC: {                                                                                  \
    const dim3 grid((unsigned)((nm + 256 / CC - 1) / (256 / CC)));                            \
    if (adjoint)                                                                              \
      hipLaunchKernelGGL((k_fno_mix<true, CC>), grid, dim3(256), 0, s, (const float2*)Xm, R,  \
                         (float2*)spec, midx, nm, B, nspec);                                  \
    else                                                                                      \
      hipLaunchKernelGGL((k_fno_mix<false, CC>), grid, dim3(256), 0, s, (const float2*)Xm, R, \
                         (float2*)spec, midx, nm, B, nspec);                                  \
    return hipGetLastError();                                                                 \
  }
    FNO_CHANNELS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t fno_dR(const void* Fm, const void* Xm, const float* mw, float* dR, int nm, int C,
                  int B, float inv_n, hipStream_t s) {
  switch (C) {
#define CASE(CC)                                                                             \
  case CC:                                                                                   \
    hipLaunchKernelGGL((k_fno_dR<CC>), dim3((unsigned)((nm + 256 / CC - 1) / (256 / CC))),   \
                       dim3(256), 0, s, (const float2*)Fm, (const float2*)Xm, mw, dR,         \
                       nm, B, inv_n);                                                        \
    return hipGetLastError();
    FNO_CHANNELS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}


hipError_t fno_pointwise(int C, const float* vin, const float* k, const uint16_t* W,
                         const uint16_t* b, float* pre, float* vout, int64_t nvox, int B,
                         int act, hipStream_t s) {
  if (C == 32) {  // matrix cores: 4 waves x kMixTiles tiles of 32 voxels per workgroup
    const int64_t per = 4 * kMixTiles * 32;
    hipLaunchKernelGGL(k_fno_pointwise_mfma, dim3((unsigned)((nvox + per - 1) / per), (unsigned)B),
                       dim3(256), 0, s, vin, k, W, b, pre, vout, nvox, act);
    return hipGetLastError();
  }
  dim3 grid((unsigned)((nvox + 255) / 256), (unsigned)B);
  switch (C) {
#define CASE(CC)                                                                              \
  case CC:                                                                                    \
    hipLaunchKernelGGL((k_fno_pointwise<CC>), grid, dim3(256), 0, s, vin, k, W, b, pre, vout, \
                       nvox, act);                                                            \
    return hipGetLastError();
    FNO_CHANNELS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t fno_pointwise_bwd(int C, const float* dv, const float* pre, const uint16_t* W,
                             float* dpre, float* dvdir, int64_t nvox, int B, int act,
                             hipStream_t s) {
  if (C == 32) {
    const int64_t per = 4 * kMixTiles * 32;
    hipLaunchKernelGGL(k_fno_pointwise_bwd_mfma,
                       dim3((unsigned)((nvox + per - 1) / per), (unsigned)B), dim3(256), 0, s, dv,
                       pre, W, dpre, dvdir, nvox, act);
    return hipGetLastError();
  }
  dim3 grid((unsigned)((nvox + 255) / 256), (unsigned)B);
  switch (C) {
#define CASE(CC)                                                                              \
  case CC:                                                                                    \
    hipLaunchKernelGGL((k_fno_pointwise_bwd<CC>), grid, dim3(256), 0, s, dv, pre, W, dpre,    \
                       dvdir, nvox, act);                                                     \
    return hipGetLastError();
    FNO_CHANNELS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t fno_add(float* a, const float* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fno_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

hipError_t fno_project(int C, const float* v, const uint16_t* Q1, const uint16_t* c1,
                       const uint16_t* Q2, const uint16_t* c2, float* out, int Cp, int64_t nvox,
                       int B, hipStream_t s) {
  dim3 grid((unsigned)((nvox + 255) / 256), (unsigned)B);
  const size_t lds = sizeof(float) * ((size_t)Cp * C + Cp + 4 * Cp);
  switch (C) {
#define CASE(CC)                                                                              \
  case CC:                                                                                    \
    hipLaunchKernelGGL((k_fno_project<CC>), grid, dim3(256), lds, s, v, Q1, c1, Q2, c2, out,  \
                       Cp, nvox);                                                             \
    return hipGetLastError();
    FNO_CHANNELS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t fno_project_bwd(int C, const float* v, const float* dout, const uint16_t* Q1,
                           const uint16_t* c1, const uint16_t* Q2, float* h, float* dh, float* dv,
                           int Cp, int64_t nvox, int B, hipStream_t s) {
  dim3 grid((unsigned)((nvox + 255) / 256), (unsigned)B);
  const size_t lds = sizeof(float) * ((size_t)Cp * C + Cp + 4 * Cp);
  switch (C) {
#define CASE(CC)                                                                              \
  case CC:                                                                                    \
    hipLaunchKernelGGL((k_fno_project_bwd<CC>), grid, dim3(256), lds, s, v, dout, Q1, c1, Q2, \
                       h, dh, dv, Cp, nvox);                                                  \
    return hipGetLastError();
    FNO_CHANNELS(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

// G[p][q] = sum A[b][p][x] Bm[b][q][x]; `part` must hold
// fno_outer_blocks(nvox, B) * P * Q floats.
constexpr int kOuterMaxBlocks = 1024;
int fno_outer_blocks(int64_t nvox, int B) {
  const int64_t tiles = (nvox * B + kOuterTile - 1) / kOuterTile;
  return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, kOuterMaxBlocks));
}

hipError_t fno_outer(const float* A, const float* Bm, const uint8_t* Bu8, int P, int Q,
                     int64_t nvox, int B, float* part, float* out, hipStream_t s) {
  if (P < 1 || Q < 1 || P * Q > 16 * 256) return hipErrorInvalidValue;
  const int64_t total = nvox * B;
  int nb;
  const bool aligned = ((uintptr_t)A % 16 == 0) && ((uintptr_t)Bm % 16 == 0) &&
                       ((uintptr_t)Bu8 % 4 == 0);
  if (nvox % kOuterTile == 0 && aligned) {
    const int PB = (P + 31) / 32, QB = (Q + 31) / 32;
    const int GP = PB >= 4 ? 4 : (PB >= 2 ? 2 : 1);
    const int GQ = std::min(QB >= 4 ? 4 : (QB >= 2 ? 2 : 1), 4 / GP);
    const int64_t ntiles = total / kOuterTile;
    nb = fno_outer_blocks(nvox, B);
    const unsigned groups = (unsigned)(((PB + GP - 1) / GP) * ((QB + GQ - 1) / GQ));
    const size_t lds = sizeof(float) * std::max<size_t>(32 * (GP + GQ) * (kOuterTile + 4), 4096);
    const int bm = Bm ? 0 : (Bu8 ? 1 : 2);
#define OUTER(GPP, GQQ, BMM)                                                              \
  if (GP == GPP && GQ == GQQ && bm == BMM)                                                \
    hipLaunchKernelGGL((k_fno_outer_mfma<GPP, GQQ, BMM>), dim3((unsigned)nb, groups),     \
                       dim3(256), lds, s, A, Bm, Bu8, P, Q, nvox, ntiles, part);
    OUTER(1, 1, 0) else OUTER(1, 2, 0) else OUTER(1, 4, 0) else OUTER(2, 1, 0)
    else OUTER(2, 2, 0) else OUTER(4, 1, 0)
    else OUTER(1, 1, 1) else OUTER(1, 2, 1) else OUTER(1, 4, 1) else OUTER(2, 1, 1)
    else OUTER(2, 2, 1) else OUTER(4, 1, 1)
    else OUTER(1, 1, 2) else OUTER(1, 2, 2) else OUTER(1, 4, 2) else OUTER(2, 1, 2)
    else OUTER(2, 2, 2) else OUTER(4, 1, 2)
#undef OUTER
  } else {  // vector kernel: unaligned operands or a voxel count off the tile
    const int64_t want = std::max<int64_t>(1, (total + 8191) / 8192);  // 8192 pairs per block
    nb = (int)std::min<int64_t>(want, fno_outer_blocks(nvox, B));
    int64_t chunk = (total + nb - 1) / nb;
    chunk = ((chunk + kOuterTile - 1) / kOuterTile) * kOuterTile;
    const size_t lds = sizeof(float) * (size_t)(P + Q) * kOuterTile;
    hipLaunchKernelGGL(k_fno_outer, dim3(nb), dim3(256), lds, s, A, Bm, Bu8, P, Q, nvox, B, chunk,
                       part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fno_sum_parts, dim3((unsigned)((P * Q + 63) / 64)), dim3(64 * kSumWaves), 0,
                     s, part, nb, P * Q, out);
  return hipGetLastError();
}

hipError_t fno_adam(float* p, uint16_t* pb, const float* g, float* m, float* v, int64_t n,
                    float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_fno_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, pb, g, m, v,
                     n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t fno_to_bf16(const float* p, uint16_t* pb, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fno_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, pb, n);
  return hipGetLastError();
}

hipError_t fno_mse(const float* out, const float* tgt, float* dout, int64_t n, double inv_count,
                   double* part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_fno_mse, dim3(nblk), dim3(256), 0, s, out, tgt, dout, n, inv_count, part);
  return hipGetLastError();
}

}  // namespace acm
