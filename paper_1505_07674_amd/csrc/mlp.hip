// mlp.hip -- the surrogate network of log L: 17 -> 256 -> 256 -> 256 -> 1, SiLU.
//
// Matrix products run on the matrix cores with bfloat16 operands and float32
// accumulation (v_mfma_f32_16x16x32_bf16): a 64x64 block tile, four waves of
// 2x2 MFMA tiles, operands staged in LDS with k contiguous so that each lane's
// eight k values are one 16-byte LDS read. Epilogues fuse the bias and SiLU
// (forward), the SiLU derivative (backward dZ) or plain stores (weight
// gradients). The 256 -> 1 head, column sums, loss and Adam run on the VALU.
// Operands are rounded to bfloat16 (nearest even) at fixed points: normalised
// input, weights, activations H and back-propagated dZ; everything else is
// float32.
//
// Flat parameter layout (float32): W1 [256][17], b1 [256], W2 [256][256], b2,
// W3 [256][256], b3, W4 [1][256], b4 [1]. Normalisation block: x_shift [17],
// x_scale [17], y_shift, y_scale.
#include <stdint.h>

#include <cmath>

#include "internal.h"
#include "kernels.h"
#include "mlp.h"

namespace lensed {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;   // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

constexpr int BM = 64, BN = 64, BK = 32, LDSK = BK + 8;

struct GemmArgs {
  const uint16_t* A;
  long sam, sak;        // A(m, k) = A[m * sam + k * sak]
  const uint16_t* B;
  long sbk, sbn;        // B(k, n) = B[k * sbk + n * sbn]
  int M, N, K;
  int epi;              // 0: Z = acc + bias, H = bf16(silu(Z)); 1: dZ = acc * silu'(Zin); 2: C = acc
  const float* bias;
  const float* Zin;
  long ldz;
  float* Cf;            // float32 output (Z, dZ or C)
  uint16_t* Cb;         // bfloat16 output (H or dZ), may be null
  long ldc;
};

// Lane l of a 16x16x32 MFMA holds A[m = l % 16][k = 8 (l / 16) + j] and
// B[k = 8 (l / 16) + j][n = l % 16], j = 0..7, and receives
// D[m = 4 (l / 16) + j][n = l % 16], j = 0..3.
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  __shared__ uint16_t As[BM][LDSK];
  __shared__ uint16_t Bt[BN][LDSK];   // B transposed: [n][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bm = blockIdx.y * BM, bn = blockIdx.x * BN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const int lr = tid >> 2, lk = (tid & 3) * 8;   // staging: one row (or column), eight k values
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    {
      const int m = bm + lr;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + lk + j;
        As[lr][lk + j] = (m < g.M && k < g.K) ? g.A[(long)m * g.sam + (long)k * g.sak] : (uint16_t)0;
      }
      const int n = bn + lr;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k0 + lk + j;
        Bt[lr][lk + j] = (n < g.N && k < g.K) ? g.B[(long)k * g.sbk + (long)n * g.sbn] : (uint16_t)0;
      }
    }
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const u16x8 va = *(const u16x8*)&As[wm + i * 16 + fr][fk];
      const u16x8 vb = *(const u16x8*)&Bt[wn + i * 16 + fr][fk];
      a[i] = __builtin_bit_cast(bf16x8, va);
      b[i] = __builtin_bit_cast(bf16x8, vb);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  const int cn = lane & 15, cm = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = bm + wm + i * 16 + cm + r;
        const int n = bn + wn + j * 16 + cn;
        if (m >= g.M || n >= g.N) continue;
        const float v = acc[i][j][r];
        const long o = (long)m * g.ldc + n;
        if (g.epi == 0) {
          const float z = v + g.bias[n];
          g.Cf[o] = z;
          g.Cb[o] = f2bf(silu(z));
        } else if (g.epi == 1) {
          const float dz = v * dsilu(g.Zin[(long)m * g.ldz + n]);
          g.Cf[o] = dz;
          g.Cb[o] = f2bf(dz);
        } else {
          g.Cf[o] = v;
        }
      }
}

// bfloat16 copies of the weights: W1 padded to [256][32], W2, W3 [256][256], W4 [256].
__global__ void convert_weights_kernel(const float* __restrict__ p, uint16_t* __restrict__ wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < MLP_H * MLP_KPAD) {
    const int o = i / MLP_KPAD, k = i - o * MLP_KPAD;
    wb[i] = k < MLP_IN ? f2bf(p[MLP_OFF_W1 + o * MLP_IN + k]) : (uint16_t)0;
  }
  if (i < MLP_H * MLP_H) {
    wb[MLP_WB_W2 + i] = f2bf(p[MLP_OFF_W2 + i]);
    wb[MLP_WB_W3 + i] = f2bf(p[MLP_OFF_W3 + i]);
  }
  if (i < MLP_H) wb[MLP_WB_W4 + i] = f2bf(p[MLP_OFF_W4 + i]);
}

// X0[m][k] = bf16((x[m][k] - x_shift[k]) * x_scale[k]) for k < 17, zero up to 32.
__global__ void input_kernel(const float* __restrict__ x, const float* __restrict__ norm, uint16_t* __restrict__ X0,
                             int B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * MLP_KPAD) return;
  const int m = i / MLP_KPAD, k = i - m * MLP_KPAD;
  X0[i] = k < MLP_IN ? f2bf((x[(long)m * MLP_IN + k] - norm[k]) * norm[MLP_IN + k]) : (uint16_t)0;
}

// Head: out = H3 . W4 + b4, one wave per row. mode 0: y = y_shift + y_scale out.
// mode 1 (training): t = (y - y_shift)/y_scale, d = 2 (out - t)/B, sq = (out - t)^2.
__global__ __launch_bounds__(256) void head_kernel(const uint16_t* __restrict__ H3, const uint16_t* __restrict__ wb,
                                                   const float* __restrict__ p, const float* __restrict__ norm,
                                                   int B, int mode, float* __restrict__ y, const float* __restrict__ yt,
                                                   float* __restrict__ d, float* __restrict__ sq) {
  const int lane = threadIdx.x & 63;
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= B) return;
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < MLP_H / 64; ++j) {
    const int n = lane + 64 * j;
    s = fmaf(bf2f(H3[(long)m * MLP_H + n]), bf2f(wb[MLP_WB_W4 + n]), s);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) {
    const float out = s + p[MLP_OFF_B4];
    if (mode == 0) {
      y[m] = norm[2 * MLP_IN] + norm[2 * MLP_IN + 1] * out;
    } else {
      const float t = (yt[m] - norm[2 * MLP_IN]) / norm[2 * MLP_IN + 1];
      const float r = out - t;
      d[m] = 2.0f * r / (float)B;
      sq[m] = r * r;
    }
  }
}

// dZ3[m][n] = d[m] W4[n] silu'(Z3[m][n]), float32 and bfloat16.
__global__ void head_bwd_kernel(const float* __restrict__ d, const uint16_t* __restrict__ wb,
                                const float* __restrict__ Z3, float* __restrict__ dZ, uint16_t* __restrict__ dZb,
                                int B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * MLP_H) return;
  const int m = i / MLP_H, n = i - m * MLP_H;
  const float v = d[m] * bf2f(wb[MLP_WB_W4 + n]) * dsilu(Z3[i]);
  dZ[i] = v;
  dZb[i] = f2bf(v);
}

// out[n] = sum_m w[m] * X[m][n] over M rows (w = 1 when null; X float32 or
// bfloat16). One block per column, fixed-order tree: deterministic.
__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ Xf, const uint16_t* __restrict__ Xb,
                                                     const float* __restrict__ w, int M, long ld,
                                                     float* __restrict__ out) {
  __shared__ float red[256];
  const int n = blockIdx.x;
  float s = 0.0f;
  for (int m = threadIdx.x; m < M; m += 256) {
    const float x = Xf ? Xf[(long)m * ld + n] : bf2f(Xb[(long)m * ld + n]);
    s += w ? w[m] * x : x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = red[0];
}

__global__ __launch_bounds__(256) void mean_kernel(const float* __restrict__ x, int n, float* __restrict__ out) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] / (float)n;
}

// Adam (Kingma & Ba 2015): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p -= lr (m / bc1) / (sqrt(v / bc2) + eps), bc = 1 - b^t. The factors 1 - b
// and the bias corrections come from the host in float64 (1 - b2 rounded from a
// float b2 would carry a 1e-5 relative error).
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float beta1, float omb1, float beta2, float omb2,
                            float eps, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = fmaf(beta1, m[i], omb1 * gi);
  const float vi = fmaf(beta2, v[i], omb2 * gi * gi);
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

hipError_t gemm(const GemmArgs& a, hipStream_t st) {
  dim3 grid((a.N + BN - 1) / BN, (a.M + BM - 1) / BM);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

GemmArgs fwd_layer(const uint16_t* X, long ldx, const uint16_t* W, long ldw, int B, int K, const float* bias, float* Z,
                   uint16_t* H) {
  GemmArgs a{};
  a.A = X; a.sam = ldx; a.sak = 1;                  // X [B][K]
  a.B = W; a.sbk = 1; a.sbn = ldw;                  // B(k, n) = W[n][k]
  a.M = B; a.N = MLP_H; a.K = K;
  a.epi = 0; a.bias = bias; a.Cf = Z; a.Cb = H; a.ldc = MLP_H;
  return a;
}

}  // namespace

hipError_t mlp_forward(const float* params, const float* norm, const float* x, float* y, int B, const MlpScratch& s,
                       hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipError_t e;
  const int T = 256;
  hipLaunchKernelGGL(convert_weights_kernel, dim3((MLP_H * MLP_H + T - 1) / T), dim3(T), 0, st, params, s.wb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(input_kernel, dim3((B * MLP_KPAD + T - 1) / T), dim3(T), 0, st, x, norm, s.X0, B);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = gemm(fwd_layer(s.X0, MLP_KPAD, s.wb, MLP_KPAD, B, MLP_KPAD, params + MLP_OFF_B1, s.Z[0], s.H[0]), st)))
    return e;
  if ((e = gemm(fwd_layer(s.H[0], MLP_H, s.wb + MLP_WB_W2, MLP_H, B, MLP_H, params + MLP_OFF_B2, s.Z[1], s.H[1]), st)))
    return e;
  if ((e = gemm(fwd_layer(s.H[1], MLP_H, s.wb + MLP_WB_W3, MLP_H, B, MLP_H, params + MLP_OFF_B3, s.Z[2], s.H[2]), st)))
    return e;
  hipLaunchKernelGGL(head_kernel, dim3((B + 3) / 4), dim3(256), 0, st, s.H[2], s.wb, params, norm, B, 0, y, nullptr,
                     nullptr, nullptr);
  return hipGetLastError();
}

hipError_t mlp_grad(const float* params, const float* norm, const float* x, const float* yt, int B, float* grad,
                    float* loss, const MlpScratch& s, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipError_t e;
  const int T = 256;
  hipLaunchKernelGGL(convert_weights_kernel, dim3((MLP_H * MLP_H + T - 1) / T), dim3(T), 0, st, params, s.wb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(input_kernel, dim3((B * MLP_KPAD + T - 1) / T), dim3(T), 0, st, x, norm, s.X0, B);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = gemm(fwd_layer(s.X0, MLP_KPAD, s.wb, MLP_KPAD, B, MLP_KPAD, params + MLP_OFF_B1, s.Z[0], s.H[0]), st)))
    return e;
  if ((e = gemm(fwd_layer(s.H[0], MLP_H, s.wb + MLP_WB_W2, MLP_H, B, MLP_H, params + MLP_OFF_B2, s.Z[1], s.H[1]), st)))
    return e;
  if ((e = gemm(fwd_layer(s.H[1], MLP_H, s.wb + MLP_WB_W3, MLP_H, B, MLP_H, params + MLP_OFF_B3, s.Z[2], s.H[2]), st)))
    return e;
  hipLaunchKernelGGL(head_kernel, dim3((B + 3) / 4), dim3(256), 0, st, s.H[2], s.wb, params, norm, B, 1, nullptr, yt,
                     s.d, s.sq);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, st, s.sq, B, loss);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // layer 4: dW4[n] = sum_m d[m] H3[m][n], db4 = sum_m d[m], dZ3 = d W4 silu'(Z3)
  hipLaunchKernelGGL(colsum_kernel, dim3(MLP_H), dim3(256), 0, st, nullptr, s.H[2], s.d, B, (long)MLP_H,
                     grad + MLP_OFF_W4);
  hipLaunchKernelGGL(colsum_kernel, dim3(1), dim3(256), 0, st, s.d, nullptr, nullptr, B, 1L, grad + MLP_OFF_B4);
  float* dz = s.dZ;
  float* dz_next = s.dZ2;
  uint16_t* dzb = s.dZb;
  uint16_t* dzb_next = s.dZb2;
  hipLaunchKernelGGL(head_bwd_kernel, dim3((B * MLP_H + T - 1) / T), dim3(T), 0, st, s.d, s.wb, s.Z[2], dz, dzb, B);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int offW[3] = {MLP_OFF_W1, MLP_OFF_W2, MLP_OFF_W3};
  const int offB[3] = {MLP_OFF_B1, MLP_OFF_B2, MLP_OFF_B3};
  const long wbo[3] = {0, MLP_WB_W2, MLP_WB_W3};
  for (int l = 2; l >= 0; --l) {
    // dW_l[o][i] = sum_b dZ_l[b][o] H_{l-1}[b][i]
    const uint16_t* Hin = l == 0 ? s.X0 : s.H[l - 1];
    const long ldh = l == 0 ? MLP_KPAD : MLP_H;
    GemmArgs a{};
    a.A = dzb; a.sam = 1; a.sak = MLP_H;
    a.B = Hin; a.sbk = ldh; a.sbn = 1;
    a.M = MLP_H; a.N = l == 0 ? MLP_IN : MLP_H; a.K = B;
    a.epi = 2; a.Cf = grad + offW[l]; a.ldc = l == 0 ? MLP_IN : MLP_H;
    if ((e = gemm(a, st))) return e;
    hipLaunchKernelGGL(colsum_kernel, dim3(MLP_H), dim3(256), 0, st, dz, nullptr, nullptr, B, (long)MLP_H,
                       grad + offB[l]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (l > 0) {
      // dZ_{l-1} = (dZ_l W_l) * silu'(Z_{l-1})
      GemmArgs b{};
      b.A = dzb; b.sam = MLP_H; b.sak = 1;
      b.B = s.wb + wbo[l]; b.sbk = MLP_H; b.sbn = 1;   // B(k = o, n = i) = W_l[o][i]
      b.M = B; b.N = MLP_H; b.K = MLP_H;
      b.epi = 1; b.Zin = s.Z[l - 1]; b.ldz = MLP_H; b.Cf = dz_next; b.Cb = dzb_next; b.ldc = MLP_H;
      if ((e = gemm(b, st))) return e;
      float* t = dz; dz = dz_next; dz_next = t;
      uint16_t* tb = dzb; dzb = dzb_next; dzb_next = tb;
    }
  }
  return hipSuccess;
}

hipError_t mlp_adam(float* params, const float* grad, float* m, float* v, int n, int step, double lr, double beta1,
                    double beta2, double eps, hipStream_t st) {
  const double bc1 = 1.0 - std::pow(beta1, (double)step), bc2 = 1.0 - std::pow(beta2, (double)step);
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, st, params, grad, m, v, n, (float)lr,
                     (float)beta1, (float)(1.0 - beta1), (float)beta2, (float)(1.0 - beta2), (float)eps, (float)bc1,
                     (float)bc2);
  return hipGetLastError();
}

}  // namespace lensed
