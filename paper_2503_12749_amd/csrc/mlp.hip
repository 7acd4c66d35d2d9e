// Small MLP surrogate: forward, mean-squared-error backward and Adam, as
// plain HIP kernels.  The network maps sweep parameters to moments of the
// binned count distribution that the matrix-P method produces; it is trained
// on method outputs and screens parameter sweeps, with the method itself
// checking its picks (see the Python driver).
//
// Layout: layer l maps width[l] -> width[l+1] with y = x W_l + b_l, W_l stored
// row-major (width[l] rows, width[l+1] columns), then b_l; the layers are
// concatenated in one FP32 parameter vector.  The forward and backward passes
// read the weights from a BF16 copy of that vector (FP32 accumulation); Adam
// updates the FP32 master copy and refreshes the BF16 one.  Hidden layers use
// SiLU, the last layer is linear.  All reductions are in a fixed order (no
// floating-point atomics), so a training run is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace mp {

__device__ inline float bf16f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

// Products with the BF16 weights run on the BF16 matrix cores: the FP32
// operand x is split into three BF16 terms, x = h + m + l (each the rounded
// remainder of the previous), so that h W + m W + l W carries x to FP32
// precision (24 bits) and each product of BF16 values is exact in the FP32
// accumulation.  A workgroup of four waves computes a 64 x 64 tile of
//   C[R x N] = Aop[R x K] Bop[K x N]
// with v_mfma_f32_32x32x16_bf16, staging 32-deep K chunks in LDS: Aop as three
// BF16 planes [row][k] and Bop transposed as [col][k] (80-byte rows: the
// 16-byte fragment reads of 16 consecutive rows hit distinct banks).
//   MODE 0 (forward):  Aop = X (batch x I), Bop = W (I x O); epilogue
//                      Z = C + b, A = SiLU(Z) on hidden layers, Z on the last.
//   MODE 1 (dX):       Aop = dZ (batch x O), Bop = W^T; epilogue multiplies by
//                      SiLU'(Zprev) when the layer below is hidden, giving its
//                      dZ directly.
// Fragment layout: lane l holds Aop[l % 32][8 (l / 32) + e], Bop[8 (l / 32) + e]
// [l % 32] (e = 0..7) of a 16-deep step; output register r is row
// 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32 of the wave's 32 x 32 block.
// (One-wave 32 x 32 workgroups, four times as many for these small layers,
// measured slower: 44.6 against 30.8 us per forward layer at batch 256.)
constexpr int MLP_T = 64, MLP_KC = 32, MLP_KP = MLP_KC + 8, MLP_THREADS = 256;

template <int MODE>
__global__ __launch_bounds__(MLP_THREADS) void mlp_gemm_bf16(const float* __restrict__ Aop,
                                                     const uint16_t* __restrict__ W16, int R,
                                                     int K, int N, const float* __restrict__ bias,
                                                     const float* __restrict__ Zprev,
                                                     float* __restrict__ Z, float* __restrict__ Act,
                                                     int silu) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[3][MLP_T][MLP_KP];
  __shared__ __attribute__((aligned(16))) uint16_t sB[MLP_T][MLP_KP];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r0 = blockIdx.x * MLP_T, n0 = blockIdx.y * MLP_T;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int lr = lane & 31, lh = lane >> 5;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int k0 = 0; k0 < K; k0 += MLP_KC) {
    for (int e = threadIdx.x; e < MLP_T * MLP_KC; e += MLP_THREADS) {
      const int r = e / MLP_KC, k = e % MLP_KC;
      const float x = (r0 + r < R && k0 + k < K) ? Aop[(int64_t)(r0 + r) * K + k0 + k] : 0.0f;
      const uint16_t h = to_bf16(x);
      const float x1 = x - bf16f(h);
      const uint16_t m = to_bf16(x1);
      sA[0][r][k] = h;
      sA[1][r][k] = m;
      sA[2][r][k] = to_bf16(x1 - bf16f(m));
    }
    for (int e = threadIdx.x; e < MLP_T * MLP_KC; e += MLP_THREADS) {
      if constexpr (MODE == 0) {  // W[k][n], coalesced along n
        const int k = e / MLP_T, n = e % MLP_T;
        sB[n][k] = (k0 + k < K && n0 + n < N) ? W16[(int64_t)(k0 + k) * N + n0 + n] : (uint16_t)0;
      } else {  // W^T: Bop[k][n] = W[n][k] (W is N x K), coalesced along k
        const int n = e / MLP_KC, k = e % MLP_KC;
        sB[n][k] = (k0 + k < K && n0 + n < N) ? W16[(int64_t)(n0 + n) * K + k0 + k] : (uint16_t)0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < MLP_KC; ks += 16) {
      const int kk = ks + 8 * lh;
      const bf16x8 b = *(const bf16x8*)&sB[wc + lr][kk];
      // small terms first
#pragma unroll
      for (int t = 2; t >= 0; --t) {
        const bf16x8 a = *(const bf16x8*)&sA[t][wr + lr][kk];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int col = n0 + wc + lr;
  if (col >= N) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = r0 + wr + 8 * (r >> 2) + 4 * lh + (r & 3);
    if (row >= R) continue;
    const int64_t o = (int64_t)row * N + col;
    if constexpr (MODE == 0) {
      const float z = acc[r] + bias[col];
      Z[o] = z;
      Act[o] = silu ? z * sigmoidf(z) : z;
    } else {
      float g = acc[r];
      if (Zprev) {
        const float z = Zprev[o], sg = sigmoidf(z);
        g *= sg * (1.0f + z * (1.0f - sg));
      }
      Z[o] = g;
    }
  }
}

// Weight and bias gradients of one layer in one product on the FP32 matrix
// cores (both operands are FP32 activations or gradients):
//   G[(I + 1) x O] = [X | 1]^T dZ,  rows i < I: dW, row I: db = sum_b dZ[b][.]
// which is the layer's slice of the gradient vector (W row-major, then b).
// v_mfma_f32_32x32x2f32: lane l holds A[l % 32][l / 32] and B[l / 32][l % 32]
// of a 2-deep step; 64 x 64 tile per workgroup of four waves, 32-deep batch
// chunks staged in LDS ([i][b] with a 33-float pitch, [b][o]).
__global__ __launch_bounds__(MLP_THREADS) void mlp_gemm_dw(const float* __restrict__ X,
                                                   const float* __restrict__ dZ, int Bt, int I,
                                                   int O, float* __restrict__ G) {
  __shared__ float sX[MLP_T][MLP_KC + 1];
  __shared__ float sD[MLP_KC][MLP_T];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i0 = blockIdx.x * MLP_T, o0 = blockIdx.y * MLP_T;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int lr = lane & 31, lh = lane >> 5;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int b0 = 0; b0 < Bt; b0 += MLP_KC) {
    for (int e = threadIdx.x; e < MLP_T * MLP_KC; e += MLP_THREADS) {
      const int b = e / MLP_T, i = e % MLP_T;  // coalesced along i
      float x = 0.0f;
      if (b0 + b < Bt && i0 + i <= I) x = (i0 + i < I) ? X[(int64_t)(b0 + b) * I + i0 + i] : 1.0f;
      sX[i][b] = x;
      const int o = i;
      sD[b][o] = (b0 + b < Bt && o0 + o < O) ? dZ[(int64_t)(b0 + b) * O + o0 + o] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < MLP_KC; ks += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(sX[wr + lr][ks + lh], sD[ks + lh][wc + lr], acc,
                                                  0, 0, 0);
    __syncthreads();
  }
  const int col = o0 + wc + lr;
  if (col >= O) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = i0 + wr + 8 * (r >> 2) + 4 * lh + (r & 3);
    if (row <= I) G[(int64_t)row * O + col] = acc[r];
  }
}

// loss = mean (Yp - Y)^2 over all entries; dY = 2 (Yp - Y) / n.  Each block
// sums its grid-stride share in FP64 into part[block]; mlp_mse_finish adds the
// partials in block order (no atomics: the same bits on every run).
constexpr int kMseBlocks = 64;
__global__ __launch_bounds__(256) void mlp_mse_part(const float* __restrict__ Yp,
                                                    const float* __restrict__ Y, int64_t n,
                                                    float* __restrict__ dY,
                                                    double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float d = Yp[i] - Y[i];
    dY[i] = 2.0f * d / (float)n;
    acc += (double)d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void mlp_mse_finish(const double* __restrict__ part, int nb, int64_t n,
                               float* __restrict__ loss) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[b];
  *loss = (float)(s / (double)n);
}

__global__ void mlp_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                         float* __restrict__ m, float* __restrict__ v, uint16_t* __restrict__ p16,
                         float lr, float b1, float b2, float eps, float wd, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  // Adam with decoupled weight decay
  const float pi = p[i] - lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * p[i]);
  p[i] = pi;
  p16[i] = to_bf16(pi);
}

__global__ void mlp_round_bf16(int64_t n, const float* __restrict__ p, uint16_t* __restrict__ p16) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p16[i] = to_bf16(p[i]);
}

// ---------------------------------------------------------------- host side

static int64_t layer_offset(const mp_mlp_shape* s, int l) {
  int64_t off = 0;
  for (int k = 0; k < l; ++k) off += (int64_t)(s->width[k] + 1) * s->width[k + 1];
  return off;
}

int64_t mlp_param_count(const mp_mlp_shape* s) { return layer_offset(s, s->n_layers); }

static int64_t act_elems(const mp_mlp_shape* s, int32_t batch) {
  // Z and A of every layer, two gradient buffers of the widest layer, and the
  // loss partials (kMseBlocks doubles)
  int64_t e = 0, wmax = 0;
  for (int l = 0; l < s->n_layers; ++l) e += 2 * (int64_t)batch * s->width[l + 1];
  for (int l = 0; l <= s->n_layers; ++l) wmax = wmax > s->width[l] ? wmax : s->width[l];
  return e + 2 * (int64_t)batch * wmax + 2 * kMseBlocks + 256;
}

static dim3 mlp_grid(int R, int N) {
  return dim3((unsigned)((R + MLP_T - 1) / MLP_T), (unsigned)((N + MLP_T - 1) / MLP_T));
}

size_t mlp_workspace(const mp_mlp_shape* s, int32_t batch) {
  return (size_t)act_elems(s, batch) * 4 + 256;
}

static mp_status mlp_fwd_impl(const mp_mlp_shape* s, const uint16_t* w16, const float* params,
                              const float* X, int32_t batch, float* ws, hipStream_t st,
                              float** Zs, float** As) {
  float* cur = ws;
  const float* in = X;
  for (int l = 0; l < s->n_layers; ++l) {
    const int I = s->width[l], O = s->width[l + 1];
    const int64_t off = layer_offset(s, l);
    Zs[l] = cur;
    cur += (int64_t)batch * O;
    As[l] = cur;
    cur += (int64_t)batch * O;
    hipLaunchKernelGGL(mlp_gemm_bf16<0>, mlp_grid(batch, O), dim3(MLP_THREADS), 0, st, in, w16 + off,
                       (int)batch, I, O, params + off + (int64_t)I * O, (const float*)nullptr,
                       Zs[l], As[l], l + 1 < s->n_layers ? 1 : 0);
    in = As[l];
  }
  MP_HIP_LAUNCH_CHECK("mlp forward launch");
  return MP_OK;
}

mp_status mlp_forward(const mp_mlp_shape* s, const uint16_t* w16, const float* params,
                      const float* X, int32_t batch, float* Y, void* ws, hipStream_t st) {
  float* Zs[MP_MLP_MAX_LAYERS];
  float* As[MP_MLP_MAX_LAYERS];
  mp_status r = mlp_fwd_impl(s, w16, params, X, batch, (float*)ws, st, Zs, As);
  if (r != MP_OK) return r;
  const int O = s->width[s->n_layers];
  const hipError_t e =
      hipMemcpyAsync(Y, As[s->n_layers - 1], (size_t)batch * O * 4, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) {
    set_error("mlp forward copy: %s", hipGetErrorString(e));
    return MP_ERR_HIP;
  }
  return MP_OK;
}

mp_status mlp_loss_grad(const mp_mlp_shape* s, const uint16_t* w16, const float* params,
                        const float* X, const float* Y, int32_t batch, float* grads, float* loss,
                        void* ws, hipStream_t st) {
  float* Zs[MP_MLP_MAX_LAYERS];
  float* As[MP_MLP_MAX_LAYERS];
  mp_status r = mlp_fwd_impl(s, w16, params, X, batch, (float*)ws, st, Zs, As);
  if (r != MP_OK) return r;
  int64_t used = 0;
  for (int l = 0; l < s->n_layers; ++l) used += 2 * (int64_t)batch * s->width[l + 1];
  int64_t wmax = 0;
  for (int l = 0; l <= s->n_layers; ++l) wmax = wmax > s->width[l] ? wmax : s->width[l];
  float* g0 = (float*)ws + used;
  float* g1 = g0 + (int64_t)batch * wmax;
  double* part = (double*)(((uintptr_t)(g1 + (int64_t)batch * wmax) + 7) & ~(uintptr_t)7);
  const int L = s->n_layers;
  const int64_t nout = (int64_t)batch * s->width[L];
  const int nb = (int)std::min<int64_t>(kMseBlocks, (nout + 255) / 256);
  hipLaunchKernelGGL(mlp_mse_part, dim3(nb), dim3(256), 0, st, As[L - 1], Y, nout, g0, part);
  hipLaunchKernelGGL(mlp_mse_finish, dim3(1), dim3(64), 0, st, part, nb, nout, loss);
  // dZ of the output layer (linear) is dY; the dX product of layer l applies
  // SiLU' of layer l - 1, so each step below starts from that layer's dZ
  float* dZ = g0;
  float* dNext = g1;
  for (int l = L - 1; l >= 0; --l) {
    const int I = s->width[l], O = s->width[l + 1];
    const int64_t off = layer_offset(s, l);
    const float* Xin = l > 0 ? As[l - 1] : X;
    hipLaunchKernelGGL(mlp_gemm_dw, mlp_grid(I + 1, O), dim3(MLP_THREADS), 0, st, Xin, dZ, (int)batch, I,
                       O, grads + off);
    if (l > 0) {
      hipLaunchKernelGGL(mlp_gemm_bf16<1>, mlp_grid(batch, I), dim3(MLP_THREADS), 0, st, dZ, w16 + off,
                         (int)batch, O, I, (const float*)nullptr, Zs[l - 1], dNext, (float*)nullptr,
                         0);
      float* t = dZ;
      dZ = dNext;
      dNext = t;
    }
  }
  MP_HIP_LAUNCH_CHECK("mlp backward launch");
  return MP_OK;
}

mp_status mlp_adam_launch(int64_t n, float* params, const float* grads, float* m, float* v,
                          uint16_t* w16, float lr, float b1, float b2, float eps, float wd,
                          int32_t step, hipStream_t st) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(mlp_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, params,
                     grads, m, v, w16, lr, b1, b2, eps, wd, c1, c2);
  MP_HIP_LAUNCH_CHECK("mlp adam launch");
  return MP_OK;
}

mp_status mlp_round_launch(int64_t n, const float* params, uint16_t* w16, hipStream_t st) {
  hipLaunchKernelGGL(mlp_round_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                     params, w16);
  MP_HIP_LAUNCH_CHECK("mlp round launch");
  return MP_OK;
}

}  // namespace mp
