// Small MLP surrogate: forward, mean-squared-error backward and Adam, as
// plain HIP kernels.  The network maps sweep parameters to moments of the
// binned count distribution that the matrix-P method produces; it is trained
// on method outputs and screens parameter sweeps, with the method itself as
// the judge (see the Python driver).
//
// Layout: layer l maps width[l] -> width[l+1] with y = x W_l + b_l, W_l stored
// row-major (width[l] rows, width[l+1] columns), then b_l; the layers are
// concatenated in one FP32 parameter vector.  The forward and backward passes
// read the weights from a BF16 copy of that vector (FP32 accumulation); Adam
// updates the FP32 master copy and refreshes the BF16 one.  Hidden layers use
// SiLU, the last layer is linear.  All reductions are in a fixed order (no
// floating-point atomics), so a training run is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "common.h"

namespace mp {

__device__ inline float bf16f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

// Z = X W + b (pre-activation), A = act(Z).  One workgroup per batch row,
// one thread per output column; the input row is staged in LDS.
__global__ __launch_bounds__(256) void mlp_linear_fwd(const float* __restrict__ X, int I, int O,
                                                      const uint16_t* __restrict__ W16,
                                                      const float* __restrict__ bias,
                                                      float* __restrict__ Z, float* __restrict__ A,
                                                      int silu) {
  __shared__ float xs[1024];
  const int b = blockIdx.x;
  for (int i = threadIdx.x; i < I; i += blockDim.x) xs[i] = X[(int64_t)b * I + i];
  __syncthreads();
  for (int o = threadIdx.x; o < O; o += blockDim.x) {
    float acc = bias[o];
    for (int i = 0; i < I; ++i) acc = fmaf(xs[i], bf16f(W16[(int64_t)i * O + o]), acc);
    Z[(int64_t)b * O + o] = acc;
    A[(int64_t)b * O + o] = silu ? acc * sigmoidf(acc) : acc;
  }
}

// dZ = dA * act'(Z) (in place on dA).
__global__ void mlp_act_bwd(float* __restrict__ dA, const float* __restrict__ Z, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float z = Z[i], s = sigmoidf(z);
  dA[i] *= s * (1.0f + z * (1.0f - s));
}

// dX = dZ W^T: one workgroup per batch row, one thread per input column.
__global__ __launch_bounds__(256) void mlp_linear_bwd_x(const float* __restrict__ dZ, int I, int O,
                                                        const uint16_t* __restrict__ W16,
                                                        float* __restrict__ dX) {
  __shared__ float ds[1024];
  const int b = blockIdx.x;
  for (int o = threadIdx.x; o < O; o += blockDim.x) ds[o] = dZ[(int64_t)b * O + o];
  __syncthreads();
  for (int i = threadIdx.x; i < I; i += blockDim.x) {
    float acc = 0.0f;
    const uint16_t* w = W16 + (int64_t)i * O;
    for (int o = 0; o < O; ++o) acc = fmaf(ds[o], bf16f(w[o]), acc);
    dX[(int64_t)b * I + i] = acc;
  }
}

// dW[i][o] = sum_b X[b][i] dZ[b][o]; db[o] = sum_b dZ[b][o] (row i = I).
__global__ void mlp_linear_bwd_w(const float* __restrict__ X, const float* __restrict__ dZ, int B,
                                 int I, int O, float* __restrict__ dW, float* __restrict__ db) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)(I + 1) * O) return;
  const int i = (int)(e / O), o = (int)(e % O);
  float acc = 0.0f;
  if (i < I) {
    for (int b = 0; b < B; ++b) acc = fmaf(X[(int64_t)b * I + i], dZ[(int64_t)b * O + o], acc);
    dW[(int64_t)i * O + o] = acc;
  } else {
    for (int b = 0; b < B; ++b) acc += dZ[(int64_t)b * O + o];
    db[o] = acc;
  }
}

// loss = mean (Yp - Y)^2 over all entries; dY = 2 (Yp - Y) / n.  One block.
__global__ __launch_bounds__(256) void mlp_mse(const float* __restrict__ Yp,
                                               const float* __restrict__ Y, int64_t n,
                                               float* __restrict__ dY, float* __restrict__ loss) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
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
  if (threadIdx.x == 0) *loss = (float)(red[0] / (double)n);
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
  // Z and A of every layer plus two gradient buffers of the widest layer
  int64_t e = 0, wmax = 0;
  for (int l = 0; l < s->n_layers; ++l) e += 2 * (int64_t)batch * s->width[l + 1];
  for (int l = 0; l <= s->n_layers; ++l) wmax = wmax > s->width[l] ? wmax : s->width[l];
  return e + 2 * (int64_t)batch * wmax + 256;
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
    hipLaunchKernelGGL(mlp_linear_fwd, dim3(batch), dim3(256), 0, st, in, I, O, w16 + off,
                       params + off + (int64_t)I * O, Zs[l], As[l],
                       l + 1 < s->n_layers ? 1 : 0);
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
  const int L = s->n_layers;
  const int64_t nout = (int64_t)batch * s->width[L];
  hipLaunchKernelGGL(mlp_mse, dim3(1), dim3(256), 0, st, As[L - 1], Y, nout, g0, loss);
  float* dA = g0;  // gradient w.r.t. the current layer's output
  float* dIn = g1;
  for (int l = L - 1; l >= 0; --l) {
    const int I = s->width[l], O = s->width[l + 1];
    const int64_t off = layer_offset(s, l);
    if (l + 1 < L) {
      const int64_t n = (int64_t)batch * O;
      hipLaunchKernelGGL(mlp_act_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dA,
                         Zs[l], n);
    }
    const float* Xin = l > 0 ? As[l - 1] : X;
    const int64_t nw = (int64_t)(I + 1) * O;
    hipLaunchKernelGGL(mlp_linear_bwd_w, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, Xin,
                       dA, batch, I, O, grads + off, grads + off + (int64_t)I * O);
    if (l > 0) {
      hipLaunchKernelGGL(mlp_linear_bwd_x, dim3(batch), dim3(256), 0, st, dA, I, O, w16 + off, dIn);
      float* t = dA;
      dA = dIn;
      dIn = t;
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
