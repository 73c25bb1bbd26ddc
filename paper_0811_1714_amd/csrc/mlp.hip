// Schedule model: a float32 multilayer perceptron, 4 inputs -> 3 hidden layers of 64
// (ReLU) -> one output per candidate schedule (predicted log runtime).  Hand-written
// forward, backward, loss and Adam kernels.  Parameters are one flat array, layer by
// layer: W (fan_in x fan_out, row-major) then b (fan_out).  Activations are kept as
// pre-activations z; the input of the next layer is relu(z), applied on read.
//
// Every reduction (over the batch for dW and db, over the mask for the count) runs in
// one thread or one workgroup in a fixed order, so results do not depend on timing.
#include "gf2_internal.h"

namespace gf2 {
namespace {

constexpr int NIN = 4, NH = 64, NL = 3;   // hidden layers

__host__ __device__ inline int fan_in(int l) { return l == 0 ? NIN : NH; }
__host__ __device__ inline int fan_out(int l, int nout) { return l == NL ? nout : NH; }
__host__ __device__ inline int64_t param_offset(int l, int nout, bool bias) {
  int64_t off = 0;
  for (int i = 0; i < l; ++i) off += (int64_t)fan_in(i) * fan_out(i, nout) + fan_out(i, nout);
  return off + (bias ? (int64_t)fan_in(l) * fan_out(l, nout) : 0);
}

// Z[b][o] = sum_i X'[b][i] W[i][o] + bias[o], with X' = relu(X) when relu_in.
__global__ void linear_fwd(const float* __restrict__ X, int64_t batch, int I, int O, const float* __restrict__ W,
                           const float* __restrict__ bias, int relu_in, float* __restrict__ Z) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= batch * O) return;
  const int64_t b = t / O;
  const int o = (int)(t % O);
  float s = bias[o];
  for (int i = 0; i < I; ++i) {
    float x = X[b * I + i];
    if (relu_in) x = x > 0.f ? x : 0.f;
    s = fmaf(x, W[(int64_t)i * O + o], s);
  }
  Z[t] = s;
}

// count = sum of the mask (one workgroup, fixed-order tree).
__global__ void mask_count(const float* __restrict__ M, int64_t n, float* __restrict__ out) {
  __shared__ float part[256];
  float s = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += M[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0] > 1.f ? part[0] : 1.f;
}

// dY = 2 (Y - T) M / count, and the per-element squared error for the loss.
__global__ void mse_grad(const float* __restrict__ Y, const float* __restrict__ T, const float* __restrict__ M,
                         int64_t n, const float* __restrict__ cnt, float* __restrict__ dY, float* __restrict__ se) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float d = (Y[i] - T[i]) * M[i];
  dY[i] = 2.f * d / cnt[0];
  if (se) se[i] = d * d / cnt[0];
}

// Loss = sum of se (one workgroup, fixed order).
__global__ void sum_reduce(const float* __restrict__ x, int64_t n, float* __restrict__ out) {
  __shared__ float part[256];
  float s = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0];
}

// dW[i][o] = sum_b X'[b][i] dZ[b][o]  (threads i*O + o),  db[o] = sum_b dZ[b][o]  (threads I*O + o).
__global__ void linear_bwd_params(const float* __restrict__ X, int64_t batch, int I, int O, int relu_in,
                                  const float* __restrict__ dZ, float* __restrict__ dW, float* __restrict__ db) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= I * O + O) return;
  if (t < I * O) {
    const int i = t / O, o = t % O;
    float s = 0.f;
    for (int64_t b = 0; b < batch; ++b) {
      float x = X[b * I + i];
      if (relu_in) x = x > 0.f ? x : 0.f;
      s = fmaf(x, dZ[b * O + o], s);
    }
    dW[t] = s;
  } else {
    const int o = t - I * O;
    float s = 0.f;
    for (int64_t b = 0; b < batch; ++b) s += dZ[b * O + o];
    db[o] = s;
  }
}

// dZprev[b][i] = (sum_o dZ[b][o] W[i][o]) * (Zprev[b][i] > 0).
__global__ void linear_bwd_input(const float* __restrict__ dZ, int64_t batch, int I, int O,
                                 const float* __restrict__ W, const float* __restrict__ Zprev,
                                 float* __restrict__ dZprev) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= batch * I) return;
  const int64_t b = t / I;
  const int i = (int)(t % I);
  float s = 0.f;
  for (int o = 0; o < O; ++o) s = fmaf(dZ[b * O + o], W[(int64_t)i * O + o], s);
  dZprev[t] = Zprev[t] > 0.f ? s : 0.f;
}

// Adam (Kingma and Ba), bias-corrected.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void argmin_kernel(const float* __restrict__ Y, int64_t batch, int O, const uint8_t* __restrict__ allowed,
                              int32_t* __restrict__ out) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  int best = -1;
  float bv = 0.f;
  for (int o = 0; o < O; ++o) {
    if (allowed && !allowed[o]) continue;
    const float y = Y[b * O + o];
    if (best < 0 || y < bv) { best = o; bv = y; }
  }
  out[b] = best;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int64_t mlp_param_count(int nout) { return param_offset(NL + 1, nout, false); }

gf2_status mlp_forward(const float* params, const float* X, int64_t batch, int nout, float* Y, float* acts,
                       hipStream_t s) {
  const float* in = X;
  for (int l = 0; l <= NL; ++l) {
    const int I = fan_in(l), O = fan_out(l, nout);
    float* out = l == NL ? Y : acts + (int64_t)l * batch * NH;
    if (batch > 0)
      hipLaunchKernelGGL(linear_fwd, dim3(blocks_for(batch * O)), dim3(256), 0, s, in, batch, I, O,
                         params + param_offset(l, nout, false), params + param_offset(l, nout, true), l > 0 ? 1 : 0,
                         out);
    gf2_status st = hip_check(hipGetLastError(), "mlp forward launch");
    if (st != GF2_OK) return st;
    in = out;
  }
  return GF2_OK;
}

gf2_status mlp_backward(const float* params, const float* X, int64_t batch, int nout, const float* acts,
                        const float* Y, const float* T, const float* M, float* grads, float* scratch, float* loss,
                        hipStream_t s) {
  // scratch layout: [cnt(1) pad(63)] [dY batch*nout] [se batch*nout] [dZa batch*NH] [dZb batch*NH]
  float* cnt = scratch;
  float* dY = scratch + 64;
  float* se = dY + batch * nout;
  float* dA = se + batch * nout;
  float* dB = dA + batch * NH;
  const int64_t ny = batch * nout;
  hipLaunchKernelGGL(mask_count, dim3(1), dim3(256), 0, s, M, ny, cnt);
  if (ny > 0) hipLaunchKernelGGL(mse_grad, dim3(blocks_for(ny)), dim3(256), 0, s, Y, T, M, ny, cnt, dY, se);
  if (loss) hipLaunchKernelGGL(sum_reduce, dim3(1), dim3(256), 0, s, se, ny, loss);
  const float* dZ = dY;
  for (int l = NL; l >= 0; --l) {
    const int I = fan_in(l), O = fan_out(l, nout);
    const float* in = l == 0 ? X : acts + (int64_t)(l - 1) * batch * NH;
    hipLaunchKernelGGL(linear_bwd_params, dim3(blocks_for((int64_t)I * O + O)), dim3(256), 0, s, in, batch, I, O,
                       l > 0 ? 1 : 0, dZ, grads + param_offset(l, nout, false), grads + param_offset(l, nout, true));
    if (l > 0) {
      float* dprev = (dZ == dA) ? dB : dA;
      if (batch > 0)
        hipLaunchKernelGGL(linear_bwd_input, dim3(blocks_for(batch * I)), dim3(256), 0, s, dZ, batch, I, O,
                           params + param_offset(l, nout, false), acts + (int64_t)(l - 1) * batch * NH, dprev);
      dZ = dprev;
    }
    gf2_status st = hip_check(hipGetLastError(), "mlp backward launch");
    if (st != GF2_OK) return st;
  }
  return GF2_OK;
}

int64_t mlp_scratch_floats(int64_t batch, int nout) { return 64 + 2 * batch * nout + 2 * batch * NH; }

gf2_status mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, int32_t step, float lr, float b1,
                    float b2, float eps, hipStream_t s) {
  if (n <= 0) return GF2_OK;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hip_check(hipGetLastError(), "adam launch");
}

gf2_status mlp_argmin(const float* Y, int64_t batch, int nout, const uint8_t* allowed, int32_t* out, hipStream_t s) {
  if (batch <= 0) return GF2_OK;
  hipLaunchKernelGGL(argmin_kernel, dim3(blocks_for(batch)), dim3(256), 0, s, Y, batch, nout, allowed, out);
  return hip_check(hipGetLastError(), "argmin launch");
}

// Host forward for one row (the single-product MODEL policy).
void mlp_forward_host(const float* params, const float* x, int nout, float* y) {
  float a[NH], b[NH];
  const float* in = x;
  for (int l = 0; l <= NL; ++l) {
    const int I = fan_in(l), O = fan_out(l, nout);
    const float* W = params + param_offset(l, nout, false);
    const float* bias = params + param_offset(l, nout, true);
    float* out = l == NL ? y : ((l & 1) ? b : a);
    for (int o = 0; o < O; ++o) {
      float s = bias[o];
      for (int i = 0; i < I; ++i) {
        float v = in[i];
        if (l > 0) v = v > 0.f ? v : 0.f;
        s = fmaf(v, W[i * O + o], s);
      }
      out[o] = s;
    }
    in = out;
  }
}

}  // namespace gf2
