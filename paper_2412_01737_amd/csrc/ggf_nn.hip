// Learned block proposal: the masked-patch convolutional conditional and its
// training kernels (forward, backward, gradient reduction, Adam).
//
// A P x P patch of sites (2 P^2 links) is resampled from a factorised
// Bernoulli whose logits come from four valid 3x3 convolutions (2 -> 32 -> 32
// -> 32 -> 2 channels, tanh between layers) over the (P+8)^2 window of the
// link field around the patch, with every periodic image of the patch masked
// to 0 (inputs 1 - 2k elsewhere).  Because the patch is masked, the forward
// and reverse proposal probabilities of a Metropolis-Hastings block move come
// from one forward pass.  Weights are bfloat16 (converted on load), biases and
// activations float32, accumulation float32.
//
// Parameter vector (float32 master copy): W1[32][2][3][3], b1[32],
// W2[32][32][3][3], b2[32], W3[32][32][3][3], b3[32], W4[2][32][3][3], b4[2].
#include "ggf_device.h"
#include "ggf_nn.h"
#include "ggf_pair.h"

namespace {

constexpr int kCh = 32;
constexpr int kHalo = 4;
constexpr int kPmax = 4;
constexpr int kWmax = kPmax + 2 * kHalo;   // 12
constexpr int kOffW1 = 0, kOffB1 = 576, kOffW2 = 608, kOffB2 = 9824, kOffW3 = 9856, kOffB3 = 19072;
constexpr int kOffW4 = 19104, kOffB4 = 19680;
static_assert(kOffB4 + 2 == GGF_NN_NPARAMS, "parameter layout");

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// Round-to-nearest-even float32 -> bfloat16.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return static_cast<uint16_t>(u >> 16);
}

struct NNView {
  const uint16_t *wq;   // bf16 weights (biases unused)
  const float *p;       // float32 master (biases read from here)
};

// Activation buffers of one example in LDS.
struct Acts {
  float in[2 * kWmax * kWmax];
  float h1[kCh * (kWmax - 2) * (kWmax - 2)];
  float h2[kCh * (kWmax - 4) * (kWmax - 4)];
  float h3[kCh * (kWmax - 6) * (kWmax - 6)];
  float z[2 * kPmax * kPmax];
};

// Window of chain c around patch p: channel mu = 1 - 2 k of link (site, mu), 0 on patch sites (all images).
__device__ void build_window(const int8_t *lk, int L, int P, int patch, float *in) {
  const int W = P + 2 * kHalo;
  const int npx = L / P;
  const int ox = P * (patch % npx), oy = P * (patch / npx);
  for (int t = threadIdx.x; t < 2 * W * W; t += blockDim.x) {
    const int mu = t / (W * W);
    const int r = t - mu * W * W;
    const int wy = r / W, wx = r - wy * W;
    const int sx = ((ox - kHalo + wx) % L + L) % L, sy = ((oy - kHalo + wy) % L + L) % L;
    const bool inside = ((sx - ox + L) % L) < P && ((sy - oy + L) % L) < P;
    in[t] = inside ? 0.0f : 1.0f - 2.0f * static_cast<float>(lk[2 * (sy * L + sx) + mu]);
  }
}

// out[co][y][x] = b[co] + sum w[co][ci][dy][dx] in[ci][y+dy][x+dx], valid, optional tanh.
__device__ void conv_fwd(const float *in, int ci_n, int Hin, const uint16_t *wq, const float *b, int co_n, float *out,
                         bool act) {
  const int Ho = Hin - 2;
  const int total = co_n * Ho * Ho;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int co = t / (Ho * Ho);
    const int r = t - co * Ho * Ho;
    const int y = r / Ho, x = r - y * Ho;
    float acc = b[co];
    const uint16_t *w = wq + co * ci_n * 9;
    for (int ci = 0; ci < ci_n; ++ci) {
      const float *src = in + ci * Hin * Hin + y * Hin + x;
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) acc = fmaf(bf16_to_f32(w[ci * 9 + dy * 3 + dx]), src[dy * Hin + dx], acc);
    }
    out[t] = act ? tanhf(acc) : acc;
  }
}

__device__ void forward_all(const NNView &nn, int P, Acts &A) {
  const int W = P + 2 * kHalo;
  conv_fwd(A.in, 2, W, nn.wq + kOffW1, nn.p + kOffB1, kCh, A.h1, true);
  __syncthreads();
  conv_fwd(A.h1, kCh, W - 2, nn.wq + kOffW2, nn.p + kOffB2, kCh, A.h2, true);
  __syncthreads();
  conv_fwd(A.h2, kCh, W - 4, nn.wq + kOffW3, nn.p + kOffB3, kCh, A.h3, true);
  __syncthreads();
  conv_fwd(A.h3, kCh, W - 6, nn.wq + kOffW4, nn.p + kOffB4, 2, A.z, false);
  __syncthreads();
}

// dW[co][ci][dy][dx] += sum_yx dout[co][y][x] in[ci][y+dy][x+dx]; db[co] += sum_yx dout[co]
// (accumulated into this workgroup's private gradient slice g).
__device__ void conv_wgrad(const float *in, int ci_n, int Hin, const float *dout, int co_n, float *gw, float *gb) {
  const int Ho = Hin - 2;
  const int nw = co_n * ci_n * 9;
  for (int t = threadIdx.x; t < nw + co_n; t += blockDim.x) {
    if (t < nw) {
      const int co = t / (ci_n * 9);
      const int r = t - co * ci_n * 9;
      const int ci = r / 9, k = r - ci * 9, dy = k / 3, dx = k - dy * 3;
      const float *d = dout + co * Ho * Ho;
      const float *s = in + ci * Hin * Hin + dy * Hin + dx;
      float acc = 0.0f;
      for (int y = 0; y < Ho; ++y)
        for (int x = 0; x < Ho; ++x) acc = fmaf(d[y * Ho + x], s[y * Hin + x], acc);
      gw[t] += acc;
    } else {
      const int co = t - nw;
      const float *d = dout + co * Ho * Ho;
      float acc = 0.0f;
      for (int q = 0; q < Ho * Ho; ++q) acc += d[q];
      gb[co] += acc;
    }
  }
}

// din[ci][yy][xx] = (1 - h^2) * sum_{co,dy,dx} w[co][ci][dy][dx] dout[co][yy-dy][xx-dx]  (h = in, a tanh output)
__device__ void conv_dgrad(const float *h, int ci_n, int Hin, const float *dout, int co_n, const uint16_t *wq,
                           float *din) {
  const int Ho = Hin - 2;
  for (int t = threadIdx.x; t < ci_n * Hin * Hin; t += blockDim.x) {
    const int ci = t / (Hin * Hin);
    const int r = t - ci * Hin * Hin;
    const int yy = r / Hin, xx = r - yy * Hin;
    float acc = 0.0f;
    for (int co = 0; co < co_n; ++co) {
      const uint16_t *w = wq + (co * ci_n + ci) * 9;
      const float *d = dout + co * Ho * Ho;
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const int y = yy - dy;
        if (y < 0 || y >= Ho) continue;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const int x = xx - dx;
          if (x < 0 || x >= Ho) continue;
          acc = fmaf(bf16_to_f32(w[dy * 3 + dx]), d[y * Ho + x], acc);
        }
      }
    }
    din[t] = acc * (1.0f - h[t] * h[t]);
  }
}

struct Grads {
  float d3[kCh * (kWmax - 6) * (kWmax - 6)];
  float d2[kCh * (kWmax - 4) * (kWmax - 4)];
  float d1[kCh * (kWmax - 2) * (kWmax - 2)];
  float dz[2 * kPmax * kPmax];
};

// One workgroup strides over examples; forward, optional backward into g_slice (this workgroup's slice).
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_nn_run(NNArgs a, const int *__restrict__ ex_chain,
                                                const int *__restrict__ ex_patch, int n_ex, float *__restrict__ logits,
                                                float *__restrict__ gpart, double *__restrict__ lpart) {
  __shared__ Acts A;
  __shared__ Grads D;
  __shared__ double s_loss;
  const int P = a.P;
  const int W = P + 2 * kHalo;
  const int np = 2 * P * P;
  const NNView nn{a.wq, a.params};
  float *g = TRAIN ? gpart + static_cast<size_t>(blockIdx.x) * GGF_NN_NPARAMS : nullptr;
  if (threadIdx.x == 0) s_loss = 0.0;
  for (int e = blockIdx.x; e < n_ex; e += gridDim.x) {
    const int c = ex_chain[e];
    const ChainDev ch = a.chains[c];
    const int8_t *lk = a.links + ch.link_off;
    build_window(lk, ch.L, P, ex_patch[e], A.in);
    __syncthreads();
    forward_all(nn, P, A);
    const int npx = ch.L / P;
    const int ox = P * (ex_patch[e] % npx), oy = P * (ex_patch[e] / npx);
    // logits in patch order l = 2 (y P + x) + mu; z is stored [mu][y][x]
    for (int l = threadIdx.x; l < np; l += blockDim.x) {
      const int mu = l & 1, s = l >> 1, y = s / P, x = s - y * P;
      const float z = A.z[mu * P * P + y * P + x];
      if (!TRAIN) {
        logits[static_cast<size_t>(e) * np + l] = z;
      } else {
        const int site = ((oy + y) % ch.L) * ch.L + (ox + x) % ch.L;
        const float lab = static_cast<float>(lk[2 * site + mu]);
        D.dz[mu * P * P + y * P + x] = 1.0f / (1.0f + expf(-z)) - lab;
        const double zd = z;
        const double bce = (zd > 0 ? zd + log1p(exp(-zd)) : log1p(exp(zd))) - lab * zd;
        atomicAdd(&s_loss, bce);
      }
    }
    __syncthreads();
    if (TRAIN) {
      conv_wgrad(A.h3, kCh, W - 6, D.dz, 2, g + kOffW4, g + kOffB4);
      conv_dgrad(A.h3, kCh, W - 6, D.dz, 2, nn.wq + kOffW4, D.d3);
      __syncthreads();
      conv_wgrad(A.h2, kCh, W - 4, D.d3, kCh, g + kOffW3, g + kOffB3);
      conv_dgrad(A.h2, kCh, W - 4, D.d3, kCh, nn.wq + kOffW3, D.d2);
      __syncthreads();
      conv_wgrad(A.h1, kCh, W - 2, D.d2, kCh, g + kOffW2, g + kOffB2);
      conv_dgrad(A.h1, kCh, W - 2, D.d2, kCh, nn.wq + kOffW2, D.d1);
      __syncthreads();
      conv_wgrad(A.in, 2, W, D.d1, kCh, g + kOffW1, g + kOffB1);
      __syncthreads();
    }
  }
  if (TRAIN && threadIdx.x == 0) lpart[blockIdx.x] = s_loss;
}

__global__ void k_nn_zero(float *__restrict__ g, size_t n) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n; i += gridDim.x * static_cast<size_t>(blockDim.x))
    g[i] = 0.0f;
}

__global__ void k_nn_reduce(const float *__restrict__ gpart, int nslices, float scale, float *__restrict__ grad,
                            const double *__restrict__ lpart, double *__restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < GGF_NN_NPARAMS) {
    float acc = 0.0f;
    for (int s = 0; s < nslices; ++s) acc += gpart[static_cast<size_t>(s) * GGF_NN_NPARAMS + i];
    grad[i] = acc * scale;
  }
  if (i == 0) {
    double l = 0.0;
    for (int s = 0; s < nslices; ++s) l += lpart[s];
    *loss = l * scale;
  }
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, p -= lr mhat / (sqrt(vhat) + eps).
__global__ void k_nn_adam(float *__restrict__ p, uint16_t *__restrict__ wq, float *__restrict__ m, float *__restrict__ v,
                          const float *__restrict__ g, float lr, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= GGF_NN_NPARAMS) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  p[i] = pi;
  wq[i] = f32_to_bf16(pi);
}

__global__ void k_nn_quantize(const float *__restrict__ p, uint16_t *__restrict__ wq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < GGF_NN_NPARAMS) wq[i] = f32_to_bf16(p[i]);
}

// Training examples of step t: (chain, patch) from Philox at counter (t, e, 0, 8).
__global__ void k_nn_examples(int *__restrict__ ex_chain, int *__restrict__ ex_patch, int n_ex, uint32_t t,
                              uint32_t k0, uint32_t k1, int n_chains, int npatch) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_ex) return;
  const uint4 x = ggf_philox(make_uint4(t, static_cast<uint32_t>(e), 0u, 8u), k0, k1);
  ex_chain[e] = static_cast<int>(x.x % static_cast<uint32_t>(n_chains));
  ex_patch[e] = static_cast<int>(x.y % static_cast<uint32_t>(npatch));
}

}  // namespace

// ---------------------------------------------------------------------------
// Block move: decision (forward pass, proposal, r x r Gauss-Jordan, K > 1 patch
// Pfaffians, Metropolis-Hastings) and the rank-r Woodbury update.
#include "ggf_block.inc"
#include "ggf_window.inc"

void ggf_nn_forward_launch(const NNArgs &a, const int *ex_chain, const int *ex_patch, int n_ex, float *logits,
                           hipStream_t s) {
  const int grid = n_ex < 1024 ? n_ex : 1024;
  hipLaunchKernelGGL((k_nn_run<false>), dim3(grid), dim3(256), 0, s, a, ex_chain, ex_patch, n_ex, logits, nullptr,
                     nullptr);
}

void ggf_nn_grad_launch(const NNArgs &a, const int *ex_chain, const int *ex_patch, int n_ex, float *gpart,
                        int nslices, double *lpart, float *grad, double *loss, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_zero, dim3(512), dim3(256), 0, s, gpart, static_cast<size_t>(nslices) * GGF_NN_NPARAMS);
  const int grid = n_ex < nslices ? n_ex : nslices;
  hipLaunchKernelGGL((k_nn_run<true>), dim3(grid), dim3(256), 0, s, a, ex_chain, ex_patch, n_ex, nullptr, gpart,
                     lpart);
  hipLaunchKernelGGL(k_nn_reduce, dim3((GGF_NN_NPARAMS + 255) / 256), dim3(256), 0, s, gpart, grid,
                     1.0f / static_cast<float>(n_ex), grad, lpart, loss);
}

void ggf_nn_adam_launch(float *p, uint16_t *wq, float *m, float *v, const float *g, float lr, int t, hipStream_t s) {
  const float c1 = 1.0f - powf(0.9f, static_cast<float>(t));
  const float c2 = 1.0f - powf(0.999f, static_cast<float>(t));
  hipLaunchKernelGGL(k_nn_adam, dim3((GGF_NN_NPARAMS + 255) / 256), dim3(256), 0, s, p, wq, m, v, g, lr, c1, c2);
}

void ggf_nn_quantize_launch(const float *p, uint16_t *wq, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_quantize, dim3((GGF_NN_NPARAMS + 255) / 256), dim3(256), 0, s, p, wq);
}

void ggf_nn_examples_launch(int *ex_chain, int *ex_patch, int n_ex, uint32_t t, uint32_t k0, uint32_t k1, int n_chains,
                            int npatch, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_examples, dim3((n_ex + 255) / 256), dim3(256), 0, s, ex_chain, ex_patch, n_ex, t, k0, k1,
                     n_chains, npatch);
}
