// sigma-surrogate network kernels (3-64-64-2 GELU MLP) for gfx950.
//
// One wave owns a 32-row tile at a time.  Layer 1 (K = 3) and layer 3 (N = 2)
// are plain FP32 fused multiply-adds on bfloat16-rounded operands; the 64x64
// products (forward layer 2, the W2 gradient and the back-propagated
// hidden-layer error) use v_mfma_f32_32x32x8_bf16.  Intermediate activations
// live in LDS; the operands that only feed matrix products are kept there in
// bfloat16 already.  Gradients are accumulated per work-group (the W2 one in
// MFMA accumulators across tiles), written out per work-group and summed in a
// second pass in a fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "lbm.h"
#include "lbm_mlp.h"

namespace mlp {

constexpr int NH = 64, TR = 32;
constexpr int OFF_W1 = 0, OFF_B1 = 192, OFF_W2 = 256, OFF_B2 = 4352, OFF_W3 = 4416, OFF_B3 = 4544;
constexpr int NP = MLP_NPARAMS;
constexpr int GMAX = 256;  // work-groups of the gradient pass

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

struct Norm {
  float in_mean[3], in_std[3], out_mean[2], out_std[2];
};

// float -> bfloat16 bits, round to nearest even (finite values)
__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }
__device__ __forceinline__ float qbf(float f) { return bf2f(f2bf(f)); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// MFMA 32x32x8 (bf16 in, FP32 accumulate), one wave:
//   C[m][n] += sum_k A(m, k) B(n, k),  m, n in [0, 32), k in [0, K), K % 8 == 0,
//   A(m, k) = a[m * sam + k * sak], B(n, k) = b[n * sbn + k * sbk]  (bfloat16 in LDS).
// Operand layout: lane l supplies row (l & 31) and k = k0 + 4 (l >> 5) + v, v < 4.
// Result layout: lane l, element i holds C[8 (i / 4) + 4 (l >> 5) + i % 4][l & 31].
__device__ __forceinline__ void mm32(const unsigned short* a, int sam, int sak,
                                     const unsigned short* b, int sbn, int sbk, int K, f16v& c) {
  const int l = threadIdx.x & 63, r = l & 31, h = l >> 5;
  for (int k0 = 0; k0 < K; k0 += 8) {
    s4 av, bv;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = k0 + 4 * h + v;
      av[v] = (short)a[r * sam + k * sak];
      bv[v] = (short)b[r * sbn + k * sbk];
    }
    c = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, c, 0, 0, 0);
  }
}
__device__ __forceinline__ int crow(int i) { return 8 * (i >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (i & 3); }

template <bool TRAIN>
__global__ __launch_bounds__(64) void k_mlp(const float* __restrict__ P, Norm nm,
                                            const float* __restrict__ X, const float* __restrict__ T,
                                            float* __restrict__ Y, int B, float* __restrict__ gpart,
                                            float* __restrict__ lpart) {
  __shared__ float W1[NH * 3], b1[NH], b2[NH], W3[2 * NH], b3[2];
  __shared__ unsigned short W2b[NH * NH];
  __shared__ float xs[TR][4];
  __shared__ float z1[TR][NH], z2[TR][NH];
  __shared__ unsigned short h1b[TR][NH], h2b[TR][NH], dzb[TR][NH];
  __shared__ float dy[TR][2];
  __shared__ float red[64][8];
  const int l = threadIdx.x;
  for (int i = l; i < NH * 3; i += 64) W1[i] = P[OFF_W1 + i];
  for (int i = l; i < NH * NH; i += 64) W2b[i] = f2bf(P[OFF_W2 + i]);
  for (int i = l; i < 2 * NH; i += 64) W3[i] = P[OFF_W3 + i];
  b1[l] = P[OFF_B1 + l];
  b2[l] = P[OFF_B2 + l];
  if (l < 2) b3[l] = P[OFF_B3 + l];
  __syncthreads();

  f16v gW2[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 16; ++i) gW2[x][y][i] = 0.f;
  float gW1[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}}, gb1[2] = {0.f, 0.f};
  float gW3[2] = {0.f, 0.f}, gb2 = 0.f, gb3 = 0.f, lsum = 0.f;

  const int ntiles = (B + TR - 1) / TR;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int row0 = t * TR;
    if (l < TR) {  // standardised inputs; rows past B are zero and carry no gradient
      const int r = row0 + l;
#pragma unroll
      for (int i = 0; i < 3; ++i) xs[l][i] = r < B ? (X[3 * r + i] - nm.in_mean[i]) / nm.in_std[i] : 0.f;
    }
    __syncthreads();
    {  // layer 1: lane -> row m, hidden units 32 (l >> 5) .. + 31
      const int m = l & 31, hb = 32 * (l >> 5);
      const float q0 = qbf(xs[m][0]), q1 = qbf(xs[m][1]), q2 = qbf(xs[m][2]);
      for (int j = 0; j < 32; ++j) {
        const int h = hb + j;
        float acc = q0 * qbf(W1[3 * h]);
        acc = fmaf(q1, qbf(W1[3 * h + 1]), acc);
        acc = fmaf(q2, qbf(W1[3 * h + 2]), acc);
        const float z = acc + b1[h];
        z1[m][h] = z;
        h1b[m][h] = f2bf(gelu(z));
      }
    }
    __syncthreads();
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {  // layer 2: z2[m][n] = sum_k h1[m][k] W2[n][k] + b2[n]
      f16v c;
#pragma unroll
      for (int i = 0; i < 16; ++i) c[i] = 0.f;
      mm32(&h1b[0][0], NH, 1, W2b + nb * 32 * NH, NH, 1, NH, c);
      const int n = nb * 32 + (l & 31);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int m = crow(i);
        const float z = c[i] + b2[n];
        z2[m][n] = z;
        h2b[m][n] = f2bf(gelu(z));
      }
    }
    __syncthreads();
    {  // layer 3: lane -> row m, output o
      const int m = l & 31, o = l >> 5;
      float acc = 0.f;
      for (int n = 0; n < NH; ++n) acc = fmaf(bf2f(h2b[m][n]), qbf(W3[o * NH + n]), acc);
      const float y = acc + b3[o];
      const int r = row0 + m;
      if (!TRAIN) {
        if (r < B) Y[2 * r + o] = y * nm.out_std[o] + nm.out_mean[o];
      } else {
        float d = 0.f;
        if (r < B) {
          d = y - (T[2 * r + o] - nm.out_mean[o]) / nm.out_std[o];
          lsum = fmaf(d, d, lsum);
        }
        dy[m][o] = d / (float)B;
      }
    }
    if (TRAIN) {
      __syncthreads();
      {  // W3, b3: lane -> output o, columns n0 and n0 + 32
        const int o = l >> 5, n0 = l & 31;
        for (int m = 0; m < TR; ++m) {
          const float q = qbf(dy[m][o]);
          gW3[0] = fmaf(q, bf2f(h2b[m][n0]), gW3[0]);
          gW3[1] = fmaf(q, bf2f(h2b[m][n0 + 32]), gW3[1]);
          if (n0 == 0) gb3 += dy[m][o];
        }
      }
      {  // dZ2 = (dY W3) * GELU'(Z2): lane -> column n
        const int n = l;
        const float w0 = qbf(W3[n]), w1 = qbf(W3[NH + n]);
        for (int m = 0; m < TR; ++m) {
          const float s = fmaf(qbf(dy[m][1]), w1, qbf(dy[m][0]) * w0);
          const float g = s * gelu_d(z2[m][n]);
          gb2 += g;
          dzb[m][n] = f2bf(g);
        }
      }
      __syncthreads();
      // dW2[n][k] += sum_m dZ2[m][n] H1[m][k]   (A(n, m) = dZ2[m][n], B(k, m) = H1[m][k])
#pragma unroll
      for (int bn = 0; bn < 2; ++bn)
#pragma unroll
        for (int bk = 0; bk < 2; ++bk) mm32(&dzb[0][bn * 32], 1, NH, &h1b[0][bk * 32], 1, NH, TR, gW2[bn][bk]);
      // dH1[m][k] = sum_n dZ2[m][n] W2[n][k]; dZ1 = dH1 * GELU'(Z1); W1, b1 partials
#pragma unroll
      for (int bk = 0; bk < 2; ++bk) {
        f16v c;
#pragma unroll
        for (int i = 0; i < 16; ++i) c[i] = 0.f;
        mm32(&dzb[0][0], NH, 1, W2b + bk * 32, 1, NH, NH, c);
        const int k = bk * 32 + (l & 31);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int m = crow(i);
          const float g = c[i] * gelu_d(z1[m][k]);
          gb1[bk] += g;
          const float q = qbf(g);
          gW1[bk][0] = fmaf(q, qbf(xs[m][0]), gW1[bk][0]);
          gW1[bk][1] = fmaf(q, qbf(xs[m][1]), gW1[bk][1]);
          gW1[bk][2] = fmaf(q, qbf(xs[m][2]), gW1[bk][2]);
        }
      }
    }
    __syncthreads();  // the next tile overwrites LDS
  }
  if (!TRAIN) return;

  float* G = gpart + (size_t)blockIdx.x * NP;
  // W1, b1: lanes l and l ^ 32 hold the same columns for different rows
#pragma unroll
  for (int bk = 0; bk < 2; ++bk) {
    red[l][4 * bk + 0] = gW1[bk][0];
    red[l][4 * bk + 1] = gW1[bk][1];
    red[l][4 * bk + 2] = gW1[bk][2];
    red[l][4 * bk + 3] = gb1[bk];
  }
  __syncthreads();
  if (l < 32) {
#pragma unroll
    for (int bk = 0; bk < 2; ++bk) {
      const int k = bk * 32 + l;
#pragma unroll
      for (int i = 0; i < 3; ++i) G[OFF_W1 + 3 * k + i] = red[l][4 * bk + i] + red[l + 32][4 * bk + i];
      G[OFF_B1 + k] = red[l][4 * bk + 3] + red[l + 32][4 * bk + 3];
    }
  }
#pragma unroll
  for (int bn = 0; bn < 2; ++bn)
#pragma unroll
    for (int bk = 0; bk < 2; ++bk)
#pragma unroll
      for (int i = 0; i < 16; ++i)
        G[OFF_W2 + (bn * 32 + crow(i)) * NH + bk * 32 + (l & 31)] = gW2[bn][bk][i];
  G[OFF_B2 + l] = gb2;
  {
    const int o = l >> 5, n0 = l & 31;
    G[OFF_W3 + o * NH + n0] = gW3[0];
    G[OFF_W3 + o * NH + n0 + 32] = gW3[1];
    if (n0 == 0) G[OFF_B3 + o] = gb3;
  }
  __syncthreads();
  red[l][0] = lsum;
  __syncthreads();
  if (l == 0) {
    float s = 0.f;
    for (int i = 0; i < 64; ++i) s += red[i][0];
    lpart[blockIdx.x] = s;
  }
}

// grad[p] = sum over work-groups in index order; loss = sum / (2 B)
__global__ void k_reduce(const float* __restrict__ gpart, int G, float* __restrict__ grad,
                         const float* __restrict__ lpart, float* __restrict__ loss, int B) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NP) {
    float s = 0.f;
    for (int b = 0; b < G; ++b) s += gpart[(size_t)b * NP + p];
    grad[p] = s;
  }
  if (p == 0 && loss) {
    float s = 0.f;
    for (int b = 0; b < G; ++b) s += lpart[b];
    loss[0] = s / (2.0f * (float)B);
  }
}

// Adam; c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)
__global__ void k_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  const float gi = g[p];
  const float mi = b1 * m[p] + (1.f - b1) * gi;
  const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
  m[p] = mi;
  v[p] = vi;
  P[p] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

}  // namespace mlp

using namespace mlp;

struct mlp_ctx {
  Norm nm;
  int max_batch;
  float *P, *m, *v, *grad, *gpart, *lpart, *loss;
  hipStream_t st;
  int64_t t;  // Adam steps taken
};

namespace {
constexpr size_t kAl = 256;
size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }
size_t layout(size_t* off) {
  size_t o = 0;
  const size_t sizes[7] = {NP * 4, NP * 4, NP * 4, NP * 4, (size_t)GMAX * NP * 4, GMAX * 4, 4};
  for (int i = 0; i < 7; ++i) {
    off[i] = o;
    o += al(sizes[i]);
  }
  return o;
}
Norm to_norm(const mlp_norm& n) {
  Norm r;
  std::memcpy(&r, &n, sizeof r);
  return r;
}
int grad_blocks(int B) { return std::min(GMAX, (B + TR - 1) / TR); }
}  // namespace

extern "C" {

int mlp_workspace_bytes(int32_t max_batch, size_t* bytes) {
  if (max_batch < 1 || !bytes) return LBM_EINVAL;
  size_t off[7];
  *bytes = layout(off);
  return LBM_OK;
}

int mlp_init(const float* host_params, const mlp_norm* norm, int32_t max_batch, void* ws,
             size_t ws_bytes, void* stream, mlp_ctx** out) {
  if (!host_params || !norm || max_batch < 1 || !ws || !out) return LBM_EINVAL;
  *out = nullptr;
  size_t off[7];
  if (ws_bytes < layout(off)) return LBM_ENOSPACE;
  if (reinterpret_cast<uintptr_t>(ws) % kAl) return LBM_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (!(norm->in_std[i] > 0)) return LBM_EINVAL;
  for (int i = 0; i < 2; ++i)
    if (!(norm->out_std[i] > 0)) return LBM_EINVAL;
  mlp_ctx* c = new mlp_ctx{};
  char* w = static_cast<char*>(ws);
  c->P = reinterpret_cast<float*>(w + off[0]);
  c->m = reinterpret_cast<float*>(w + off[1]);
  c->v = reinterpret_cast<float*>(w + off[2]);
  c->grad = reinterpret_cast<float*>(w + off[3]);
  c->gpart = reinterpret_cast<float*>(w + off[4]);
  c->lpart = reinterpret_cast<float*>(w + off[5]);
  c->loss = reinterpret_cast<float*>(w + off[6]);
  c->nm = to_norm(*norm);
  c->max_batch = max_batch;
  c->st = static_cast<hipStream_t>(stream);
  int st = mlp_set_params(c, host_params);
  if (st != LBM_OK) {
    delete c;
    return st;
  }
  *out = c;
  return LBM_OK;
}

int mlp_set_params(mlp_ctx* c, const float* host_params) {
  if (!c || !host_params) return LBM_EINVAL;
  std::vector<float> zero(NP, 0.f);
  if (hipMemcpyAsync(c->P, host_params, NP * 4, hipMemcpyHostToDevice, c->st) != hipSuccess ||
      hipMemcpyAsync(c->m, zero.data(), NP * 4, hipMemcpyHostToDevice, c->st) != hipSuccess ||
      hipMemcpyAsync(c->v, zero.data(), NP * 4, hipMemcpyHostToDevice, c->st) != hipSuccess ||
      hipStreamSynchronize(c->st) != hipSuccess)
    return LBM_EHIP;
  c->t = 0;
  return LBM_OK;
}

int mlp_get_params(mlp_ctx* c, float* host_params) {
  if (!c || !host_params) return LBM_EINVAL;
  if (hipMemcpyAsync(host_params, c->P, NP * 4, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
      hipStreamSynchronize(c->st) != hipSuccess)
    return LBM_EHIP;
  return LBM_OK;
}

int mlp_set_norm(mlp_ctx* c, const mlp_norm* norm) {
  if (!c || !norm) return LBM_EINVAL;
  c->nm = to_norm(*norm);
  return LBM_OK;
}

int mlp_forward(mlp_ctx* c, const float* X, float* Y, int32_t B) {
  if (!c || !X || !Y || B < 1 || B > c->max_batch) return LBM_EINVAL;
  const int G = std::min(4096, (B + TR - 1) / TR);
  hipLaunchKernelGGL(k_mlp<false>, dim3(G), dim3(64), 0, c->st, c->P, c->nm, X, (const float*)nullptr, Y,
                     B, (float*)nullptr, (float*)nullptr);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}

int mlp_gradient(mlp_ctx* c, const float* X, const float* T, int32_t B, float* grad, float* loss) {
  if (!c || !X || !T || !grad || B < 1 || B > c->max_batch) return LBM_EINVAL;
  const int G = grad_blocks(B);
  hipLaunchKernelGGL(k_mlp<true>, dim3(G), dim3(64), 0, c->st, c->P, c->nm, X, T, (float*)nullptr, B,
                     c->gpart, c->lpart);
  hipLaunchKernelGGL(k_reduce, dim3((NP + 255) / 256), dim3(256), 0, c->st, (const float*)c->gpart, G,
                     grad, (const float*)c->lpart, loss, B);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}

int mlp_adam(mlp_ctx* c, const float* grad, float lr, float b1, float b2, float eps) {
  if (!c || !grad || !(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return LBM_EINVAL;
  c->t += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)c->t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)c->t)));
  hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, c->st, c->P, c->m, c->v, grad, lr, b1,
                     b2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}

int mlp_train_step(mlp_ctx* c, const float* X, const float* T, int32_t B, float lr, float* loss) {
  int st = mlp_gradient(c, X, T, B, c ? c->grad : nullptr, loss);
  if (st != LBM_OK) return st;
  return mlp_adam(c, c->grad, lr, 0.9f, 0.999f, 1e-8f);
}

int mlp_destroy(mlp_ctx* c) {
  if (!c) return LBM_EINVAL;
  (void)hipStreamSynchronize(c->st);
  delete c;
  return LBM_OK;
}

}  // extern "C"
