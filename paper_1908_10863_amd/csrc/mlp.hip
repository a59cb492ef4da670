// The learned form's network on the GPU: a 4-layer tanh perceptron of width 128
// that maps (reaction component, four features of (rho, zeta)) to the
// remainders of the 4p+1 Sommerfeld initial values (eq. scaledsommerfeldint,
// M = 0 and 1), trained in FP32 by the kernels below (forward pass, backward
// pass by the chain rule, deterministic gradient reduction, Adam).
//
// Parameters, one flat FP32 vector: E [ncomp][128] (first layer, one-hot
// component input), A [4][128] (first layer, features), b1 [128], W2 [128][128],
// b2, W3 [128][128], b3, W4 [128][nout], b4 [nout]; W[k][j] maps input k to
// output j, so that a row of W is contiguous across the outputs that the
// threads of a wave compute together.
//
// Work layout: one workgroup of 256 threads per tile of 64 samples.  The
// tile's activations stay in LDS between layers ([64][132] floats per
// buffer, rows padded to keep 16-byte alignment); the weights are read from
// global memory, shared by all tiles through L2/L1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "fmm_internal.h"

namespace fmmlm {
namespace {

constexpr int kH = kMlpH;
constexpr int kT = 64;         // samples per workgroup
constexpr int kP = kH + 4;     // LDS row stride (floats)
constexpr int kThreads = 256;

struct MlpDev {
  const float *E, *A, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
  int ncomp, nout;
};

MlpDev dev_view(const MlpNet& n) {
  const float* p = n.params;
  return MlpDev{p + n.off[0], p + n.off[1], p + n.off[2], p + n.off[3], p + n.off[4],
                p + n.off[5], p + n.off[6], p + n.off[7], p + n.off[8], n.ncomp, n.nout};
}

__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ inline uint64_t rng64(uint64_t seed, uint64_t stream, uint64_t i) {
  return mix64(seed ^ mix64(stream + 0x9E3779B97F4A7C15ull * (i + 1)));
}

// Out[s][j] = tanh(b[j] + sum_k In[s][k] W[k][j]) for the tile's 64 x 128
// outputs: thread (ts, tj) computes samples 4ts..4ts+3 x outputs 8tj..8tj+7.
__device__ inline void dense_tanh(const float (*In)[kP], float (*Out)[kP], const float* __restrict__ W,
                                  const float* __restrict__ b) {
  const int ts = threadIdx.x >> 4, tj = threadIdx.x & 15;
  float acc[4][8];
#pragma unroll
  for (int jj = 0; jj < 8; ++jj) {
    const float bb = b[8 * tj + jj];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i][jj] = bb;
  }
  for (int k = 0; k < kH; k += 4) {
    float4 x[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = *reinterpret_cast<const float4*>(&In[4 * ts + i][k]);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const float4 w0 = *reinterpret_cast<const float4*>(W + (k + kk) * kH + 8 * tj);
      const float4 w1 = *reinterpret_cast<const float4*>(W + (k + kk) * kH + 8 * tj + 4);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float xv = kk == 0 ? x[i].x : kk == 1 ? x[i].y : kk == 2 ? x[i].z : x[i].w;
        acc[i][0] += xv * w0.x;
        acc[i][1] += xv * w0.y;
        acc[i][2] += xv * w0.z;
        acc[i][3] += xv * w0.w;
        acc[i][4] += xv * w1.x;
        acc[i][5] += xv * w1.y;
        acc[i][6] += xv * w1.z;
        acc[i][7] += xv * w1.w;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) Out[4 * ts + i][8 * tj + jj] = tanhf(acc[i][jj]);
}

__device__ inline void store_rows(const float (*S)[kP], float* __restrict__ g, int64_t s0, int ns) {
  for (int o = threadIdx.x; o < kT * kH; o += kThreads) {
    const int s = o / kH, k = o - s * kH;
    if (s < ns) g[(s0 + s) * kH + k] = S[s][k];
  }
}

__device__ inline void load_rows(float (*S)[kP], const float* __restrict__ g, int64_t s0, int ns) {
  for (int o = threadIdx.x; o < kT * kH; o += kThreads) {
    const int s = o / kH, k = o - s * kH;
    S[s][k] = (s < ns) ? g[(s0 + s) * kH + k] : 0.0f;
  }
}

// First layer: tanh(E[c] + f A + b1) into Out.
__device__ inline void first_layer(const MlpDev& w, const int32_t* __restrict__ comp,
                                   const float4* __restrict__ feat, int64_t s0, int ns, float (*Out)[kP]) {
  const int j = threadIdx.x & (kH - 1);
  const float a0 = w.A[j], a1 = w.A[kH + j], a2 = w.A[2 * kH + j], a3 = w.A[3 * kH + j], bb = w.b1[j];
  for (int s = threadIdx.x >> 7; s < kT; s += kThreads / kH) {
    float v = 0.0f;
    if (s < ns) {
      const float4 f = feat[s0 + s];
      const int c = comp[s0 + s];
      v = tanhf(w.E[(int64_t)c * kH + j] + a0 * f.x + a1 * f.y + a2 * f.z + a3 * f.w + bb);
    }
    Out[s][j] = v;
  }
}

__global__ __launch_bounds__(kThreads) void mlp_forward_kernel(MlpDev w, const int32_t* __restrict__ comp,
                                                               const float4* __restrict__ feat, int64_t n,
                                                               float* __restrict__ out, int ldo, int ocols,
                                                               float* __restrict__ h1g, float* __restrict__ h2g,
                                                               float* __restrict__ h3g) {
  __shared__ float Ha[kT][kP];
  __shared__ float Hb[kT][kP];
  const int64_t s0 = (int64_t)blockIdx.x * kT;
  const int ns = (int)std::min<int64_t>(kT, n - s0);
  first_layer(w, comp, feat, s0, ns, Ha);
  __syncthreads();
  if (h1g) store_rows(Ha, h1g, s0, ns);
  dense_tanh(Ha, Hb, w.W2, w.b2);
  __syncthreads();
  if (h2g) store_rows(Hb, h2g, s0, ns);
  dense_tanh(Hb, Ha, w.W3, w.b3);
  __syncthreads();
  if (h3g) store_rows(Ha, h3g, s0, ns);
  // output layer: samples sg + 4q (q < 16) of wave sg, outputs j = lane, lane + 64
  const int sg = threadIdx.x >> 6;
  for (int j = threadIdx.x & 63; j < ocols; j += 64) {
    float acc[16];
    const float bb = w.b4[j];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = bb;
    for (int k = 0; k < kH; ++k) {
      const float wk = w.W4[k * w.nout + j];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] += Ha[sg + 4 * q][k] * wk;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int s = sg + 4 * q;
      if (s < ns) out[(s0 + s) * ldo + j] = acc[q];
    }
  }
}

// g[k][j] = sum_s In[s][k] Dl[s][j], k < nin, j < nj (this tile's partial).
__device__ inline void grad_w(const float (*In)[kP], const float (*Dl)[kP], int nin, int nj,
                              float* __restrict__ g) {
  for (int o = threadIdx.x; o < nin * nj; o += kThreads) {
    const int k = o / nj, j = o - k * nj;
    float acc = 0.0f;
    for (int s = 0; s < kT; ++s) acc += In[s][k] * Dl[s][j];
    g[o] = acc;
  }
}

__device__ inline void col_sum(const float (*Dl)[kP], int nj, float* __restrict__ g) {
  for (int j = threadIdx.x; j < nj; j += kThreads) {
    float acc = 0.0f;
    for (int s = 0; s < kT; ++s) acc += Dl[s][j];
    g[j] = acc;
  }
}

// Gout[s][k] = (sum_j Dl[s][j] W[k][j]) (1 - Hs[s][k]^2): the gradient with
// respect to the pre-activation of the layer whose output is Hs.
__device__ inline void back_dense(const float (*Dl)[kP], int nj, const float* __restrict__ W, int ldw,
                                  const float (*Hs)[kP], float (*Gout)[kP]) {
  const int k = threadIdx.x & (kH - 1), sg = threadIdx.x >> 7;
  float acc[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) acc[q] = 0.0f;
  for (int j = 0; j < nj; ++j) {
    const float wv = W[k * ldw + j];
#pragma unroll
    for (int q = 0; q < 32; ++q) acc[q] += Dl[sg * 32 + q][j] * wv;
  }
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    const int s = sg * 32 + q;
    const float h = Hs[s][k];
    Gout[s][k] = acc[q] * (1.0f - h * h);
  }
}

// One tile's share of the gradient of mean((out - y)^2) over n * nout entries,
// written to part (layout of the parameters); the tile's sum of squared
// residuals to lossp.
__global__ __launch_bounds__(kThreads) void mlp_backward_kernel(
    MlpDev w, const int32_t* __restrict__ comp, const float4* __restrict__ feat, const float* __restrict__ y,
    const float* __restrict__ out, const float* __restrict__ h1g, const float* __restrict__ h2g,
    const float* __restrict__ h3g, int64_t n, float scale, float* __restrict__ part, int64_t nparams,
    int64_t offA, int64_t offb1, int64_t offW2, int64_t offb2, int64_t offW3, int64_t offb3, int64_t offW4,
    int64_t offb4, float* __restrict__ lossp) {
  __shared__ float X[kT][kP];
  __shared__ float D[kT][kP];
  __shared__ float G[kT][kP];
  __shared__ int cs[kT];
  __shared__ float fs[kT][4];
  __shared__ float red[kThreads];
  const int tid = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * kT;
  const int ns = (int)std::min<int64_t>(kT, n - s0);
  const int nout = w.nout;
  float* g = part + (int64_t)blockIdx.x * nparams;
  if (tid < kT) {
    const bool ok = tid < ns;
    cs[tid] = ok ? comp[s0 + tid] : -1;
    const float4 f = ok ? feat[s0 + tid] : make_float4(0.f, 0.f, 0.f, 0.f);
    fs[tid][0] = f.x;
    fs[tid][1] = f.y;
    fs[tid][2] = f.z;
    fs[tid][3] = f.w;
  }
  float lsum = 0.0f;
  for (int o = tid; o < kT * nout; o += kThreads) {
    const int s = o / nout, j = o - s * nout;
    float r = 0.0f;
    if (s < ns) r = out[(s0 + s) * nout + j] - y[(s0 + s) * nout + j];
    D[s][j] = scale * r;
    lsum += r * r;
  }
  load_rows(X, h3g, s0, ns);
  red[tid] = lsum;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) lossp[blockIdx.x] = red[0];
  // layer 4
  grad_w(X, D, kH, nout, g + offW4);
  col_sum(D, nout, g + offb4);
  back_dense(D, nout, w.W4, nout, X, G);  // G = dZ3
  __syncthreads();
  load_rows(X, h2g, s0, ns);
  __syncthreads();
  // layer 3
  grad_w(X, G, kH, kH, g + offW3);
  col_sum(G, kH, g + offb3);
  back_dense(G, kH, w.W3, kH, X, D);  // D = dZ2
  __syncthreads();
  load_rows(X, h1g, s0, ns);
  __syncthreads();
  // layer 2
  grad_w(X, D, kH, kH, g + offW2);
  col_sum(D, kH, g + offb2);
  back_dense(D, kH, w.W2, kH, X, G);  // G = dZ1
  __syncthreads();
  // layer 1
  for (int o = tid; o < kMlpF * kH; o += kThreads) {
    const int f = o / kH, j = o - f * kH;
    float acc = 0.0f;
    for (int s = 0; s < kT; ++s) acc += fs[s][f] * G[s][j];
    g[offA + o] = acc;
  }
  col_sum(G, kH, g + offb1);
  for (int o = tid; o < w.ncomp * kH; o += kThreads) {
    const int c = o / kH, j = o - c * kH;
    float acc = 0.0f;
    for (int s = 0; s < kT; ++s)
      if (cs[s] == c) acc += G[s][j];
    g[o] = acc;  // E is the first block (offset 0)
  }
}

// grad[i] = sum over tiles of part[t][i] (fixed order: deterministic).
__global__ void reduce_partials_kernel(const float* __restrict__ part, int ntiles, int64_t nparams,
                                       float* __restrict__ grad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nparams;
       i += (int64_t)gridDim.x * blockDim.x) {
    float acc = 0.0f;
    for (int t = 0; t < ntiles; ++t) acc += part[(int64_t)t * nparams + i];
    grad[i] = acc;
  }
}

__global__ void reduce_loss_kernel(const float* __restrict__ lossp, int ntiles, double inv, double* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double acc = 0.0;
    for (int t = 0; t < ntiles; ++t) acc += (double)lossp[t];
    *dst = acc * inv;
  }
}

// Adam (Kingma & Ba): m, v moving averages; c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t).
// The weights 1 - beta come from the host, rounded once from their FP64 values
// (1 - 0.999f in FP32 would be 1.3e-5 away from 0.001).
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float beta1, float beta2, float omb1,
                            float omb2, float c1, float c2, float eps) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = beta1 * m[i] + omb1 * gi;
    const float vi = beta2 * v[i] + omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

// Minibatch by counter-based sampling with replacement from the training set.
__global__ void gather_batch_kernel(uint64_t seed, uint64_t step, int64_t ntrain, int B, int nout,
                                    const int32_t* __restrict__ comp, const float4* __restrict__ feat,
                                    const float* __restrict__ y, int32_t* __restrict__ cb,
                                    float4* __restrict__ fb, float* __restrict__ yb) {
  const int i = blockIdx.x;
  const int64_t idx = (int64_t)(rng64(seed, 1000 + step, (uint64_t)i) % (uint64_t)ntrain);
  if (threadIdx.x == 0) {
    cb[i] = comp[idx];
    fb[i] = feat[idx];
  }
  for (int j = threadIdx.x; j < nout; j += blockDim.x) yb[(int64_t)i * nout + j] = y[idx * nout + j];
}

// Glorot-uniform weights (fan-in 5 for the first layer: one-hot + 4 features),
// output layer scaled by 1/4, biases 0.
__global__ void init_kernel(float* __restrict__ p, int64_t n, int64_t offW2, int64_t offW4, int64_t offb,
                            int64_t offW3, int64_t offb3, int64_t offb4, int64_t offb2, int nout, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double u = 2.0 * ((double)(rng64(seed, 7, (uint64_t)i) >> 11) * 0x1.0p-53) - 1.0;
    double bound;
    if (i < offb) {
      bound = sqrt(6.0 / (5.0 + kH));  // E, A
    } else if ((i >= offb && i < offW2) || (i >= offb2 && i < offW3) || (i >= offb3 && i < offW4) || i >= offb4) {
      bound = 0.0;  // biases
    } else if (i >= offW4) {
      bound = 0.25 * sqrt(6.0 / (kH + nout));
    } else {
      bound = sqrt(6.0 / (2.0 * kH));
    }
    p[i] = (float)(u * bound);
  }
}

template <class T>
int alloc(T** p, size_t count) {
  FMM_HIP_TRY(hipMalloc(p, count * sizeof(T)));
  return FMMLM_OK;
}

struct Work {
  std::vector<void*> ptrs;
  template <class T>
  int get(T** p, size_t count) {
    int rc = alloc(p, std::max<size_t>(count, 1));
    if (rc == FMMLM_OK) ptrs.push_back(*p);
    return rc;
  }
  ~Work() {
    for (void* q : ptrs) hipFree(q);
  }
};

int launch_backward(const MlpNet& net, const int32_t* comp, const float* feat, const float* y, const float* out,
                    const float* h1, const float* h2, const float* h3, int64_t n, float* part, float* lossp,
                    hipStream_t st) {
  const int ntiles = (int)((n + kT - 1) / kT);
  const float scale = (float)(2.0 / ((double)n * net.nout));
  mlp_backward_kernel<<<ntiles, kThreads, 0, st>>>(dev_view(net), comp, reinterpret_cast<const float4*>(feat),
                                                   y, out, h1, h2, h3, n, scale, part, net.nparams, net.off[1],
                                                   net.off[2], net.off[3], net.off[4], net.off[5], net.off[6],
                                                   net.off[7], net.off[8], lossp);
  FMM_HIP_TRY(hipGetLastError());
  return FMMLM_OK;
}

}  // namespace

void mlp_layout(MlpNet& net) {
  const int64_t sizes[9] = {(int64_t)net.ncomp * kH, (int64_t)kMlpF * kH, kH, (int64_t)kH * kH, kH,
                            (int64_t)kH * kH, kH, (int64_t)kH * net.nout, net.nout};
  int64_t o = 0;
  for (int i = 0; i < 9; ++i) {
    net.off[i] = o;
    o += sizes[i];
  }
  net.nparams = o;
}

int gpu_mlp_forward(const MlpNet& net, const int32_t* comp, const float* feat, int64_t n, float* out, int ldo,
                    int ocols, float* h1, float* h2, float* h3, hipStream_t st) {
  if (n <= 0) return FMMLM_OK;
  if (ocols > 128 || ocols > net.nout) return FMMLM_EINVAL;
  const int64_t ntiles = (n + kT - 1) / kT;
  for (int64_t t0 = 0; t0 < ntiles; t0 += (int64_t)1 << 30) {
    const int64_t nt = std::min<int64_t>(ntiles - t0, (int64_t)1 << 30);
    const int64_t s0 = t0 * kT;
    mlp_forward_kernel<<<(unsigned)nt, kThreads, 0, st>>>(
        dev_view(net), comp + s0, reinterpret_cast<const float4*>(feat) + s0, n - s0, out + s0 * ldo, ldo,
        ocols, h1 ? h1 + s0 * kH : nullptr, h2 ? h2 + s0 * kH : nullptr, h3 ? h3 + s0 * kH : nullptr);
    FMM_HIP_TRY(hipGetLastError());
  }
  return FMMLM_OK;
}

int gpu_mlp_init(const MlpNet& net, uint64_t seed, hipStream_t st) {
  init_kernel<<<256, 256, 0, st>>>(net.params, net.nparams, net.off[3], net.off[7], net.off[2], net.off[5],
                                   net.off[6], net.off[8], net.off[4], net.nout, seed);
  FMM_HIP_TRY(hipGetLastError());
  return FMMLM_OK;
}

// One forward + backward pass over n samples (device arrays): gradient of the
// mean squared error into grad (device, nparams floats), the loss into *loss (host).
int gpu_mlp_grad(const MlpNet& net, const int32_t* comp, const float* feat, const float* y, int64_t n,
                 float* grad, double* loss, hipStream_t st) {
  if (n <= 0) return FMMLM_EINVAL;
  const int ntiles = (int)((n + kT - 1) / kT);
  Work wk;
  float *out, *h1, *h2, *h3, *part, *lossp;
  double* dl;
  int rc;
  if ((rc = wk.get(&out, (size_t)n * net.nout)) || (rc = wk.get(&h1, (size_t)n * kH)) ||
      (rc = wk.get(&h2, (size_t)n * kH)) || (rc = wk.get(&h3, (size_t)n * kH)) ||
      (rc = wk.get(&part, (size_t)ntiles * net.nparams)) || (rc = wk.get(&lossp, (size_t)ntiles)) ||
      (rc = wk.get(&dl, 1)))
    return rc;
  if ((rc = gpu_mlp_forward(net, comp, feat, n, out, net.nout, net.nout, h1, h2, h3, st))) return rc;
  if ((rc = launch_backward(net, comp, feat, y, out, h1, h2, h3, n, part, lossp, st))) return rc;
  reduce_partials_kernel<<<256, 256, 0, st>>>(part, ntiles, net.nparams, grad);
  FMM_HIP_TRY(hipGetLastError());
  reduce_loss_kernel<<<1, 64, 0, st>>>(lossp, ntiles, 1.0 / ((double)n * net.nout), dl);
  FMM_HIP_TRY(hipGetLastError());
  FMM_HIP_TRY(hipMemcpyAsync(loss, dl, sizeof(double), hipMemcpyDeviceToHost, st));
  FMM_HIP_TRY(hipStreamSynchronize(st));
  return FMMLM_OK;
}

// nsteps Adam steps t = 1..nsteps from zero moments with the given gradients
// (device, [nsteps][nparams]) and learning rates (host), through the training
// kernel; the parameters after each step go to trace (device, [nsteps][nparams])
// when it is not null.
int gpu_mlp_adam_steps(const MlpNet& net, int nsteps, const float* grads, const double* lr, float* trace,
                       hipStream_t st) {
  if (nsteps < 1) return FMMLM_EINVAL;
  Work wk;
  float *m, *v;
  int rc;
  if ((rc = wk.get(&m, net.nparams)) || (rc = wk.get(&v, net.nparams))) return rc;
  FMM_HIP_TRY(hipMemsetAsync(m, 0, net.nparams * sizeof(float), st));
  FMM_HIP_TRY(hipMemsetAsync(v, 0, net.nparams * sizeof(float), st));
  const double beta1 = 0.9, beta2 = 0.999;
  for (int t = 1; t <= nsteps; ++t) {
    adam_kernel<<<256, 256, 0, st>>>(net.params, grads + (int64_t)(t - 1) * net.nparams, m, v, net.nparams,
                                     (float)lr[t - 1], (float)beta1, (float)beta2,
                                     (float)(1.0 - beta1), (float)(1.0 - beta2),
                                     (float)(1.0 / (1.0 - std::pow(beta1, t))),
                                     (float)(1.0 / (1.0 - std::pow(beta2, t))), 1e-8f);
    FMM_HIP_TRY(hipGetLastError());
    if (trace)
      FMM_HIP_TRY(hipMemcpyAsync(trace + (int64_t)(t - 1) * net.nparams, net.params, net.nparams * sizeof(float),
                                 hipMemcpyDeviceToDevice, st));
  }
  FMM_HIP_TRY(hipStreamSynchronize(st));
  return FMMLM_OK;
}

// Adam over `steps` minibatches of B samples drawn from the n training samples.
// Learning rate: linear warm-up over the first 2% of the steps, then cosine
// decay from lr to lr/100.  Mean minibatch loss of the first and last 2% of
// the steps into loss_first / loss_last.
int gpu_mlp_train(const MlpNet& net, const int32_t* comp, const float* feat, const float* y, int64_t n,
                  int steps, int B, double lr, uint64_t seed, double* loss_first, double* loss_last,
                  hipStream_t st) {
  if (n <= 0 || steps < 0 || B < kT || B % kT) return FMMLM_EINVAL;
  const int ntiles = B / kT;
  Work wk;
  int32_t* cb;
  float *fb, *yb, *out, *h1, *h2, *h3, *part, *lossp, *grad, *m, *v;
  double* hist;
  int rc;
  if ((rc = wk.get(&cb, B)) || (rc = wk.get(&fb, (size_t)B * 4)) || (rc = wk.get(&yb, (size_t)B * net.nout)) ||
      (rc = wk.get(&out, (size_t)B * net.nout)) || (rc = wk.get(&h1, (size_t)B * kH)) ||
      (rc = wk.get(&h2, (size_t)B * kH)) || (rc = wk.get(&h3, (size_t)B * kH)) ||
      (rc = wk.get(&part, (size_t)ntiles * net.nparams)) || (rc = wk.get(&lossp, ntiles)) ||
      (rc = wk.get(&grad, net.nparams)) || (rc = wk.get(&m, net.nparams)) || (rc = wk.get(&v, net.nparams)) ||
      (rc = wk.get(&hist, std::max(steps, 1))))
    return rc;
  FMM_HIP_TRY(hipMemsetAsync(m, 0, net.nparams * sizeof(float), st));
  FMM_HIP_TRY(hipMemsetAsync(v, 0, net.nparams * sizeof(float), st));
  const double beta1 = 0.9, beta2 = 0.999;
  const int warm = std::max(1, steps / 50);
  for (int t = 1; t <= steps; ++t) {
    double lrt;
    if (t <= warm) {
      lrt = lr * t / warm;
    } else {
      const double x = (double)(t - warm) / std::max(1, steps - warm);
      lrt = lr * (0.01 + 0.99 * 0.5 * (1.0 + std::cos(M_PI * x)));
    }
    gather_batch_kernel<<<B, 64, 0, st>>>(seed, (uint64_t)t, n, B, net.nout, comp,
                                          reinterpret_cast<const float4*>(feat), y, cb,
                                          reinterpret_cast<float4*>(fb), yb);
    FMM_HIP_TRY(hipGetLastError());
    if ((rc = gpu_mlp_forward(net, cb, fb, B, out, net.nout, net.nout, h1, h2, h3, st))) return rc;
    if ((rc = launch_backward(net, cb, fb, yb, out, h1, h2, h3, B, part, lossp, st))) return rc;
    reduce_partials_kernel<<<256, 256, 0, st>>>(part, ntiles, net.nparams, grad);
    reduce_loss_kernel<<<1, 64, 0, st>>>(lossp, ntiles, 1.0 / ((double)B * net.nout), hist + (t - 1));
    adam_kernel<<<256, 256, 0, st>>>(net.params, grad, m, v, net.nparams, (float)lrt, (float)beta1,
                                     (float)beta2, (float)(1.0 - beta1), (float)(1.0 - beta2),
                                     (float)(1.0 / (1.0 - std::pow(beta1, t))),
                                     (float)(1.0 / (1.0 - std::pow(beta2, t))), 1e-8f);
    FMM_HIP_TRY(hipGetLastError());
  }
  std::vector<double> h(std::max(steps, 1), 0.0);
  if (steps > 0) FMM_HIP_TRY(hipMemcpyAsync(h.data(), hist, steps * sizeof(double), hipMemcpyDeviceToHost, st));
  FMM_HIP_TRY(hipStreamSynchronize(st));
  const int k = std::max(1, steps / 50);
  double a = 0.0, b = 0.0;
  for (int i = 0; i < std::min(k, steps); ++i) {
    a += h[i];
    b += h[steps - 1 - i];
  }
  *loss_first = steps ? a / std::min(k, steps) : 0.0;
  *loss_last = steps ? b / std::min(k, steps) : 0.0;
  return FMMLM_OK;
}

}  // namespace fmmlm
