// Restarted GMRES around the layered-media FMM matvec: the iterative solve of a
// dense system whose product is the layered-media potential, the application
// the method is built for (Sec. 1).  GMRES as defined by Saad & Schultz (1986):
// Arnoldi (here classical Gram-Schmidt applied twice), Givens rotations for the
// Hessenberg least-squares problem, restart after `restart` steps.
//
// Device work per Arnoldi step k: one plan evaluation (v_{k+1} = G v_k, plus the
// diagonal), two Gram-Schmidt passes (k + 1 dot products in one launch, then
// v_{k+1} -= V h), the norm and the scaling, all FP64 with fixed-order
// reductions (slices of the vector summed in a fixed tree).  The host reads the
// k + 2 Hessenberg entries once per step and applies the rotations.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "fmm_internal.h"

namespace fmmlm {
namespace {

constexpr int kSolveThreads = 256;
constexpr int kDotSlices = 256;  // blocks per dot product (one partial each)
constexpr int kMaxRestart = 256;
static_assert(kDotSlices == kSolveThreads, "the finishing block sums one partial per thread");

// Tree sum of the block's values in LDS (fixed order); result in red[0].
__device__ inline void block_tree_sum(double* red) {
  for (int h = kSolveThreads / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
}

// partial[j][s] = sum over slice s of V_j[i] w[i], for j = blockIdx.y
__global__ void __launch_bounds__(kSolveThreads)
gm_dots_partial_kernel(int64_t n, const double* __restrict__ V, int64_t ldv, const double* __restrict__ w,
                       double* __restrict__ partial) {
  __shared__ double red[kSolveThreads];
  const int s = blockIdx.x, j = blockIdx.y;
  const int64_t per = (n + kDotSlices - 1) / kDotSlices;
  const int64_t i0 = (int64_t)s * per;
  const int64_t i1 = std::min(n, i0 + per);
  const double* v = V + (int64_t)j * ldv;
  double acc = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kSolveThreads) acc = fma(v[i], w[i], acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  block_tree_sum(red);
  if (threadIdx.x == 0) partial[(int64_t)j * kDotSlices + s] = red[0];
}

// out[j] = sum_s partial[j][s]; one block per j
__global__ void __launch_bounds__(kSolveThreads)
gm_dots_finish_kernel(const double* __restrict__ partial, double* __restrict__ out) {
  __shared__ double red[kSolveThreads];
  red[threadIdx.x] = partial[(int64_t)blockIdx.x * kDotSlices + threadIdx.x];
  __syncthreads();
  block_tree_sum(red);
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// w[i] += sign * sum_{j < k} c[j] V_j[i]   (c on the device)
__global__ void __launch_bounds__(kSolveThreads)
gm_combine_kernel(int64_t n, int k, const double* __restrict__ V, int64_t ldv, const double* __restrict__ c,
                  double sign, double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * kSolveThreads + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int j = 0; j < k; ++j) acc = fma(c[j], V[(int64_t)j * ldv + i], acc);
  w[i] = fma(sign, acc, w[i]);
}

// w[i] *= 1 / sqrt(*nrm2) when *nrm2 > 0 (otherwise w is the zero vector)
__global__ void __launch_bounds__(kSolveThreads)
gm_scale_kernel(int64_t n, const double* __restrict__ nrm2, double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * kSolveThreads + threadIdx.x;
  const double s = *nrm2;
  if (i >= n || !(s > 0.0)) return;
  w[i] = w[i] / sqrt(s);
}

// w[i] += diag[i] v[i]
__global__ void __launch_bounds__(kSolveThreads)
gm_diag_kernel(int64_t n, const double* __restrict__ diag, const double* __restrict__ v, double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * kSolveThreads + threadIdx.x;
  if (i < n) w[i] = fma(diag[i], v[i], w[i]);
}

// r[i] = b[i] - r[i]   (r holds A x on entry)
__global__ void __launch_bounds__(kSolveThreads)
gm_residual_kernel(int64_t n, const double* __restrict__ b, double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * kSolveThreads + threadIdx.x;
  if (i < n) r[i] = b[i] - r[i];
}

__global__ void __launch_bounds__(kSolveThreads)
gm_fill_kernel(int64_t n, double v, double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * kSolveThreads + threadIdx.x;
  if (i < n) w[i] = v;
}

// Device buffers of one call, freed on every exit.
struct GmresWork {
  double* V = nullptr;        // [restart + 1][n] Krylov basis
  double* partial = nullptr;  // [restart + 2][kDotSlices]
  double* small = nullptr;    // h1 [restart + 2] | h2 [restart + 2] | nrm2 | y [restart]
  ~GmresWork() {
    if (V) (void)hipFree(V);
    if (partial) (void)hipFree(partial);
    if (small) (void)hipFree(small);
  }
};

}  // namespace
}  // namespace fmmlm

using namespace fmmlm;

extern "C" int fmm_layered_solve(fmmlm_plan_t plan, const double* diag, const double* b, double* x,
                                 const fmmlm_solve_opts* opts, void* hip_stream, fmmlm_solve_info* info) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!plan || !b || !x || !info) return FMMLM_EINVAL;
  fmmlm_solve_opts o{30, 300, 1e-6, 0, 0};
  if (opts) o = *opts;
  if (o.restart < 1 || o.restart > kMaxRestart || o.max_iters < 1 || !(o.tol > 0.0 && o.tol < 1.0))
    return FMMLM_EINVAL;
  const int64_t n = plan->N;
  if (x < b + n && b < x + n) return FMMLM_EINVAL;  // x must not overlap b
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (int rc = plan_acquire(plan, st)) return rc;
  // every step synchronises st, so the plan is free again when the call returns
  struct Hold {
    fmmlm_plan_s* P;
    hipStream_t st;
    ~Hold() { plan_release(P, st, false); }
  } hold{plan, st};
  *info = fmmlm_solve_info{0, 0, 0, 0, 0.0, 0.0, 0.0};
  const int m = o.restart;
  const int64_t ldv = n;
  GmresWork wk;
  if (hipMalloc(&wk.V, sizeof(double) * (size_t)(m + 1) * (size_t)n) != hipSuccess ||
      hipMalloc(&wk.partial, sizeof(double) * (size_t)(m + 2) * kDotSlices) != hipSuccess ||
      hipMalloc(&wk.small, sizeof(double) * (size_t)(3 * m + 5)) != hipSuccess) {
    set_last_error("fmm_layered_solve: workspace allocation failed");
    return FMMLM_ENOMEM;
  }
  double* h1 = wk.small;
  double* h2 = wk.small + (m + 2);
  double* nrm2 = wk.small + 2 * (m + 2);
  double* yd = nrm2 + 1;
  auto V = [&](int j) { return wk.V + (int64_t)j * ldv; };
  const unsigned nb = (unsigned)((n + kSolveThreads - 1) / kSolveThreads);
  // dots of V_0..V_{k-1} with w into out[0..k)
  auto dots = [&](const double* Vs, int k, const double* w, double* out) {
    gm_dots_partial_kernel<<<dim3(kDotSlices, (unsigned)k), kSolveThreads, 0, st>>>(n, Vs, ldv, w, wk.partial);
    gm_dots_finish_kernel<<<(unsigned)k, kSolveThreads, 0, st>>>(wk.partial, out);
  };
  auto read_scalar = [&](const double* dptr, double* h) -> int {
    FMM_HIP_TRY(hipMemcpyAsync(h, dptr, sizeof(double), hipMemcpyDeviceToHost, st));
    FMM_HIP_TRY(hipStreamSynchronize(st));
    return FMMLM_OK;
  };
  // G v + diag v into w
  auto matvec = [&](const double* v, double* w) -> int {
    if (int rc = eval_held(plan, 1, v, n, w, n, FMMLM_FREE | FMMLM_REACTION, st)) return rc;
    if (diag) gm_diag_kernel<<<nb, kSolveThreads, 0, st>>>(n, diag, v, w);
    info->matvecs++;
    return FMMLM_OK;
  };
  // r = b - A x into V_0, and its squared norm into *nrm2
  auto residual = [&]() -> int {
    if (int rc = matvec(x, V(0))) return rc;
    gm_residual_kernel<<<nb, kSolveThreads, 0, st>>>(n, b, V(0));
    dots(V(0), 1, V(0), nrm2);
    return FMMLM_OK;
  };

  double bn2 = 0.0;
  dots(b, 1, b, nrm2);
  if (int rc = read_scalar(nrm2, &bn2)) return rc;
  const double bn = std::sqrt(bn2);
  if (!(bn > 0.0)) {
    // b = 0: x = 0 solves it exactly
    gm_fill_kernel<<<nb, kSolveThreads, 0, st>>>(n, 0.0, x);
    FMM_HIP_TRY(hipStreamSynchronize(st));
    info->converged = 1;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return FMMLM_OK;
  }
  double beta2 = 0.0;
  if (o.zero_guess) {
    gm_fill_kernel<<<nb, kSolveThreads, 0, st>>>(n, 0.0, x);
    FMM_HIP_TRY(hipMemcpyAsync(V(0), b, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, st));
    FMM_HIP_TRY(hipMemcpyAsync(nrm2, &bn2, sizeof(double), hipMemcpyHostToDevice, st));
    beta2 = bn2;
  } else {
    if (int rc = residual()) return rc;
    if (int rc = read_scalar(nrm2, &beta2)) return rc;
  }
  double relres = std::sqrt(beta2) / bn;

  // Hessenberg columns after rotation (upper triangle R), rotations, rhs g
  std::vector<double> R((size_t)m * m, 0.0), cs(m), sn(m), g(m + 1), col(m + 2), hh(2 * (m + 2) + 1), y(m);
  while (relres > o.tol && info->iters < o.max_iters) {
    info->cycles++;
    const double beta = std::sqrt(beta2);
    gm_scale_kernel<<<nb, kSolveThreads, 0, st>>>(n, nrm2, V(0));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int kk = 0;
    for (int k = 0; k < m && info->iters < o.max_iters; ++k) {
      if (int rc = matvec(V(k), V(k + 1))) return rc;
      info->iters++;
      // classical Gram-Schmidt, twice
      dots(V(0), k + 1, V(k + 1), h1);
      gm_combine_kernel<<<nb, kSolveThreads, 0, st>>>(n, k + 1, V(0), ldv, h1, -1.0, V(k + 1));
      dots(V(0), k + 1, V(k + 1), h2);
      gm_combine_kernel<<<nb, kSolveThreads, 0, st>>>(n, k + 1, V(0), ldv, h2, -1.0, V(k + 1));
      dots(V(k + 1), 1, V(k + 1), nrm2);
      gm_scale_kernel<<<nb, kSolveThreads, 0, st>>>(n, nrm2, V(k + 1));
      FMM_HIP_TRY(hipGetLastError());
      FMM_HIP_TRY(hipMemcpyAsync(hh.data(), wk.small, sizeof(double) * (2 * (m + 2) + 1), hipMemcpyDeviceToHost, st));
      FMM_HIP_TRY(hipStreamSynchronize(st));
      for (int j = 0; j <= k; ++j) col[j] = hh[j] + hh[(m + 2) + j];
      const double hnext = std::sqrt(hh[2 * (m + 2)]);
      // previous rotations, then the one that zeroes the subdiagonal entry
      for (int j = 0; j < k; ++j) {
        const double a = col[j], c = col[j + 1];
        col[j] = cs[j] * a + sn[j] * c;
        col[j + 1] = -sn[j] * a + cs[j] * c;
      }
      const double den = std::hypot(col[k], hnext);
      if (den > 0.0) {
        cs[k] = col[k] / den;
        sn[k] = hnext / den;
      } else {
        cs[k] = 1.0;
        sn[k] = 0.0;
      }
      col[k] = den;
      g[k + 1] = -sn[k] * g[k];
      g[k] = cs[k] * g[k];
      for (int j = 0; j <= k; ++j) R[(size_t)j * m + k] = col[j];
      kk = k + 1;
      info->relres_est = std::fabs(g[k + 1]) / bn;
      if (info->relres_est <= o.tol || !(hnext > 0.0)) break;
    }
    // y = R^{-1} g (back substitution), x += V y
    for (int i = kk - 1; i >= 0; --i) {
      double s = g[i];
      for (int j = i + 1; j < kk; ++j) s -= R[(size_t)i * m + j] * y[j];
      const double rii = R[(size_t)i * m + i];
      y[i] = rii != 0.0 ? s / rii : 0.0;
    }
    FMM_HIP_TRY(hipMemcpyAsync(yd, y.data(), sizeof(double) * kk, hipMemcpyHostToDevice, st));
    gm_combine_kernel<<<nb, kSolveThreads, 0, st>>>(n, kk, V(0), ldv, yd, 1.0, x);
    // the true residual decides convergence and restarts the next cycle
    if (int rc = residual()) return rc;
    if (int rc = read_scalar(nrm2, &beta2)) return rc;
    relres = std::sqrt(beta2) / bn;
  }
  FMM_HIP_TRY(hipGetLastError());
  FMM_HIP_TRY(hipStreamSynchronize(st));
  info->relres = relres;
  info->converged = relres <= o.tol ? 1 : 0;
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  return FMMLM_OK;
}
