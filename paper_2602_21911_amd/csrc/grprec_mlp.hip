// grprec_mlp.hip -- exact Riemann problems in bulk and the learned
// star-pressure proposal (float32 network 6-32-32-1, tanh): features,
// inference, loss gradient and Adam, all on the GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/grprec.h"
#include "grprec_device.h"
#include "grprec_internal.h"

using namespace grp;

namespace {

Gas gas_of(double g) { return make_gas(g); }

int grid_for(long long n, int block, int cap) {
  long long g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

__global__ void riemann_batch_kernel(const double *wl, const double *wr, long long n, Gas G, int guess,
                                     const float *mlp, double gate, double tol, int maxit, double *pstar,
                                     int *iters) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double rl = wl[3 * i], ul = wl[3 * i + 1], pl = wl[3 * i + 2];
    const double rr = wr[3 * i], ur = wr[3 * i + 1], pr = wr[3 * i + 2];
    bool ok = rl > 0.0 && rr > 0.0 && pl > 0.0 && pr > 0.0 && isfinite(ul) && isfinite(ur) &&
              isfinite(rl) && isfinite(rr) && isfinite(pl) && isfinite(pr);
    int code = 0;
    double ps = __longlong_as_double(0x7ff8000000000000ll);
    if (!ok) {
      code = GRPREC_E_NONPHYSICAL;
    } else {
      Prim L, R;
      prim_from(G, rl, ul, pl, L);
      prim_from(G, rr, ur, pr, R);
      if (G.two_gm1 * (L.c + R.c) <= R.u - L.u) {
        code = GRPREC_E_VACUUM;
      } else {
        bool used;
        double p0 = start_pressure(G, L, R, guess, gate, mlp, used);
        double us, pp;
        Side sl, sr;
        int it = newton_pstar(G, L, R, p0, maxit, tol, pp, us, sl, sr);
        if (it > maxit) code = GRPREC_E_NEWTON;
        else { ps = pp; code = it; }
      }
    }
    if (pstar) pstar[i] = ps;
    if (iters) iters[i] = code;
  }
}

__global__ void features_kernel(const double *wl, const double *wr, const double *pstar, long long n, Gas G,
                                float *x, float *y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    Prim L, R;
    L.r = wl[3 * i]; L.u = wl[3 * i + 1]; L.p = wl[3 * i + 2];
    R.r = wr[3 * i]; R.u = wr[3 * i + 1]; R.p = wr[3 * i + 2];
    float f[6];
    double pbar;
    mlp_features(G.g, L.r, L.u, L.p, R.r, R.u, R.p, f, pbar);
#pragma unroll
    for (int k = 0; k < 6; ++k) x[6 * i + k] = f[k];
    if (pstar && y) y[i] = (float)log(pstar[i] / pbar);
  }
}

__global__ void forward_kernel(const float *P, const float *x, float *y, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    float f[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) f[k] = x[6 * i + k];
    y[i] = mlp_eval(P, f);
  }
}

// Backward pass.  Block of 64 samples (one per thread): forward and
// backward per sample in registers; the per-sample outer products are then
// summed over the block from LDS, one group of parameters per thread, and
// written as this block's partial sums (deterministic, no atomics).
// LOSS: t holds targets, the upstream gradient is dy = 2 (y - t) / n and the
// last partial is the block's share of the mean squared error; otherwise t
// holds dy itself and the last partial is 0.
constexpr int GB = 64;
constexpr int NW = GRPREC_MLP_WEIGHTS;

template <bool LOSS>
__global__ __launch_bounds__(GB) void grad_partial(const float *P, const float *xin, const float *t,
                                                   long long n, float inv_n, float *partial) {
  __shared__ float sx[6][GB];
  __shared__ float sh1[32][GB];
  __shared__ float sh2[32][GB];
  __shared__ float sd1[32][GB];
  __shared__ float sd2[32][GB];
  __shared__ float sdy[GB];
  __shared__ float sloss[GB];
  const float *W1 = P, *b1 = P + 192, *W2 = P + 224, *b2 = P + 1248, *W3 = P + 1280, *b3 = P + 1312;
  const float *mean = P + 1313, *stdv = P + 1319;
  const int e = threadIdx.x;
  const long long i = blockIdx.x * (long long)GB + e;
  const bool live = i < n;
  float x[6], h1[32], h2[32];
#pragma unroll
  for (int k = 0; k < 6; ++k) x[k] = live ? (xin[6 * i + k] - mean[k]) / stdv[k] : 0.0f;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    float a = b1[j];
#pragma unroll
    for (int k = 0; k < 6; ++k) a = fmaf(W1[j * 6 + k], x[k], a);
    h1[j] = mlp_tanh(a);
  }
  float y = b3[0];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    float a = b2[j];
#pragma unroll
    for (int k = 0; k < 32; ++k) a = fmaf(W2[j * 32 + k], h1[k], a);
    h2[j] = mlp_tanh(a);
    y = fmaf(W3[j], h2[j], y);
  }
  const float r = (LOSS && live) ? y - t[i] : 0.0f;
  const float dy = LOSS ? 2.0f * r * inv_n : (live ? t[i] : 0.0f);
  float d2[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) d2[j] = dy * W3[j] * (1.0f - h2[j] * h2[j]);
  float d1[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    float a = 0.0f;
#pragma unroll
    for (int j = 0; j < 32; ++j) a = fmaf(W2[j * 32 + k], d2[j], a);
    d1[k] = a * (1.0f - h1[k] * h1[k]);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) sx[k][e] = x[k];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    sh1[j][e] = h1[j];
    sh2[j][e] = h2[j];
    sd1[j][e] = d1[j];
    sd2[j][e] = d2[j];
  }
  sdy[e] = dy;
  sloss[e] = r * r * inv_n;
  __syncthreads();
  float *out = partial + (long long)blockIdx.x * (NW + 1);
  for (int p = e; p < NW + 1; p += GB) {
    float acc = 0.0f;
    if (p < 192) {  // W1[j][k] += d1_j x_k
      const int j = p / 6, k = p % 6;
      for (int s = 0; s < GB; ++s) acc = fmaf(sd1[j][s], sx[k][s], acc);
    } else if (p < 224) {  // b1
      const int j = p - 192;
      for (int s = 0; s < GB; ++s) acc += sd1[j][s];
    } else if (p < 1248) {  // W2[j][k] += d2_j h1_k
      const int j = (p - 224) / 32, k = (p - 224) % 32;
      for (int s = 0; s < GB; ++s) acc = fmaf(sd2[j][s], sh1[k][s], acc);
    } else if (p < 1280) {  // b2
      const int j = p - 1248;
      for (int s = 0; s < GB; ++s) acc += sd2[j][s];
    } else if (p < 1312) {  // W3[j] += dy h2_j
      const int j = p - 1280;
      for (int s = 0; s < GB; ++s) acc = fmaf(sdy[s], sh2[j][s], acc);
    } else if (p < 1313) {  // b3
      for (int s = 0; s < GB; ++s) acc += sdy[s];
    } else {  // loss
      for (int s = 0; s < GB; ++s) acc += sloss[s];
    }
    out[p] = acc;
  }
}

__global__ void reduce_partials(const float *partial, int nblocks, float *grad, float *loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > NW) return;
  float acc = 0.0f;
  for (int b = 0; b < nblocks; ++b) acc += partial[(long long)b * (NW + 1) + p];
  if (p < NW) grad[p] = acc;
  else if (loss) loss[0] = acc;
}

__global__ void adam_kernel(float *P, const float *g, float *m, float *v, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NW) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.0f - b1) * gp;
  const float vp = b2 * v[p] + (1.0f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  P[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

// Both passes of the gradient: per-block partial sums into `partial`
// (nb x (NW + 1) floats), then their sum over the blocks.
int gradient(bool with_loss, const float *params, const float *x, const float *t, int64_t n, float *grad,
             float *loss, float *partial, hipStream_t st) {
  const int nb = (int)((n + GB - 1) / GB);
  if (with_loss)
    hipLaunchKernelGGL(grad_partial<true>, dim3(nb), dim3(GB), 0, st, params, x, t, (long long)n,
                       1.0f / (float)n, partial);
  else
    hipLaunchKernelGGL(grad_partial<false>, dim3(nb), dim3(GB), 0, st, params, x, t, (long long)n, 0.0f,
                       partial);
  if (hipGetLastError() != hipSuccess) return GRPREC_E_HIP;
  hipLaunchKernelGGL(reduce_partials, dim3((NW + 1 + 255) / 256), dim3(256), 0, st, (const float *)partial,
                     nb, grad, loss);
  return hipGetLastError() == hipSuccess ? GRPREC_OK : GRPREC_E_HIP;
}
// Partial sums of grprec_mlp_backward_noalloc, in a fixed device array
// instead of caller workspace: room for kNoAllocBlocks blocks of GB samples
// (5.1 MiB, held on every device the library runs on until the process ends).
// Host code never passes the array's name to a kernel: the name is a host-side
// stand-in, and each device's copy has its own address, looked up once per
// device with hipGetSymbolAddress.
constexpr int kNoAllocBlocks = 1024;
__device__ __align__(256) float scratch[(size_t)kNoAllocBlocks * (NW + 1)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device, with it current).
int scratch_of_current_device(float **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GRPREC_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return GRPREC_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GRPREC_E_HIP;
    g_scratch[dev] = (float *)p;
  }
  *out = g_scratch[dev];
  return GRPREC_OK;
}

}  // namespace

extern "C" {

int grprec_riemann_batch(const double *wl, const double *wr, int64_t n, double gamma, int guess,
                         const float *mlp_params, double gate, double tol, int max_iter, double *pstar,
                         int *iters, void *hip_stream) {
  if (n < 0 || (n > 0 && (!wl || !wr)) || !(gamma > 1.0) || max_iter < 1 || !(tol > 0.0))
    return GRPREC_E_INVALID;
  if (guess == GRPREC_GUESS_MLP && !mlp_params) return GRPREC_E_INVALID;
  if (n == 0) return GRPREC_OK;
  hipLaunchKernelGGL(riemann_batch_kernel, dim3(grid_for(n, 256, 65536)), dim3(256), 0,
                     (hipStream_t)hip_stream, wl, wr, (long long)n, gas_of(gamma), guess, mlp_params, gate,
                     tol, max_iter, pstar, iters);
  return hipGetLastError() == hipSuccess ? GRPREC_OK : GRPREC_E_HIP;
}

int grprec_mlp_features(const double *wl, const double *wr, const double *pstar, int64_t n, double gamma,
                        float *x, float *y, void *hip_stream) {
  if (n < 0 || (n > 0 && (!wl || !wr || !x)) || !(gamma > 1.0)) return GRPREC_E_INVALID;
  if (pstar && !y) return GRPREC_E_INVALID;
  if (n == 0) return GRPREC_OK;
  hipLaunchKernelGGL(features_kernel, dim3(grid_for(n, 256, 65536)), dim3(256), 0, (hipStream_t)hip_stream,
                     wl, wr, pstar, (long long)n, gas_of(gamma), x, y);
  return hipGetLastError() == hipSuccess ? GRPREC_OK : GRPREC_E_HIP;
}

int grprec_mlp_forward(const float *params, const float *x, float *y, int64_t n, void *hip_stream) {
  if (!params || n < 0 || (n > 0 && (!x || !y))) return GRPREC_E_INVALID;
  if (n == 0) return GRPREC_OK;
  hipLaunchKernelGGL(forward_kernel, dim3(grid_for(n, 256, 65536)), dim3(256), 0, (hipStream_t)hip_stream,
                     params, x, y, (long long)n);
  return hipGetLastError() == hipSuccess ? GRPREC_OK : GRPREC_E_HIP;
}

size_t grprec_mlp_work_bytes(int64_t n) {
  if (n < 1) return 0;
  long long nb = (n + GB - 1) / GB;
  return sizeof(float) * (size_t)nb * (NW + 1);
}

int grprec_mlp_backward(const float *params, const float *x, const float *dy, float *grad, int64_t n,
                        void *work, void *hip_stream) {
  if (!params || !x || !dy || n < 1 || !grad || !work) return GRPREC_E_INVALID;
  if (n > (int64_t)GB * 1048576) return GRPREC_E_INVALID;
  return gradient(false, params, x, dy, n, grad, nullptr, (float *)work, (hipStream_t)hip_stream);
}

int grprec_mlp_backward_noalloc(const float *params, const float *x, const float *dy, float *grad, int64_t n,
                                void *hip_stream) {
  if (!params || !x || !dy || n < 1 || !grad) return GRPREC_E_INVALID;
  if (n > (int64_t)GB * kNoAllocBlocks) return GRPREC_E_INVALID;
  float *partial = nullptr;
  const int rc = scratch_of_current_device(&partial);
  if (rc != GRPREC_OK) return rc;
  return gradient(false, params, x, dy, n, grad, nullptr, partial, (hipStream_t)hip_stream);
}

int grprec_mlp_loss_grad(const float *params, const float *x, const float *y, int64_t n, float *grad,
                         float *loss, void *work, void *hip_stream) {
  if (!params || !x || !y || n < 1 || !grad || !work) return GRPREC_E_INVALID;
  if (n > (int64_t)GB * 1048576) return GRPREC_E_INVALID;
  return gradient(true, params, x, y, n, grad, loss, (float *)work, (hipStream_t)hip_stream);
}

int grprec_mlp_adam(float *params, const float *grad, float *m, float *v, int step, float lr, float beta1,
                    float beta2, float eps, void *hip_stream) {
  if (!params || !grad || !m || !v || step < 1) return GRPREC_E_INVALID;
  const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((NW + 255) / 256), dim3(256), 0, (hipStream_t)hip_stream, params, grad,
                     m, v, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? GRPREC_OK : GRPREC_E_HIP;
}

}  // extern "C"
