// Learned bin-width allocation: per-level statistics, a small MLP (forward,
// backward, Adam) and the L-infinity check (gfx950).
//
// This part is a project addition (the paper defines no learned component).
// The network maps four features of a level's coefficients to a log-scale
// factor theta_l of that level's bin width:
//   features: log(rms/tau), log(max/tau), log(count / stream length), l/L,
//             normalised by a per-feature mean and standard deviation stored
//             with the weights;
//   layers:   Linear(4,64) - ReLU - Linear(64,64) - ReLU - Linear(64,1).
// Parameter buffer (float32): mean[4], std[4], W1[64][4], b1[64],
// W2[64][64], b2[64], W3[64], b3[1]; y = x W^T + b.  All sums run in a fixed
// order (one thread per output, inputs or batch rows in index order), so
// results are reproducible.  Plain FMA-free float arithmetic; no matrix cores
// (the layers are 64 wide and run on a few hundred rows).
#include <cfloat>

#include "internal.hpp"

namespace mg {

namespace {
constexpr int TPB = 256;
constexpr int F = MLP_IN, H = MLP_HID;

inline unsigned grid_for(uint64_t n, unsigned cap = 4096) {
  uint64_t g = (n + TPB - 1) / TPB;
  if (g < 1) g = 1;
  return (unsigned)std::min<uint64_t>(g, cap);
}

// ------------------------------------------------------------ level stats
// stats[3l+0] = count, [3l+1] = sum of squares (float64), [3l+2] = max |c|.
// Pass 1: per block partial sums per level; pass 2: one thread per level sums
// the partials in block order.
template <typename T>
__global__ void __launch_bounds__(TPB) k_stats_partial(const T* __restrict__ c, const uint64_t* __restrict__ off,
                                                       int nlev, double* __restrict__ part, int nblocks_per_level) {
  const int l = blockIdx.x / nblocks_per_level;
  const int b = blockIdx.x % nblocks_per_level;
  const uint64_t beg = off[l], end = off[l + 1];
  double ss = 0.0, mx = 0.0;
  for (uint64_t i = beg + (uint64_t)b * TPB + threadIdx.x; i < end; i += (uint64_t)nblocks_per_level * TPB) {
    const double v = (double)c[i];
    ss += v * v;
    const double a = fabs(v);
    mx = a > mx ? a : mx;
  }
  __shared__ double rs[TPB], rm[TPB];
  rs[threadIdx.x] = ss;
  rm[threadIdx.x] = mx;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      rs[threadIdx.x] += rs[threadIdx.x + s];
      rm[threadIdx.x] = rm[threadIdx.x] > rm[threadIdx.x + s] ? rm[threadIdx.x] : rm[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = rs[0];
    part[2 * blockIdx.x + 1] = rm[0];
  }
}

__global__ void k_stats_final(const double* __restrict__ part, const uint64_t* __restrict__ off, int nlev,
                              int nblocks_per_level, double* __restrict__ stats) {
  const int l = threadIdx.x;
  if (l >= nlev) return;
  double ss = 0.0, mx = 0.0;
  for (int b = 0; b < nblocks_per_level; ++b) {
    ss += part[2 * (l * nblocks_per_level + b)];
    const double m = part[2 * (l * nblocks_per_level + b) + 1];
    mx = m > mx ? m : mx;
  }
  stats[3 * l] = (double)(off[l + 1] - off[l]);
  stats[3 * l + 1] = ss;
  stats[3 * l + 2] = mx;
}

// features of every level from the stats and tau (scalars[0]); normalised by
// the mean and standard deviation in params, or raw when params is null
__global__ void k_features(const double* __restrict__ stats, const double* __restrict__ scalars, int nlev,
                           const float* __restrict__ params, float* __restrict__ x) {
  const int l = threadIdx.x;
  if (l >= nlev) return;
  const double tau = scalars[0] > 0.0 ? scalars[0] : 1.0;
  double total = 0.0;
  for (int k = 0; k < nlev; ++k) total += stats[3 * k];
  total = total > 0.0 ? total : 1.0;
  const double cnt = stats[3 * l];
  const double rms = sqrt(stats[3 * l + 1] / (cnt > 0.0 ? cnt : 1.0));
  const double mx = stats[3 * l + 2];
  double f[F];
  f[0] = log(rms / tau + 1e-30);
  f[1] = log(mx / tau + 1e-30);
  f[2] = log((cnt > 0.0 ? cnt : 1.0) / total);  // the level's share of the stream: independent of the field size
  f[3] = nlev > 1 ? (double)l / (double)(nlev - 1) : 0.0;
  for (int i = 0; i < F; ++i)
    x[l * F + i] = params ? (float)((f[i] - (double)params[i]) / (double)params[F + i]) : (float)f[i];
}

// bins[l] = plain * exp(clamp(theta_l)); written to learned[], plain kept in bins[]
__global__ void k_apply_theta(const double* __restrict__ bins, const float* __restrict__ theta, int nlev,
                              double scale, double* __restrict__ learned) {
  const int l = threadIdx.x;
  if (l >= nlev) return;
  double t = (double)theta[l];
  t = t < -3.0 ? -3.0 : (t > 5.0 ? 5.0 : t);
  learned[l] = bins[l] * exp(t * scale);
}

// ------------------------------------------------------------ L-infinity error
template <typename T>
__global__ void __launch_bounds__(TPB) k_linf(const T* __restrict__ a, const T* __restrict__ b, uint64_t n,
                                              unsigned long long* __restrict__ out) {
  double m = 0.0;
  for (uint64_t i = (uint64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (uint64_t)gridDim.x * TPB) {
    const double d = fabs((double)a[i] - (double)b[i]);
    m = d > m ? d : m;
  }
  __shared__ double r[TPB];
  r[threadIdx.x] = m;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s && r[threadIdx.x + s] > r[threadIdx.x]) r[threadIdx.x] = r[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(r[0]));
}

// keep the learned widths if the measured error meets tau, else fall back to the plain ones
__global__ void k_select_bins(const unsigned long long* __restrict__ errbits, double* __restrict__ scalars,
                              double* __restrict__ bins, const double* __restrict__ learned, int nlev) {
  if (threadIdx.x != 0) return;
  const double err = __longlong_as_double((long long)*errbits);
  const bool ok = err <= scalars[0];
  scalars[4] = err;
  scalars[5] = ok ? 0.0 : 1.0;
  if (ok)
    for (int l = 0; l < nlev; ++l) bins[l] = learned[l];
}

// ------------------------------------------------------------ MLP layers
// out[b][o] = act(sum_k in[b][k] W[o][k] + bias[o]); pre-activation kept in z
template <bool RELU>
__global__ void __launch_bounds__(TPB) k_dense_fwd(const float* __restrict__ in, int K, const float* __restrict__ W,
                                                   const float* __restrict__ bias, int O, int B, float* __restrict__ z,
                                                   float* __restrict__ out) {
  const uint64_t t = (uint64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= (uint64_t)B * O) return;
  const int b = (int)(t / O), o = (int)(t % O);
  float s = 0.0f;
  for (int k = 0; k < K; ++k) s = s + in[(uint64_t)b * K + k] * W[o * K + k];
  s = s + bias[o];
  if (z) z[t] = s;
  out[t] = RELU ? (s > 0.0f ? s : 0.0f) : s;
}

// dW[o][k] = sum_b g[b][o] in[b][k]; db[o] = sum_b g[b][o]  (batch in order)
__global__ void __launch_bounds__(TPB) k_dense_wgrad(const float* __restrict__ g, const float* __restrict__ in, int K,
                                                     int O, int B, float* __restrict__ dW, float* __restrict__ db) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  if (t >= O * (K + 1)) return;
  const int o = t / (K + 1), k = t % (K + 1);
  float s = 0.0f;
  if (k < K) {
    for (int b = 0; b < B; ++b) s = s + g[(uint64_t)b * O + o] * in[(uint64_t)b * K + k];
    dW[o * K + k] = s;
  } else {
    for (int b = 0; b < B; ++b) s = s + g[(uint64_t)b * O + o];
    db[o] = s;
  }
}

// gin[b][k] = (sum_o g[b][o] W[o][k]) * (zin[b][k] > 0)   (ReLU derivative of the input layer)
__global__ void __launch_bounds__(TPB) k_dense_dgrad(const float* __restrict__ g, const float* __restrict__ W, int K,
                                                     int O, int B, const float* __restrict__ zin,
                                                     float* __restrict__ gin) {
  const uint64_t t = (uint64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= (uint64_t)B * K) return;
  const int b = (int)(t / K), k = (int)(t % K);
  float s = 0.0f;
  for (int o = 0; o < O; ++o) s = s + g[(uint64_t)b * O + o] * W[o * K + k];
  gin[t] = zin[t] > 0.0f ? s : 0.0f;
}

__global__ void k_normalize_inputs(const float* __restrict__ x, const float* __restrict__ params, int B,
                                   float* __restrict__ xn) {
  const int t = blockIdx.x * TPB + threadIdx.x;
  if (t >= B * F) return;
  const int i = t % F;
  xn[t] = (x[t] - params[i]) / params[F + i];
}

__global__ void __launch_bounds__(TPB) k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int i = blockIdx.x * TPB + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  p[i] = p[i] - lr * mh / (sqrtf(vh) + eps);
}

__global__ void __launch_bounds__(TPB) k_mse(const float* __restrict__ pred, const float* __restrict__ target, int B,
                                             float* __restrict__ dout, double* __restrict__ loss) {
  __shared__ double r[TPB];
  double s = 0.0;
  for (int b = threadIdx.x; b < B; b += TPB) {
    const float d = pred[b] - target[b];
    dout[b] = 2.0f / (float)B * d;
    s += (double)d * (double)d;
  }
  r[threadIdx.x] = s;
  __syncthreads();
  for (int k = TPB / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) r[threadIdx.x] += r[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = r[0] / B;
}

}  // namespace

// ----------------------------------------------------------------- launchers
template <typename T>
void launch_level_stats(const T* c, const uint64_t* d_off, int nlev, double* d_part, double* d_stats,
                        hipStream_t st) {
  KernelTimer kt("level_stats", st);
  hipLaunchKernelGGL(k_stats_partial<T>, dim3(nlev * STATS_BLOCKS), dim3(TPB), 0, st, c, d_off, nlev, d_part,
                     STATS_BLOCKS);
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, st, d_part, d_off, nlev, STATS_BLOCKS, d_stats);
  MG_HIP(hipGetLastError());
}

void launch_features(const double* d_stats, const double* d_scalars, int nlev, const float* d_params, float* d_x,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_features, dim3(1), dim3(64), 0, st, d_stats, d_scalars, nlev, d_params, d_x);
  MG_HIP(hipGetLastError());
}

void launch_apply_theta(const double* d_bins, const float* d_theta, int nlev, double scale, double* d_learned,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_apply_theta, dim3(1), dim3(64), 0, st, d_bins, d_theta, nlev, scale, d_learned);
  MG_HIP(hipGetLastError());
}

template <typename T>
void launch_linf(const T* a, const T* b, uint64_t n, unsigned long long* d_err, hipStream_t st) {
  launch_fill_u64(reinterpret_cast<uint64_t*>(d_err), 1, 0, st);
  KernelTimer kt("linf", st);
  hipLaunchKernelGGL(k_linf<T>, dim3(grid_for(n, 8192)), dim3(TPB), 0, st, a, b, n, d_err);
  MG_HIP(hipGetLastError());
}

void launch_select_bins(const unsigned long long* d_err, double* d_scalars, double* d_bins, const double* d_learned,
                        int nlev, hipStream_t st) {
  hipLaunchKernelGGL(k_select_bins, dim3(1), dim3(1), 0, st, d_err, d_scalars, d_bins, d_learned, nlev);
  MG_HIP(hipGetLastError());
}

// forward over B rows; x already normalised.  cache (nullable): z1, h1, z2, h2 (B x H each)
void mlp_forward(const float* params, const float* x, int B, float* out, float* cache, float* tmp,
                 hipStream_t st) {
  const float* W1 = params + MLP_W1;
  const float* b1 = params + MLP_B1;
  const float* W2 = params + MLP_W2;
  const float* b2 = params + MLP_B2;
  const float* W3 = params + MLP_W3;
  const float* b3 = params + MLP_B3;
  const uint64_t BH = (uint64_t)B * H;
  float* z1 = cache ? cache : nullptr;
  float* h1 = cache ? cache + BH : tmp;
  float* z2 = cache ? cache + 2 * BH : nullptr;
  float* h2 = cache ? cache + 3 * BH : tmp + BH;
  KernelTimer kt("mlp_forward", st);
  hipLaunchKernelGGL(k_dense_fwd<true>, dim3(grid_for(BH, 1u << 20)), dim3(TPB), 0, st, x, F, W1, b1, H, B, z1, h1);
  hipLaunchKernelGGL(k_dense_fwd<true>, dim3(grid_for(BH, 1u << 20)), dim3(TPB), 0, st, h1, H, W2, b2, H, B, z2, h2);
  hipLaunchKernelGGL(k_dense_fwd<false>, dim3(grid_for((uint64_t)B, 1u << 20)), dim3(TPB), 0, st, h2, H, W3, b3, 1, B,
                     (float*)nullptr, out);
  MG_HIP(hipGetLastError());
}

void mlp_backward(const float* params, const float* x, const float* cache, const float* dout, int B, float* grads,
                  float* tmp, hipStream_t st) {
  const float* W2 = params + MLP_W2;
  const float* W3 = params + MLP_W3;
  const uint64_t BH = (uint64_t)B * H;
  const float* z1 = cache;
  const float* h1 = cache + BH;
  const float* z2 = cache + 2 * BH;
  const float* h2 = cache + 3 * BH;
  float* g2 = tmp;       // dL/dz2
  float* g1 = tmp + BH;  // dL/dz1
  KernelTimer kt("mlp_backward", st);
  // layer 3: dW3, db3; dz2 = (dout W3) * relu'(z2)
  hipLaunchKernelGGL(k_dense_wgrad, dim3(grid_for(H + 1)), dim3(TPB), 0, st, dout, h2, H, 1, B, grads + MLP_W3,
                     grads + MLP_B3);
  hipLaunchKernelGGL(k_dense_dgrad, dim3(grid_for(BH, 1u << 20)), dim3(TPB), 0, st, dout, W3, H, 1, B, z2, g2);
  // layer 2
  hipLaunchKernelGGL(k_dense_wgrad, dim3(grid_for((uint64_t)H * (H + 1))), dim3(TPB), 0, st, g2, h1, H, H, B,
                     grads + MLP_W2, grads + MLP_B2);
  hipLaunchKernelGGL(k_dense_dgrad, dim3(grid_for(BH, 1u << 20)), dim3(TPB), 0, st, g2, W2, H, H, B, z1, g1);
  // layer 1
  hipLaunchKernelGGL(k_dense_wgrad, dim3(grid_for((uint64_t)H * (F + 1))), dim3(TPB), 0, st, g1, x, F, H, B,
                     grads + MLP_W1, grads + MLP_B1);
  MG_HIP(hipGetLastError());
}

void mlp_normalize(const float* x, const float* params, int B, float* xn, hipStream_t st) {
  hipLaunchKernelGGL(k_normalize_inputs, dim3(grid_for((uint64_t)B * F)), dim3(TPB), 0, st, x, params, B, xn);
  MG_HIP(hipGetLastError());
}

void mlp_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps, int step,
              hipStream_t st) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_for((uint64_t)n)), dim3(TPB), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  MG_HIP(hipGetLastError());
}

void mlp_mse(const float* pred, const float* target, int B, float* dout, double* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(TPB), 0, st, pred, target, B, dout, loss);
  MG_HIP(hipGetLastError());
}

template void launch_level_stats<float>(const float*, const uint64_t*, int, double*, double*, hipStream_t);
template void launch_level_stats<double>(const double*, const uint64_t*, int, double*, double*, hipStream_t);
template void launch_linf<float>(const float*, const float*, uint64_t, unsigned long long*, hipStream_t);
template void launch_linf<double>(const double*, const double*, uint64_t, unsigned long long*, hipStream_t);

}  // namespace mg
