// Tolerance, bin widths and level-wise quantization kernels (gfx950).
//
// Paper Sec. 2: each multilevel coefficient is replaced by an integer
// multiple of a bin width, and the error is controlled in a chosen norm; the
// relative bound of the first listing (Sec. 3) is read as tol * max|u|.
//   y = float64(c) * (1/b_l),  q = sign(y) floor(|y| + 0.5),
//   symbol = q + R for |q| < R (R = dict/2), else 0 with q kept aside.
// Bin widths are computed on the device from max|u| so that no host round
// trip sits between the max pass and the decomposition.
#include <cfloat>

#include "internal.hpp"

namespace mg {

namespace {
constexpr int TPB = 256;

inline unsigned grid_for(uint64_t n, unsigned cap = 8192) {
  uint64_t g = (n + TPB - 1) / TPB;
  if (g < 1) g = 1;
  return (unsigned)std::min<uint64_t>(g, cap);
}

__device__ inline uint64_t abs_bits(float x) { return (uint64_t)(__float_as_uint(x) & 0x7fffffffu); }
__device__ inline uint64_t abs_bits(double x) {
  return (uint64_t)__double_as_longlong(x) & 0x7fffffffffffffffull;
}

// max of |x| as ordered bit patterns (NaN patterns sort above infinity)
__device__ inline uint64_t abs_bits4(uint4 w, float) {
  const uint32_t m0 = max(w.x & 0x7fffffffu, w.y & 0x7fffffffu);
  const uint32_t m1 = max(w.z & 0x7fffffffu, w.w & 0x7fffffffu);
  return (uint64_t)max(m0, m1);
}
__device__ inline uint64_t abs_bits4(uint4 w, double) {
  const uint64_t b0 = (((uint64_t)w.y << 32) | w.x) & 0x7fffffffffffffffull;
  const uint64_t b1 = (((uint64_t)w.w << 32) | w.z) & 0x7fffffffffffffffull;
  return b0 > b1 ? b0 : b1;
}

template <typename T>
__device__ __forceinline__ void k_maxabs(G3 mg_bid, G3 mg_gdim, const T* __restrict__ d, uint64_t n, uint64_t* out) {
  // The 16-byte-aligned interior is read as 16-byte words, in groups of two
  // loads per lane in two buffers: the next group is in flight while this one
  // is reduced (64 bytes in flight per lane: four loads per group, or more
  // blocks, read slower).  Indices past the end read the last word again (a max is
  // unchanged by repeats), so no load is under a branch and none waits for
  // the group after it.  The unaligned head and the tail (fewer than 16 bytes
  // each) are read element by element by the first lanes of the grid.
  constexpr uint64_t V = 16 / sizeof(T);
  uint64_t m = 0;
  if (n == 0) return;
  uint64_t h = ((16u - ((uintptr_t)d & 15u)) & 15u) / sizeof(T);
  if (h > n) h = n;
  const uint64_t nv = (n - h) / V;
  const uint4* __restrict__ dv = (const uint4*)(d + h);
  const uint64_t step = (uint64_t)mg_gdim.x * TPB;
  const uint64_t gid = (uint64_t)mg_bid.x * TPB + threadIdx.x;
  const uint64_t tail0 = h + nv * V;
  const uint64_t edge = h + (n - tail0);
  if (gid < edge) {
    const uint64_t e = gid < h ? gid : tail0 + (gid - h);
    m = abs_bits(d[e]);
  }
  if (nv > 0) {
    auto load = [&](uint64_t base, uint4 (&v)[2]) {
#pragma unroll
      for (int u = 0; u < 2; ++u) v[u] = dv[min(base + u * step, nv - 1)];
    };
    auto reduce = [&](const uint4 (&v)[2]) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const uint64_t b = abs_bits4(v[u], T());
        m = b > m ? b : m;
      }
    };
    uint4 va[2], vb[2];
    uint64_t i = gid;
    load(i, va);
    for (; i < nv; i += 4 * step) {
      load(i + 2 * step, vb);
      reduce(va);
      load(i + 4 * step, va);
      reduce(vb);
    }
  }
  __shared__ uint64_t red[TPB];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      uint64_t o = red[threadIdx.x + s];
      if (o > red[threadIdx.x]) red[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax((unsigned long long*)out, (unsigned long long)red[0]);
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_maxabs_k(const T* __restrict__ d, uint64_t n, uint64_t* out) {
  k_maxabs<T>(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, d, n, out);
}


// Largest max|u| / b accepted: coefficients stay within a small multiple of
// max|u| (interpolation is convex and the L2 projections are stable in the
// maximum norm), so |c / b| stays far below 2^63 and the integer conversion of
// the quantizer is exact; learned widths, down to exp(-3) b, keep that margin.
constexpr double kMaxScale = 562949953421312.0;  // 2^49

// scalars: [0] tau_abs, [1] maxabs, [2] non-finite flag, [3] tau_eff,
// [6] tolerance outside the supported range: the rounding reserve
// rho = 4 (L+1) eps max|u| exceeds tau / 2, or max|u| / b_l reaches 2^49
__device__ __forceinline__ void k_bins(G3 mg_bid, G3 mg_gdim, int f64, const uint64_t* __restrict__ maxbits, double tol, int rel, double S,
                       int L, int alloc, const BinArgs& args, double* __restrict__ bins,
                       double* __restrict__ scalars) {
  const double* K = args.K;
  const double* counts = args.counts;
  if (threadIdx.x != 0 || mg_bid.x != 0) return;
  const uint64_t mb = *maxbits;
  double maxabs;
  int nonfinite;
  double eps;
  if (f64) {
    nonfinite = mb >= 0x7ff0000000000000ull;
    maxabs = __longlong_as_double((long long)mb);
    eps = DBL_EPSILON;
  } else {
    nonfinite = mb >= 0x7f800000ull;
    maxabs = (double)__uint_as_float((unsigned)mb);
    eps = (double)FLT_EPSILON;
  }
  const double tau = rel ? tol * maxabs : tol;
  const double rho = 4.0 * (double)(L + 1) * eps * maxabs;
  const double half = 0.5 * tau;
  const double tau_eff = tau - (rho < half ? rho : half);
  scalars[0] = tau;
  scalars[1] = maxabs;
  scalars[2] = (double)nonfinite;
  scalars[3] = tau_eff;
  scalars[6] = 0.0;
  if (!(tau_eff > 0.0)) {
    for (int l = 0; l <= L; ++l) bins[l] = 1.0;
    return;
  }
  if (alloc == MGARD_ALLOC_COUNT) {
    double tot = 0.0;
    for (int l = 0; l <= L; ++l) tot += counts[l];
    for (int l = 0; l <= L; ++l) bins[l] = 2.0 * tau_eff * counts[l] / ((1.0 + K[l]) * tot);
  } else {
    const double b = 2.0 * tau_eff / S;
    for (int l = 0; l <= L; ++l) bins[l] = b;
  }
  bool out = rho > half;
  for (int l = 0; l <= L; ++l) out = out || !(maxabs < kMaxScale * bins[l]);
  scalars[6] = (!nonfinite && out) ? 1.0 : 0.0;
}

__global__ void k_bins_k(int f64, const uint64_t* __restrict__ maxbits, double tol, int rel, double S,
                       int L, int alloc, BinArgs args, double* __restrict__ bins,
                       double* __restrict__ scalars) {
  k_bins(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, f64, maxbits, tol, rel, S, L, alloc, args, bins, scalars);
}


__device__ inline int level_of(uint64_t i, const uint64_t* __restrict__ off, int nlev) {
  int l = 0;
  while (l + 1 < nlev && i >= off[l + 1]) ++l;
  return l;
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_quantize(const T* __restrict__ c, uint64_t n,
                                                  const uint64_t* __restrict__ off, int nlev,
                                                  const double* __restrict__ bins, int R,
                                                  uint16_t* __restrict__ sym, int64_t* __restrict__ qside) {
  for (uint64_t i = (uint64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (uint64_t)gridDim.x * TPB) {
    const int l = level_of(i, off, nlev);
    const double inv_b = 1.0 / bins[l];
    const double y = (double)c[i] * inv_b;
    const double a = floor(fabs(y) + 0.5);
    const int64_t q = (int64_t)(y < 0.0 ? -a : a);
    if (q > -R && q < R) {
      sym[i] = (uint16_t)(q + R);
    } else {
      sym[i] = 0;
      qside[i] = q;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_dequantize(const uint16_t* __restrict__ sym,
                                                    const int64_t* __restrict__ qside, uint64_t n,
                                                    const uint64_t* __restrict__ off, int nlev,
                                                    const double* __restrict__ bins, int R,
                                                    T* __restrict__ c) {
  for (uint64_t i = (uint64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (uint64_t)gridDim.x * TPB) {
    const int l = level_of(i, off, nlev);
    const uint16_t s = sym[i];
    const int64_t q = s ? (int64_t)s - R : qside[i];
    c[i] = static_cast<T>((double)q * bins[l]);
  }
}

}  // namespace

namespace {
__device__ __forceinline__ void k_fill_u64(G3 mg_bid, G3 mg_gdim, uint64_t* __restrict__ p, uint64_t n, uint64_t v) {
  for (uint64_t t = (uint64_t)mg_bid.x * TPB + threadIdx.x; t < n; t += (uint64_t)mg_gdim.x * TPB) p[t] = v;
}

__global__ void __launch_bounds__(TPB) k_fill_u64_k(uint64_t* __restrict__ p, uint64_t n, uint64_t v) {
  k_fill_u64(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, p, n, v);
}

}  // namespace

// A kernel rather than hipMemsetAsync, so that captured graphs hold no memset node.
void launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t st) {
  if (!n) return;
  MG_LAUNCH((&k_fill_u64), (k_fill_u64_k), (TPB), (0), (dim3(grid_for(n, 1024))), st, p, n, v);
  MG_HIP(hipGetLastError());
}

template <typename T>
void launch_maxabs(const T* d, uint64_t n, uint64_t* d_bits, hipStream_t st) {
  launch_fill_u64(d_bits, 1, 0, st);
  KernelTimer kt("maxabs", st);
  // 1024 blocks (16 wavefronts per CU) read faster than 2048 or more in a sweep
  // of the cap; below that, at least 32 elements per thread (two trips), so a
  // small array (a field of a batch) is not spread over blocks that each
  // reduce a few values
  MG_LAUNCH((&k_maxabs<T>), (k_maxabs_k<T>), (TPB), (0), (dim3(grid_for(n / 32, 1024))), st, d, n, d_bits);
  MG_HIP(hipGetLastError());
}

void launch_bins(int f64, const uint64_t* d_maxbits, double tol, int rel, double S, int L,
                 int alloc, const BinArgs& a, double* d_bins, double* d_scalars, hipStream_t st) {
  MG_LAUNCH((&k_bins), (k_bins_k), (64), (0), (dim3(1)), st, f64, d_maxbits, tol, rel, S, L, alloc, a, d_bins, d_scalars);
  MG_HIP(hipGetLastError());
}

template <typename T>
void launch_quantize(const T* c, uint64_t n, const uint64_t* d_level_off, int nlev,
                     const double* d_bins, int R, uint16_t* sym, int64_t* qside, hipStream_t st) {
  if (n == 0) return;
  KernelTimer kt("quantize", st);
  hipLaunchKernelGGL(k_quantize<T>, dim3(grid_for(n, 1u << 20)), dim3(TPB), 0, st, c, n, d_level_off, nlev,
                     d_bins, R, sym, qside);
  MG_HIP(hipGetLastError());
}

template <typename T>
void launch_dequantize(const uint16_t* sym, const int64_t* qside, uint64_t n,
                       const uint64_t* d_level_off, int nlev, const double* d_bins, int R, T* c,
                       hipStream_t st) {
  if (n == 0) return;
  KernelTimer kt("dequantize", st);
  hipLaunchKernelGGL(k_dequantize<T>, dim3(grid_for(n, 1u << 20)), dim3(TPB), 0, st, sym, qside, n,
                     d_level_off, nlev, d_bins, R, c);
  MG_HIP(hipGetLastError());
}

template void launch_maxabs<float>(const float*, uint64_t, uint64_t*, hipStream_t);
template void launch_maxabs<double>(const double*, uint64_t, uint64_t*, hipStream_t);
template void launch_quantize<float>(const float*, uint64_t, const uint64_t*, int, const double*, int,
                                     uint16_t*, int64_t*, hipStream_t);
template void launch_quantize<double>(const double*, uint64_t, const uint64_t*, int, const double*, int,
                                      uint16_t*, int64_t*, hipStream_t);
template void launch_dequantize<float>(const uint16_t*, const int64_t*, uint64_t, const uint64_t*, int,
                                       const double*, int, float*, hipStream_t);
template void launch_dequantize<double>(const uint16_t*, const int64_t*, uint64_t, const uint64_t*, int,
                                        const double*, int, double*, hipStream_t);

}  // namespace mg
