// L2 norm of a field and the bin widths of the s-norm bound (gfx950).
//
// The paper controls the error in several norms chosen by a smoothness
// parameter s, with level-wise bin widths from error estimators (Sec. 2;
// Sec. 3, first listing).  For the P1 hierarchy of the decomposition:
//   * ||u||^2 = u^T M u, M = kron_d M_d the consistent mass matrices of the
//     decomposed sides (identity for sides that are not decomposed);
//   * the s-norm sums the level components (Q_l - Q_{l-1}) u weighted by
//     4^(s l); a coefficient error delta_l adds (I - Q_{l-1}) delta_l, these
//     are orthogonal across levels, so ||e||_s^2 <= sum_l 4^(s l) W_l
//     max|delta_l|^2 with W_l the hat integrals of level l's new nodes;
//   * widths b_l = 2 tau_eff g_l, g_l = sqrt(N_l / ((N 4^(s l)) W_l)) (host,
//     float64), keep the most bits under that bound;
//   * tau_eff = tau minus the rounding reserve 4 (L+1) eps max|u| scaled by
//     max(1, 2^(s L)) sqrt(W_0); tau = tol ||u|| (relative, s = 0) or tol.
//
// k_mass_norm: one block per row of the contiguous dimension (grid-stride
// over rows), lanes along the row; every element sums its 3^D stencil of
// mass weights (row weights are block-uniform) and adds u_i (M u)_i to a
// float64 partial; the block partials are summed in block order by one
// thread, so the result does not depend on the launch order.
#include <cfloat>

#include "internal.hpp"

namespace mg {

namespace {
constexpr int TPB = 256;
constexpr int NORM_BLOCKS = 4096;

struct MassArgs {
  const double* a[MAXD];  // sub-diagonal, diagonal, super-diagonal per slot (null: identity)
  const double* b[MAXD];
  const double* c[MAXD];
  int64_t n[MAXD];
};

// weight of offset o in {-1, 0, 1} at index i of slot s
__device__ inline double band(const MassArgs& m, int s, int64_t i, int o) {
  if (!m.b[s]) return o == 0 ? 1.0 : 0.0;
  if (o == 0) return m.b[s][i];
  if (o < 0) return i > 0 ? m.a[s][i] : 0.0;
  return i + 1 < m.n[s] ? m.c[s][i] : 0.0;
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_mass_norm(const T* __restrict__ u, MassArgs m, double* __restrict__ part) {
  const int64_t n3 = m.n[3];
  const uint64_t rows = (uint64_t)m.n[0] * (uint64_t)m.n[1] * (uint64_t)m.n[2];
  const uint64_t st2 = (uint64_t)n3, st1 = st2 * (uint64_t)m.n[2], st0 = st1 * (uint64_t)m.n[1];
  double acc = 0.0;
  for (uint64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const int64_t i2 = (int64_t)(r % (uint64_t)m.n[2]);
    const uint64_t r01 = r / (uint64_t)m.n[2];
    const int64_t i1 = (int64_t)(r01 % (uint64_t)m.n[1]);
    const int64_t i0 = (int64_t)(r01 / (uint64_t)m.n[1]);
    for (int64_t i3 = threadIdx.x; i3 < n3; i3 += TPB) {
      double mu = 0.0;
      for (int o0 = -1; o0 <= 1; ++o0) {
        const double w0 = band(m, 0, i0, o0);
        if (w0 == 0.0) continue;
        for (int o1 = -1; o1 <= 1; ++o1) {
          const double w1 = band(m, 1, i1, o1);
          if (w1 == 0.0) continue;
          for (int o2 = -1; o2 <= 1; ++o2) {
            const double w2 = band(m, 2, i2, o2);
            if (w2 == 0.0) continue;
            const double w012 = (w0 * w1) * w2;
            const T* row = u + (uint64_t)(i0 + o0) * st0 + (uint64_t)(i1 + o1) * st1 + (uint64_t)(i2 + o2) * st2;
            for (int o3 = -1; o3 <= 1; ++o3) {
              const double w3 = band(m, 3, i3, o3);
              if (w3 == 0.0) continue;
              mu += (w012 * w3) * (double)row[i3 + o3];
            }
          }
        }
      }
      acc += (double)u[r * st2 + (uint64_t)i3] * mu;
    }
  }
  __shared__ double red[TPB];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_partials(const double* __restrict__ part, int n, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  *out = s;
}

constexpr double kMaxScale = 562949953421312.0;  // 2^49, as for the L-infinity widths

// scalars: [0] tau_abs, [1] maxabs, [2] non-finite flag, [3] tau_eff, [6] out of range
__global__ void k_bins_snorm(int f64, const uint64_t* __restrict__ maxbits, const double* __restrict__ nrm2, double tol,
                             int rel, int L, SnormArgs a, double* __restrict__ bins, double* __restrict__ scalars) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint64_t mb = *maxbits;
  double maxabs, eps;
  int nonfinite;
  if (f64) {
    nonfinite = mb >= 0x7ff0000000000000ull;
    maxabs = __longlong_as_double((long long)mb);
    eps = DBL_EPSILON;
  } else {
    nonfinite = mb >= 0x7f800000ull;
    maxabs = (double)__uint_as_float((unsigned)mb);
    eps = (double)FLT_EPSILON;
  }
  const double tau = rel ? tol * sqrt(*nrm2) : tol;
  const double rho = 4.0 * (double)(L + 1) * eps * maxabs;
  const double rs = rho * a.reserve;
  const double half = 0.5 * tau;
  const double tau_eff = tau - (rs < half ? rs : half);
  scalars[0] = tau;
  scalars[1] = maxabs;
  scalars[2] = (double)nonfinite;
  scalars[3] = tau_eff;
  scalars[6] = 0.0;
  if (!(tau_eff > 0.0)) {
    for (int l = 0; l <= L; ++l) bins[l] = 1.0;
    return;
  }
  bool out = rs > half;
  for (int l = 0; l <= L; ++l) {
    bins[l] = 2.0 * tau_eff * a.g[l];
    out = out || !(maxabs < kMaxScale * bins[l]);
  }
  scalars[6] = (!nonfinite && out) ? 1.0 : 0.0;
}

}  // namespace

SnormArgs snorm_args(const Hierarchy& h, double s) {
  SnormArgs a{};
  double N = 0.0;
  for (int l = 0; l <= h.L; ++l) N += (double)h.level_count[l];
  for (int l = 0; l <= h.L; ++l)
    a.g[l] = std::sqrt((double)h.level_count[l] / ((N * std::pow(2.0, 2.0 * s * l)) * h.W[l]));
  a.reserve = std::max(1.0, std::pow(2.0, s * h.L)) * std::sqrt(h.W[0]);
  return a;
}

uint64_t mass_norm_scratch_bytes() { return carve_size<double>(NORM_BLOCKS) + carve_size<double>(1); }

template <typename T>
void launch_mass_norm(const Hierarchy& h, const double* d_bands, const T* u, void* scratch, double* d_out,
                      hipStream_t st) {
  MassArgs m{};
  for (int s = 0; s < MAXD; ++s) {
    m.n[s] = h.shape[s];
    if (h.active[s]) {
      const double* base = d_bands + h.mass_off[s];
      m.a[s] = base;
      m.b[s] = base + h.shape[s];
      m.c[s] = base + 2 * h.shape[s];
    }
  }
  const uint64_t rows = (uint64_t)h.shape[0] * (uint64_t)h.shape[1] * (uint64_t)h.shape[2];
  const unsigned blocks = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(rows, NORM_BLOCKS));
  double* part = static_cast<double*>(scratch);
  KernelTimer kt("mass_norm", st);
  hipLaunchKernelGGL(k_mass_norm<T>, dim3(blocks), dim3(TPB), 0, st, u, m, part);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, st, part, (int)blocks, d_out);
  MG_HIP(hipGetLastError());
}

void launch_bins_snorm(int f64, const uint64_t* d_maxbits, const double* d_nrm2, double tol, int rel, int L,
                       const SnormArgs& a, double* d_bins, double* d_scalars, hipStream_t st) {
  hipLaunchKernelGGL(k_bins_snorm, dim3(1), dim3(64), 0, st, f64, d_maxbits, d_nrm2, tol, rel, L, a, d_bins,
                     d_scalars);
  MG_HIP(hipGetLastError());
}

template void launch_mass_norm<float>(const Hierarchy&, const double*, const float*, void*, double*, hipStream_t);
template void launch_mass_norm<double>(const Hierarchy&, const double*, const double*, void*, double*, hipStream_t);

}  // namespace mg
