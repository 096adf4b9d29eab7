// Multilevel decomposition and recomposition kernels (gfx950).
//
// One level of the decomposition (paper Sec. 2, recursive multilevel
// decomposition; P1 finite-element reading):
//   1. coefficients c = u - Pi u at the new nodes, Pi the multilinear
//      interpolant from the coarse nodes, evaluated as nested 1D
//      interpolations with the highest dimension innermost, each step
//      (wl*a) + (wr*b) rounded to T;
//   2. load vector f = (P^T M) cbar along dimensions D-1 .. 0 (mass stencil
//      ((a*g[i-1] + b*g[i]) + c*g[i+1]), restriction ((rl*g[c-1] + g[c]) +
//      rr*g[c+1]));
//   3. Thomas solves with the coarse mass matrix along dimensions 0 .. D-1;
//   4. u_{l-1} = u_l|coarse + z.
// Recomposition inverts it: z from c, u_l|coarse = u_{l-1} - z,
// u_l = c + Pi(u_l|coarse) at new nodes.
//
// The order of every rounding is fixed above so that results are
// reproducible; the library is built with floating-point contraction off.
#include <algorithm>

#include "internal.hpp"

namespace mg {

namespace {

constexpr int TPB = 256;

inline unsigned grid_for(uint64_t n, unsigned cap = 1u << 20) {
  uint64_t g = (n + TPB - 1) / TPB;
  if (g < 1) g = 1;
  return (unsigned)std::min<uint64_t>(g, cap);
}

// slot coordinates of a fine-grid linear index
struct Coord {
  int32_t i[MAXD];
};

template <typename T>
__device__ inline Coord unflatten(uint64_t p, const LevelGeom<T>& g) {
  Coord c;
#pragma unroll
  for (int s = MAXD - 1; s >= 0; --s) {
    uint64_t n = (uint64_t)g.nf[s];
    c.i[s] = (int32_t)(p % n);
    p /= n;
  }
  return c;
}

// mask of slots whose index is a new node of this level
template <typename T>
__device__ inline int new_mask(const Coord& c, const LevelGeom<T>& g) {
  int m = 0;
#pragma unroll
  for (int s = 0; s < MAXD; ++s)
    if (g.act[s] && (c.i[s] & 1) && c.i[s] < g.nf[s] - 1) m |= 1 << s;
  return m;
}

template <typename T>
__device__ inline int coarse_idx(int i, int s, const LevelGeom<T>& g) {
  return g.act[s] ? ((i + 1) >> 1) : i;
}

// stream position of a new node
template <typename T>
__device__ inline uint64_t stream_pos(const Coord& c, int mslot, const LevelGeom<T>& g) {
  const int m = mslot >> g.pad_slots;
  uint64_t pos = g.level_off + g.sub[m];
#pragma unroll
  for (int s = 0; s < MAXD; ++s) {
    int idx = ((mslot >> s) & 1) ? (c.i[s] >> 1) : coarse_idx(c.i[s], s, g);
    pos += (uint64_t)idx * g.sub[16 + 4 * m + s];
  }
  return pos;
}

template <class X>
__device__ inline X sel4(const X* a, int s) {
  return s == 0 ? a[0] : (s == 1 ? a[1] : (s == 2 ? a[2] : a[3]));
}

// Pi at a new node.  FINE: corners read from the fine grid `src` (coarse
// positions of grid l); otherwise from the dense coarse grid `src` (grid l-1).
template <typename T, bool FINE>
__device__ inline T interpolate(const T* __restrict__ src, const Coord& c, int mslot,
                                const LevelGeom<T>& g) {
  uint64_t st[MAXD];  // strides of the grid we read
  uint64_t acc = 1;
#pragma unroll
  for (int s = MAXD - 1; s >= 0; --s) {
    st[s] = acc;
    acc *= (uint64_t)(FINE ? g.nf[s] : g.nc[s]);
  }
  uint64_t base = 0;
#pragma unroll
  for (int s = 0; s < MAXD; ++s) {
    int id;
    if ((mslot >> s) & 1)
      id = FINE ? c.i[s] - 1 : (c.i[s] >> 1);
    else
      id = FINE ? c.i[s] : coarse_idx(c.i[s], s, g);
    base += (uint64_t)id * st[s];
  }
  // odd slots in increasing order: their corner step and weights
  uint64_t ost[MAXD];
  T owl[MAXD], owr[MAXD];
  int mm = mslot;
#pragma unroll
  for (int j = 0; j < MAXD; ++j) {
    const int s = mm ? __builtin_ctz(mm) : 0;
    const bool live = mm != 0;
    mm &= mm - 1;
    ost[j] = (uint64_t)(FINE ? 2 : 1) * sel4(st, s);
    const int is = sel4(c.i, s);
    owl[j] = live ? sel4(g.wl, s)[is] : T(0);
    owr[j] = live ? sel4(g.wr, s)[is] : T(0);
  }
  const int k = __builtin_popcount(mslot);
  T v[16];
#pragma unroll
  for (int cc = 0; cc < 16; ++cc) {
    if (cc < (1 << k)) {
      uint64_t off = base;
#pragma unroll
      for (int j = 0; j < MAXD; ++j)
        if ((cc >> j) & 1) off += ost[j];
      v[cc] = src[off];
    }
  }
  // reduce the highest odd dimension first (innermost interpolation)
#pragma unroll
  for (int j = MAXD - 1; j >= 0; --j) {
    if (j < k) {
      const int half = 1 << j;
#pragma unroll
      for (int cc = 0; cc < 8; ++cc)
        if (cc < half) v[cc] = owl[j] * v[cc] + owr[j] * v[cc + half];
    }
  }
  return v[0];
}

template <typename T>
__device__ inline void quantize_one(T c, double inv_b, int R, uint64_t pos, uint16_t* __restrict__ sym,
                                    int64_t* __restrict__ qside) {
  double y = (double)c * inv_b;
  double a = floor(fabs(y) + 0.5);
  int64_t q = (int64_t)(y < 0.0 ? -a : a);
  if (q > -R && q < R) {
    sym[pos] = (uint16_t)(q + R);
  } else {
    sym[pos] = 0;
    qside[pos] = q;
  }
}

template <typename T>
__device__ inline T dequantize_one(const uint16_t* __restrict__ sym, const int64_t* __restrict__ qside,
                                   uint64_t pos, double b, int R) {
  uint16_t s = sym[pos];
  int64_t q = s ? (int64_t)s - R : qside[pos];
  return static_cast<T>((double)q * b);
}

// Step 1 (+ fused quantization when MODE == 1).
template <typename T, int MODE>
__device__ __forceinline__ void k_coeff(G3 mg_bid, G3 mg_gdim, const T* __restrict__ u, T* __restrict__ cbar,
                                               T* __restrict__ ucoarse, T* __restrict__ cstream,
                                               uint16_t* __restrict__ sym, int64_t* __restrict__ qside,
                                               const double* __restrict__ bins, int level, int R,
                                               const LevelGeom<T>& g, uint64_t nfine) {
  double inv_b = 0.0;
  if (MODE == 1) inv_b = 1.0 / bins[level];
  for (uint64_t p = (uint64_t)mg_bid.x * TPB + threadIdx.x; p < nfine;
       p += (uint64_t)mg_gdim.x * TPB) {
    Coord c = unflatten(p, g);
    const int m = new_mask(c, g);
    const T up = u[p];
    if (m == 0) {
      uint64_t q = 0;
#pragma unroll
      for (int s = 0; s < MAXD; ++s) q = q * (uint64_t)g.nc[s] + (uint64_t)coarse_idx(c.i[s], s, g);
      ucoarse[q] = up;
      cbar[p] = T(0);
      continue;
    }
    const T cv = up - interpolate<T, true>(u, c, m, g);
    cbar[p] = cv;
    const uint64_t pos = stream_pos(c, m, g);
    if (MODE == 0)
      cstream[pos] = cv;
    else
      quantize_one(cv, inv_b, R, pos, sym, qside);
  }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(TPB) k_coeff_k(const T* __restrict__ u, T* __restrict__ cbar,
                                               T* __restrict__ ucoarse, T* __restrict__ cstream,
                                               uint16_t* __restrict__ sym, int64_t* __restrict__ qside,
                                               const double* __restrict__ bins, int level, int R,
                                               LevelGeom<T> g, uint64_t nfine) {
  k_coeff<T, MODE>(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, u, cbar, ucoarse, cstream, sym, qside, bins, level, R, g, nfine);
}


// Step 2 along one dimension: (outer, nf, inner) -> (outer, nc, inner).
template <typename T>
__device__ __forceinline__ void k_mass_restrict(G3 mg_bid, G3 mg_gdim, const T* __restrict__ in, T* __restrict__ out,
                                                       uint64_t outer, int nf, int nc, uint64_t inner,
                                                       const DimConsts<T>& w) {
  const uint64_t total = outer * (uint64_t)nc * inner;
  for (uint64_t t = (uint64_t)mg_bid.x * TPB + threadIdx.x; t < total;
       t += (uint64_t)mg_gdim.x * TPB) {
    const uint64_t k = t % inner;
    const uint64_t r = t / inner;
    const int j = (int)(r % (uint64_t)nc);
    const uint64_t o = r / (uint64_t)nc;
    const T* line = in + o * (uint64_t)nf * inner + k;
    auto G = [&](int i) { return line[(uint64_t)i * inner]; };
    auto Mg = [&](int i) {
      T s = w.mb[i] * G(i);
      if (i > 0) s = w.ma[i] * G(i - 1) + s;
      if (i < nf - 1) s = s + w.mc[i] * G(i + 1);
      return s;
    };
    const int c = (j == nc - 1) ? nf - 1 : 2 * j;
    T f = Mg(c);
    if (c >= 2 && !(c & 1)) f = w.rl[j] * Mg(c - 1) + f;
    if (!(c & 1) && c < nf - 2) f = f + w.rr[j] * Mg(c + 1);
    out[(o * (uint64_t)nc + j) * inner + k] = f;
  }
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_mass_restrict_k(const T* __restrict__ in, T* __restrict__ out,
                                                       uint64_t outer, int nf, int nc, uint64_t inner,
                                                       DimConsts<T> w) {
  k_mass_restrict<T>(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, in, out, outer, nf, nc, inner, w);
}


// Step 3 along one dimension, in place, one thread per line.
template <typename T>
__device__ __forceinline__ void k_thomas(G3 mg_bid, G3 mg_gdim, T* __restrict__ data, uint64_t outer, int n, uint64_t inner,
                                                const T* __restrict__ ta, const T* __restrict__ tr,
                                                const T* __restrict__ tcp) {
  // Both sweeps load G values of the line before the group's
  // recurrence; the weights are restrict (scalar loads).  Same arithmetic and
  // order as the plain loops.
  constexpr int G = 16;
  const uint64_t lines = outer * inner;
  for (uint64_t t = (uint64_t)mg_bid.x * TPB + threadIdx.x; t < lines;
       t += (uint64_t)mg_gdim.x * TPB) {
    const uint64_t k = t % inner;
    const uint64_t o = t / inner;
    T* line = data + o * (uint64_t)n * inner + k;
    T prev = line[0] * tr[0];
    line[0] = prev;
    // two buffers: the next group's loads are issued before this group's
    // recurrence.  Indices are clamped into the line and every load is
    // unconditional, so the wait before a group covers only the older group's
    // loads (a load under a branch makes the compiler wait for all of them);
    // the sweeps use only values whose index lies in the line.
    auto load_f = [&](int i0, T* v) {
#pragma unroll
      for (int q = 0; q < G; ++q) v[q] = line[(uint64_t)min(i0 + q, n - 1) * inner];
    };
    auto fwd = [&](int i0, const T* v) {
      if (i0 + G <= n) {  // whole group: one straight block, weight loads issued together
#pragma unroll
        for (int q = 0; q < G; ++q) {
          prev = (v[q] - ta[i0 + q] * prev) * tr[i0 + q];
          line[(uint64_t)(i0 + q) * inner] = prev;
        }
        return;
      }
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const int i = i0 + q;
        if (i < n) {
          prev = (v[q] - ta[i] * prev) * tr[i];
          line[(uint64_t)i * inner] = prev;
        }
      }
    };
    {
      T va[G], vb[G];
      load_f(1, va);
      for (int i0 = 1; i0 < n; i0 += 2 * G) {
        load_f(i0 + G, vb);
        fwd(i0, va);
        load_f(i0 + 2 * G, va);
        fwd(i0 + G, vb);
      }
    }
    T x = prev;
    auto load_b = [&](int i0, T* v) {
#pragma unroll
      for (int q = 0; q < G; ++q) v[q] = line[(uint64_t)max(i0 - q, 0) * inner];
    };
    auto bwd = [&](int i0, const T* v) {
      if (i0 - (G - 1) >= 0) {
#pragma unroll
        for (int q = 0; q < G; ++q) {
          x = v[q] - tcp[i0 - q] * x;
          line[(uint64_t)(i0 - q) * inner] = x;
        }
        return;
      }
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const int i = i0 - q;
        if (i >= 0) {
          x = v[q] - tcp[i] * x;
          line[(uint64_t)i * inner] = x;
        }
      }
    };
    {
      T va[G], vb[G];
      load_b(n - 2, va);
      for (int i0 = n - 2; i0 >= 0; i0 -= 2 * G) {
        load_b(i0 - G, vb);
        bwd(i0, va);
        load_b(i0 - 2 * G, va);
        bwd(i0 - G, vb);
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_thomas_k(T* __restrict__ data, uint64_t outer, int n, uint64_t inner,
                                                const T* __restrict__ ta, const T* __restrict__ tr,
                                                const T* __restrict__ tcp) {
  k_thomas<T>(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, data, outer, n, inner, ta, tr, tcp);
}


// Thomas along the contiguous dimension: `rows` lines per block staged in LDS
// (coalesced, every load of a lane in flight at once), one lane per line, the same
// arithmetic as k_thomas, then written back.  Lines sit `stride` (odd)
// elements apart in LDS so the lanes of a wavefront fall in different banks.
constexpr int ROWS_LDS = 65536;  // bytes

template <typename T>
__device__ __forceinline__ void k_thomas_rows(G3 mg_bid, G3 mg_gdim, T* __restrict__ data, uint64_t nrows, int n, int rows,
                                                     int stride, const T* __restrict__ ta,
                                                     const T* __restrict__ tr, const T* __restrict__ tcp) {
  constexpr int CAP = ROWS_LDS / (int)sizeof(T);
  __shared__ T tile[CAP];
  // every element a lane copies is loaded before any is stored (clamped
  // indices, unconditional loads): one wait for memory per block
  constexpr int EPT = CAP / TPB;
  const uint64_t r0 = (uint64_t)mg_bid.x * rows;
  const int nr = (int)min((uint64_t)rows, nrows - r0);
  const int cnt = nr * n;
  T* g = data + r0 * (uint64_t)n;
  {
    T v[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) v[u] = g[min(threadIdx.x + (unsigned)(u * TPB), (unsigned)cnt - 1)];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const int k = threadIdx.x + u * TPB;
      if (k < cnt) tile[(k / n) * stride + k % n] = v[u];
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nr) {
    T* line = tile + threadIdx.x * stride;
    T prev = line[0] * tr[0];
    line[0] = prev;
#pragma unroll 8
    for (int i = 1; i < n; ++i) {
      prev = (line[i] - ta[i] * prev) * tr[i];
      line[i] = prev;
    }
    T x = prev;
#pragma unroll 8
    for (int i = n - 2; i >= 0; --i) {
      x = line[i] - tcp[i] * x;
      line[i] = x;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < cnt; k += TPB) g[k] = tile[(k / n) * stride + k % n];
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_thomas_rows_k(T* __restrict__ data, uint64_t nrows, int n, int rows,
                                                     int stride, const T* __restrict__ ta,
                                                     const T* __restrict__ tr, const T* __restrict__ tcp) {
  k_thomas_rows<T>(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, data, nrows, n, rows, stride, ta, tr, tcp);
}


// Thomas along slot s: lines of the contiguous dimension go through LDS when a
// line fits, other dimensions use the strided kernel.
template <typename T>
void launch_thomas_any(T* data, uint64_t outer, int n, uint64_t inner, const DimConsts<T>& w, hipStream_t st) {
  const int stride = n | 1;
  if (inner == 1 && (uint64_t)stride * sizeof(T) <= (uint64_t)ROWS_LDS) {
    const int rows = (int)std::min<uint64_t>(TPB, (uint64_t)ROWS_LDS / ((uint64_t)stride * sizeof(T)));
    MG_LAUNCH((&k_thomas_rows<T>), (k_thomas_rows_k<T>), (TPB), (0), (dim3((unsigned)((outer + rows - 1) / rows))), st, data, outer, n, rows, stride, w.ta, w.tr, w.tcp);
  } else {
    MG_LAUNCH((&k_thomas<T>), (k_thomas_k<T>), (TPB), (0), (dim3(grid_for(outer * inner))), st, data, outer, n, inner, w.ta, w.tr, w.tcp);
  }
}

template <typename T, bool ADD>
__device__ __forceinline__ void k_axpy(G3 mg_bid, G3 mg_gdim, T* __restrict__ dst, const T* __restrict__ a,
                                              const T* __restrict__ b, uint64_t n) {
  for (uint64_t t = (uint64_t)mg_bid.x * TPB + threadIdx.x; t < n; t += (uint64_t)mg_gdim.x * TPB)
    dst[t] = ADD ? a[t] + b[t] : a[t] - b[t];
}

template <typename T, bool ADD>
__global__ void __launch_bounds__(TPB) k_axpy_k(T* __restrict__ dst, const T* __restrict__ a,
                                              const T* __restrict__ b, uint64_t n) {
  k_axpy<T, ADD>(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, dst, a, b, n);
}


// coarsest grid <-> stream[0, n0)
template <typename T, int MODE>
__device__ __forceinline__ void k_coarsest_out(G3 mg_bid, G3 mg_gdim, const T* __restrict__ src, T* __restrict__ cstream,
                                                      uint16_t* __restrict__ sym,
                                                      int64_t* __restrict__ qside,
                                                      const double* __restrict__ bins, int R, uint64_t n) {
  double inv_b = 0.0;
  if (MODE == 1) inv_b = 1.0 / bins[0];
  for (uint64_t t = (uint64_t)mg_bid.x * TPB + threadIdx.x; t < n; t += (uint64_t)mg_gdim.x * TPB) {
    if (MODE == 0)
      cstream[t] = src[t];
    else
      quantize_one(src[t], inv_b, R, t, sym, qside);
  }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(TPB) k_coarsest_out_k(const T* __restrict__ src, T* __restrict__ cstream,
                                                      uint16_t* __restrict__ sym,
                                                      int64_t* __restrict__ qside,
                                                      const double* __restrict__ bins, int R, uint64_t n) {
  k_coarsest_out<T, MODE>(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, src, cstream, sym, qside, bins, R, n);
}


template <typename T, int MODE>
__global__ void __launch_bounds__(TPB) k_coarsest_in(T* __restrict__ dst, const T* __restrict__ cstream,
                                                     const uint16_t* __restrict__ sym,
                                                     const int64_t* __restrict__ qside,
                                                     const double* __restrict__ bins, int R, uint64_t n) {
  for (uint64_t t = (uint64_t)blockIdx.x * TPB + threadIdx.x; t < n; t += (uint64_t)gridDim.x * TPB)
    dst[t] = MODE == 0 ? cstream[t] : dequantize_one<T>(sym, qside, t, bins[0], R);
}

// Recomposition: scatter the level's coefficients to the fine grid (zeros at coarse nodes).
template <typename T, int MODE>
__global__ void __launch_bounds__(TPB) k_scatter(T* __restrict__ cbar, const T* __restrict__ cstream,
                                                 const uint16_t* __restrict__ sym,
                                                 const int64_t* __restrict__ qside,
                                                 const double* __restrict__ bins, int level, int R,
                                                 LevelGeom<T> g, uint64_t nfine) {
  double b = MODE == 1 ? bins[level] : 0.0;
  for (uint64_t p = (uint64_t)blockIdx.x * TPB + threadIdx.x; p < nfine;
       p += (uint64_t)gridDim.x * TPB) {
    Coord c = unflatten(p, g);
    const int m = new_mask(c, g);
    if (m == 0) {
      cbar[p] = T(0);
      continue;
    }
    const uint64_t pos = stream_pos(c, m, g);
    cbar[p] = MODE == 0 ? cstream[pos] : dequantize_one<T>(sym, qside, pos, b, R);
  }
}

// Recomposition: u_l = c + Pi(uc) at new nodes, uc at coarse nodes.
template <typename T>
__global__ void __launch_bounds__(TPB) k_interp_add(T* __restrict__ out, const T* __restrict__ cbar,
                                                    const T* __restrict__ uc, LevelGeom<T> g,
                                                    uint64_t nfine) {
  for (uint64_t p = (uint64_t)blockIdx.x * TPB + threadIdx.x; p < nfine;
       p += (uint64_t)gridDim.x * TPB) {
    Coord c = unflatten(p, g);
    const int m = new_mask(c, g);
    if (m == 0) {
      uint64_t q = 0;
#pragma unroll
      for (int s = 0; s < MAXD; ++s) q = q * (uint64_t)g.nc[s] + (uint64_t)coarse_idx(c.i[s], s, g);
      out[p] = uc[q];
      continue;
    }
    out[p] = cbar[p] + interpolate<T, false>(uc, c, m, g);
  }
}

// Load vector + solves on cbar (grid l) -> z on grid l-1, written to `zout`.
// Uses two ping-pong buffers of at least count(l)/2 ... count(l) elements.
template <typename T>
void correction(const Hierarchy& h, int l, const T* table, const T* cbar, T* bufA, T* bufB,
                T** zout, hipStream_t st) {
  std::array<int64_t, MAXD> shp = h.sizes[l];
  const T* src = cbar;
  T* dst = bufA;
  for (int s = MAXD - 1; s >= 0; --s) {
    if (!h.active[s]) continue;
    uint64_t outer = 1, inner = 1;
    for (int q = 0; q < s; ++q) outer *= (uint64_t)shp[q];
    for (int q = s + 1; q < MAXD; ++q) inner *= (uint64_t)shp[q];
    const int nf = (int)shp[s], nc = (int)h.sizes[l - 1][s];
    const uint64_t total = outer * (uint64_t)nc * inner;
    KernelTimer kt(l == h.L ? "mass_restrict_fine" : "mass_restrict_coarse", st);
    MG_LAUNCH((&k_mass_restrict<T>), (k_mass_restrict_k<T>), (TPB), (0), (dim3(grid_for(total))), st, src, dst, outer, nf, nc, inner, dim_consts<T>(h, l, s, table));
    shp[s] = nc;
    src = dst;
    dst = (dst == bufA) ? bufB : bufA;
  }
  T* z = const_cast<T*>(src);
  for (int s = 0; s < MAXD; ++s) {
    if (!h.active[s]) continue;
    uint64_t outer = 1, inner = 1;
    for (int q = 0; q < s; ++q) outer *= (uint64_t)shp[q];
    for (int q = s + 1; q < MAXD; ++q) inner *= (uint64_t)shp[q];
    KernelTimer kt(l == h.L ? "thomas_fine" : "thomas_coarse", st);
    launch_thomas_any<T>(z, outer, (int)shp[s], inner, dim_consts<T>(h, l, s, table), st);
  }
  *zout = z;
}

struct Scratch {
  uint64_t cbar, pa, pb, ga, gb;  // element counts
};

Scratch scratch_counts(const Hierarchy& h) {
  Scratch s{};
  const int L = h.L;
  s.cbar = L >= 1 ? h.count(L) : 0;
  // restriction ping-pong: the first restriction halves (roughly) the finest grid
  uint64_t g = 0;
  for (int l = 1; l <= L; ++l) {
    std::array<int64_t, MAXD> shp = h.sizes[l];
    for (int q = MAXD - 1; q >= 0; --q) {
      if (!h.active[q]) continue;
      shp[q] = h.sizes[l - 1][q];
      uint64_t n = 1;
      for (int r = 0; r < MAXD; ++r) n *= (uint64_t)shp[r];
      g = std::max(g, n);
    }
  }
  s.ga = s.gb = g;
  s.pa = L >= 1 ? h.count(L - 1) : h.count(0);
  s.pb = L >= 2 ? h.count(L - 2) : h.count(0);
  return s;
}

}  // namespace

constexpr int SIDE_MAXDEV = 64;

void SideStream::fork(hipStream_t st) {
  static std::mutex mtx[SIDE_MAXDEV];
  static hipStream_t streams[SIDE_MAXDEV] = {};
  static hipEvent_t evs[SIDE_MAXDEV][2] = {};
  int dev = 0;
  MG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= SIDE_MAXDEV) fail(MGARD_ERR_DEVICE, "device index beyond the side-stream table");
  lk_ = std::unique_lock<std::mutex>(mtx[dev]);
  if (!streams[dev]) {
    MG_HIP(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
    MG_HIP(hipEventCreateWithFlags(&evs[dev][0], hipEventDisableTiming));
    MG_HIP(hipEventCreateWithFlags(&evs[dev][1], hipEventDisableTiming));
  }
  s = streams[dev];
  ef_ = evs[dev][0];
  ej_ = evs[dev][1];
  MG_HIP(hipEventRecord(ef_, st));
  MG_HIP(hipStreamWaitEvent(s, ef_, 0));
}

void SideStream::record_join() { MG_HIP(hipEventRecord(ej_, s)); }

void SideStream::join(hipStream_t st) {
  if (ej_) MG_HIP(hipStreamWaitEvent(st, ej_, 0));
}

template <typename T>
void launch_thomas_strided(T* data, uint64_t outer, int n, uint64_t inner, DimConsts<T> w, hipStream_t st) {
  MG_LAUNCH((&k_thomas<T>), (k_thomas_k<T>), (TPB), (0), (dim3(grid_for(outer * inner))), st, data, outer, n, inner, w.ta, w.tr, w.tcp);
}

template <typename T>
LevelGeom<T> level_geom(const Hierarchy& h, int l, const T* table) {
  LevelGeom<T> g{};
  g.pad_slots = MAXD - h.D;
  for (int s = 0; s < MAXD; ++s) {
    g.nf[s] = (int32_t)h.sizes[l][s];
    g.nc[s] = (int32_t)h.sizes[l - 1][s];
    g.act[s] = h.active[s] ? 1 : 0;
    g.wl[s] = h.active[s] ? table + h.devoff[l][s].wl : nullptr;
    g.wr[s] = h.active[s] ? table + h.devoff[l][s].wr : nullptr;
  }
  g.level_off = h.level_off[l];
  g.sub = static_cast<const uint64_t*>(h.dev_itab) + 80 * (uint64_t)l;
  return g;
}

template <typename T>
DimConsts<T> dim_consts(const Hierarchy& h, int l, int s, const T* t) {
  const DevDim& o = h.devoff[l][s];
  return DimConsts<T>{t + o.wl, t + o.wr, t + o.ma, t + o.mb, t + o.mc,
                      t + o.rl, t + o.rr, t + o.ta, t + o.tr, t + o.tcp};
}

template <typename T>
uint64_t decompose_scratch_bytes(const Hierarchy& h) {
  Scratch s = scratch_counts(h);
  return carve_size<T>(s.cbar) + carve_size<T>(s.pa) + carve_size<T>(s.pb) + carve_size<T>(s.ga) +
         carve_size<T>(s.gb) + 1024;
}

template <typename T>
uint64_t recompose_scratch_bytes(const Hierarchy& h) {
  return decompose_scratch_bytes<T>(h);
}

template <typename T>
void decompose(const Hierarchy& h, const T* table, const T* d_in, T* d_stream, const QuantOut* q,
               void* scratch, hipStream_t st, const std::function<void()>* fine_written) {
  bool fired = false;
  auto fire = [&] {
    if (fine_written && !fired) (*fine_written)();
    fired = true;
  };
  Scratch sc = scratch_counts(h);
  Carver cv(scratch);
  T* cbar = cv.take<T>(sc.cbar);
  T* pa = cv.take<T>(sc.pa);
  T* pb = cv.take<T>(sc.pb);
  T* ga = cv.take<T>(sc.ga);
  T* gb = cv.take<T>(sc.gb);
  const T* cur = d_in;
  T* nxt = pa;
  const int mode = q ? 1 : 0;
  const bool f3 = fused3d_ok<T>(h);
  const int lt = f3 ? fused3d_tail_levels<T>(h) : 0;  // levels 1..lt: one small-level kernel
  const std::function<void()> fire_fn = fire;
  for (int l = h.L; l > lt && f3; --l) {
    fused3d_decompose_level<T>(h, l, table, cur, nxt, ga, gb, q, d_stream, st, l == h.L ? &fire_fn : nullptr);
    cur = nxt;
    nxt = (nxt == pa) ? pb : pa;
  }
  if (lt > 0) {
    // the small levels and the coarsest grid
    fused3d_tail_decompose<T>(h, lt, table, cur, q, d_stream, st);
    fire();
    return;
  }
  for (int l = f3 ? 0 : h.L; l >= 1; --l) {
    LevelGeom<T> g = level_geom<T>(h, l, table);
    const uint64_t nfine = h.count(l);
    {
    KernelTimer kt(l == h.L ? "coeff_fine" : "coeff_coarse", st);
    if (mode == 0)
      MG_LAUNCH((&k_coeff<T, 0>), (k_coeff_k<T, 0>), (TPB), (0), (dim3(grid_for(nfine))), st, cur, cbar, nxt, d_stream, nullptr, nullptr, nullptr, l, 0, g, nfine);
    else
      MG_LAUNCH((&k_coeff<T, 1>), (k_coeff_k<T, 1>), (TPB), (0), (dim3(grid_for(nfine))), st, cur, cbar, nxt, nullptr, q->sym, q->qside, q->bins, l, q->R, g, nfine);
    }
    if (l == h.L) fire();
    T* z = nullptr;
    correction<T>(h, l, table, cbar, ga, gb, &z, st);
    const uint64_t nc = h.count(l - 1);
    KernelTimer kt(l == h.L ? "add_fine" : "add_coarse", st);
    MG_LAUNCH((&k_axpy<T, true>), (k_axpy_k<T, true>), (TPB), (0), (dim3(grid_for(nc))), st, nxt, nxt, z, nc);
    cur = nxt;
    nxt = (nxt == pa) ? pb : pa;
  }
  const uint64_t n0 = h.count(0);
  if (mode == 0)
    MG_LAUNCH((&k_coarsest_out<T, 0>), (k_coarsest_out_k<T, 0>), (TPB), (0), (dim3(grid_for(n0))), st, cur, d_stream, nullptr, nullptr, nullptr, 0, n0);
  else
    MG_LAUNCH((&k_coarsest_out<T, 1>), (k_coarsest_out_k<T, 1>), (TPB), (0), (dim3(grid_for(n0))), st, cur, nullptr, q->sym,
                       q->qside, q->bins, q->R, n0);
  MG_HIP(hipGetLastError());
  fire();
}

template <typename T>
void recompose(const Hierarchy& h, const T* table, const T* d_stream, const QuantOut* q, T* d_out,
               void* scratch, hipStream_t st) {
  Scratch sc = scratch_counts(h);
  Carver cv(scratch);
  T* cbar = cv.take<T>(sc.cbar);
  T* pa = cv.take<T>(sc.pa);
  T* pb = cv.take<T>(sc.pb);
  T* ga = cv.take<T>(sc.ga);
  T* gb = cv.take<T>(sc.gb);
  const int mode = q ? 1 : 0;
  const uint64_t n0 = h.count(0);
  // grid 0 goes where level 1 reads it; the last level writes d_out
  auto level_buf = [&](int l) -> T* {
    if (l == h.L) return d_out;
    return ((h.L - l) % 2 == 1) ? pa : pb;
  };
  const bool f3 = fused3d_ok<T>(h);
  const int lt = f3 ? fused3d_tail_levels<T>(h) : 0;  // levels 1..lt: one small-level kernel
  // The finest level's correction reads only the finest level's coefficients:
  // it runs on a side stream, into ga / gb, while the coarser levels recompose
  // on st with their solve scratch in the c-bar region (unused by the fused
  // levels) whenever that region holds it.
  T* cga = ga;
  T* cgb = gb;
  bool overlap = false;
  if (f3 && h.L > lt) {
    uint64_t g1c = 0;
    for (int l = lt + 1; l < h.L; ++l)
      g1c = std::max<uint64_t>(g1c, (uint64_t)h.sizes[l][1] * h.sizes[l - 1][2] * h.sizes[l - 1][3]);
    const uint64_t zc = h.L - 1 > lt ? h.count(h.L - 2) : 0;
    overlap = carve_size<T>(g1c) + carve_size<T>(zc) <= carve_size<T>(sc.cbar);
    if (overlap) {
      Carver cc(cbar);
      cga = cc.take<T>(g1c);
      cgb = cc.take<T>(zc);
    }
  }
  SideStream side;
  if (overlap) {
    side.fork(st);
    fused3d_recompose_correction<T>(h, h.L, table, ga, gb, q, d_stream, side.s);
    side.record_join();
  }
  T* cur = level_buf(lt);
  if (lt > 0)
    fused3d_tail_recompose<T>(h, lt, table, cur, q, d_stream, st);
  else if (mode == 0)
    hipLaunchKernelGGL((k_coarsest_in<T, 0>), dim3(grid_for(n0)), dim3(TPB), 0, st, cur, d_stream, nullptr,
                       nullptr, nullptr, 0, n0);
  else
    hipLaunchKernelGGL((k_coarsest_in<T, 1>), dim3(grid_for(n0)), dim3(TPB), 0, st, cur, nullptr, q->sym,
                       q->qside, q->bins, q->R, n0);
  for (int l = lt + 1; l <= h.L && f3; ++l) {
    T* out = level_buf(l);
    if (l == h.L && overlap) {
      side.join(st);
      fused3d_recompose_finish<T>(h, l, table, cur, out, gb, q, d_stream, st);
    } else {
      fused3d_recompose_level<T>(h, l, table, cur, out, cga, cgb, q, d_stream, st);
    }
    cur = out;
  }
  for (int l = f3 ? h.L + 1 : 1; l <= h.L; ++l) {
    LevelGeom<T> g = level_geom<T>(h, l, table);
    const uint64_t nfine = h.count(l);
    {
    KernelTimer kt(l == h.L ? "scatter_fine" : "scatter_coarse", st);
    if (mode == 0)
      hipLaunchKernelGGL((k_scatter<T, 0>), dim3(grid_for(nfine)), dim3(TPB), 0, st, cbar, d_stream, nullptr,
                         nullptr, nullptr, l, 0, g, nfine);
    else
      hipLaunchKernelGGL((k_scatter<T, 1>), dim3(grid_for(nfine)), dim3(TPB), 0, st, cbar, nullptr, q->sym,
                         q->qside, q->bins, l, q->R, g, nfine);
    }
    T* z = nullptr;
    correction<T>(h, l, table, cbar, ga, gb, &z, st);
    const uint64_t nc = h.count(l - 1);
    // uc = u_{l-1} - z, in place in z
    {
      KernelTimer kt(l == h.L ? "sub_fine" : "sub_coarse", st);
      MG_LAUNCH((&k_axpy<T, false>), (k_axpy_k<T, false>), (TPB), (0), (dim3(grid_for(nc))), st, z, cur, z, nc);
    }
    T* out = level_buf(l);
    KernelTimer kt(l == h.L ? "interp_add_fine" : "interp_add_coarse", st);
    hipLaunchKernelGGL(k_interp_add<T>, dim3(grid_for(nfine)), dim3(TPB), 0, st, out, cbar, z, g, nfine);
    cur = out;
  }
  if (h.L == 0 && cur != d_out) MG_HIP(hipMemcpyAsync(d_out, cur, n0 * sizeof(T), hipMemcpyDeviceToDevice, st));
  MG_HIP(hipGetLastError());
}

// The tuner runs the real level functions with each candidate forced, on the
// decomposition's own level grids (the finest is d_in), and keeps the fastest
// of three timed runs after a warm-up.  The level functions read their input
// and rewrite their outputs, so repeating them is harmless; the recomposition
// writes the finest level into the c-bar buffer, never into d_in.
template <typename T>
void fused3d_tune(const Hierarchy& h, const T* table, const T* d_in, const QuantOut* q, void* scratch,
                  hipStream_t st) {
  if (!fused3d_ok<T>(h) || h.L < 1) return;
  const bool f64 = sizeof(T) == 8;
  Scratch sc = scratch_counts(h);
  Carver cv(scratch);
  T* cbar = cv.take<T>(sc.cbar);
  T* pa = cv.take<T>(sc.pa);
  T* pb = cv.take<T>(sc.pb);
  T* ga = cv.take<T>(sc.ga);
  T* gb = cv.take<T>(sc.gb);
  hipEvent_t e0, e1;
  MG_HIP(hipEventCreate(&e0));
  MG_HIP(hipEventCreate(&e1));
  auto time_it = [&](auto&& run) -> float {
    run();
    MG_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < 3; ++r) run();
    MG_HIP(hipEventRecord(e1, st));
    MG_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    MG_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ms;
  };
  struct Reset {
    ~Reset() {
      tune_force(TUNE_COEFF_SEG, 0);
      tune_force(TUNE_SCATTER_PLANES, 0);
    }
  } reset;
  const T* cur = d_in;
  T* nxt = pa;
  for (int l = h.L; l >= 1; --l) {
    const int n0 = (int)h.sizes[l][1], n1 = (int)h.sizes[l][2], n2 = (int)h.sizes[l][3];
    const int c0 = (int)h.sizes[l - 1][1];
    int best = 1;
    float bt = 3.4e38f;
    for (int seg = 1; seg <= 16 && seg <= std::max(1, c0 - 1); seg *= 2) {
      tune_force(TUNE_COEFF_SEG, seg);
      const float t = time_it([&] { fused3d_decompose_level<T>(h, l, table, cur, nxt, ga, gb, q, nullptr, st); });
      if (t < bt) {
        bt = t;
        best = seg;
      }
    }
    tune_force(TUNE_COEFF_SEG, 0);
    tune_set(TUNE_COEFF_SEG, f64, n0, n1, n2, best);
    cur = nxt;
    nxt = (nxt == pa) ? pb : pa;
  }
  // cur holds the coarsest grid; recompose upwards
  for (int l = 1; l <= h.L; ++l) {
    const int n0 = (int)h.sizes[l][1], n1 = (int)h.sizes[l][2], n2 = (int)h.sizes[l][3];
    T* out = l == h.L ? cbar : (cur == pa ? pb : pa);
    int best = 8;
    float bt = 3.4e38f;
    for (int planes = 2; planes <= 16 && planes <= std::max(2, n0); planes *= 2) {
      tune_force(TUNE_SCATTER_PLANES, planes);
      const float t = time_it([&] { fused3d_recompose_level<T>(h, l, table, cur, out, ga, gb, q, nullptr, st); });
      if (t < bt) {
        bt = t;
        best = planes;
      }
    }
    tune_force(TUNE_SCATTER_PLANES, 0);
    tune_set(TUNE_SCATTER_PLANES, f64, n0, n1, n2, best);
    cur = out;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tune_save();
}

#define MG_INST(T)                                                                                    \
  template LevelGeom<T> level_geom<T>(const Hierarchy&, int, const T*);                             \
  template DimConsts<T> dim_consts<T>(const Hierarchy&, int, int, const T*);                        \
  template void launch_thomas_strided<T>(T*, uint64_t, int, uint64_t, DimConsts<T>, hipStream_t);   \
  template uint64_t decompose_scratch_bytes<T>(const Hierarchy&);                                   \
  template uint64_t recompose_scratch_bytes<T>(const Hierarchy&);                                   \
  template void fused3d_tune<T>(const Hierarchy&, const T*, const T*, const QuantOut*, void*, hipStream_t); \
  template void decompose<T>(const Hierarchy&, const T*, const T*, T*, const QuantOut*, void*,      \
                             hipStream_t, const std::function<void()>*);                            \
  template void recompose<T>(const Hierarchy&, const T*, const T*, const QuantOut*, T*, void*,      \
                             hipStream_t);
MG_INST(float)
MG_INST(double)
#undef MG_INST

}  // namespace mg
