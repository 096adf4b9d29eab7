// Fused 3D level kernels (gfx950): the same arithmetic, in the same rounding
// order, as the generic kernels of transform.hip, with fewer passes over HBM.
//
// Decomposition of one level (fine n0 x n1 x n2 -> coarse c0 x c1 x c2):
//   k3_coeff_r21   tiles of (dim 1, dim 2) marching over the fine planes of
//                  dim 0: in-plane interpolant (dim 2 sweep, then dim 1),
//                  plane interpolation along dim 0, coefficients, quantization
//                  of the owned nodes, coarse copy, then mass + restriction
//                  along dim 2 and dim 1 in LDS -> g1 (n0 x c1 x c2);
//   k3_r0_thomas0  mass + restriction along dim 0 fused with the Thomas solve
//                  along dim 0, one lane per (j1, j2) line -> z;
//   k_thomas       (generic) Thomas along dim 1;
//   k3_thomas2_axpy rows of the contiguous dimension staged in LDS, Thomas
//                  along dim 2, then u_{l-1} = u_l|coarse + z (or - z).
// Recomposition: k3_scatter_r21 (dequantize + restriction along dims 2, 1),
// the same solves, then k3_interp_add (dequantize + interpolant + add).
//
// Tiles start at even fine indices, so every new node inside a tile has both
// coarse neighbours inside the tile, and every fine index outside [0, n) is
// skipped.
#include <algorithm>

#include "internal.hpp"

namespace mg {

namespace {

constexpr int NT = 256;             // threads per block
constexpr int AXPY_LDS = 65536;     // bytes of LDS for the contiguous-dimension solve

__device__ inline bool is_new(int f, int n) { return (f & 1) && f < n - 1; }
__device__ inline int cidx(int f) { return (f + 1) >> 1; }          // coarse index of a coarse fine index
__device__ inline int cpos(int j, int nc, int nf) { return j == nc - 1 ? nf - 1 : 2 * j; }

template <typename T>
struct Lv3 {
  int n0, n1, n2, c0, c1, c2;
  DimConsts<T> d0, d1, d2;
  uint64_t level_off;
  const uint64_t* sub;  // sub-grid table of the level (slot layout: user dim d in slot d + 1)
};

// A block's copy of one dimension's weights in LDS: element i of the full
// array sits at p[i - off].
template <typename T>
struct OffArr {
  const T* p;
  int off;
  __device__ T operator[](int i) const { return p[i - off]; }
};
template <typename T>
struct TileW {
  OffArr<T> wl, wr, ma, mb, mc, rl, rr;
};

// Stages, for fine indices [F, F + NF) and coarse indices [J, J + NJ) of a
// dimension of fine size n and coarse size nc, the weights a tile reads into
// W (7 arrays: wl, wr, ma, mb, mc over NF, rl, rr over NJ); outside entries are 0.
template <typename T, int NF, int NJ>
__device__ inline TileW<T> stage_weights(T* W, const DimConsts<T>& d, int F, int J, int n, int nc) {
  for (int k = threadIdx.x; k < NF; k += blockDim.x) {
    const int f = F + k;
    const bool in = f >= 0 && f < n;
    W[k] = in ? d.wl[f] : T(0);
    W[NF + k] = in ? d.wr[f] : T(0);
    W[2 * NF + k] = in ? d.ma[f] : T(0);
    W[3 * NF + k] = in ? d.mb[f] : T(0);
    W[4 * NF + k] = in ? d.mc[f] : T(0);
  }
  for (int k = threadIdx.x; k < NJ; k += blockDim.x) {
    const int j = J + k;
    const bool in = j < nc;
    W[5 * NF + k] = in ? d.rl[j] : T(0);
    W[5 * NF + NJ + k] = in ? d.rr[j] : T(0);
  }
  TileW<T> w;
  w.wl = {W, F};
  w.wr = {W + NF, F};
  w.ma = {W + 2 * NF, F};
  w.mb = {W + 3 * NF, F};
  w.mc = {W + 4 * NF, F};
  w.rl = {W + 5 * NF, J};
  w.rr = {W + 5 * NF + NJ, J};
  return w;
}

// mass stencil of a line at fine index i: ((a*g[i-1] + b*g[i]) + c*g[i+1])
template <typename T, typename W, typename G>
__device__ inline T mass_at(int i, int n, const W& w, G g) {
  T s = w.mb[i] * g(i);
  if (i > 0) s = w.ma[i] * g(i - 1) + s;
  if (i < n - 1) s = s + w.mc[i] * g(i + 1);
  return s;
}

// restriction to coarse j of the mass-weighted line: ((rl*M[c-1] + M[c]) + rr*M[c+1])
template <typename T, typename W, typename G>
__device__ inline T restrict_at(int j, int nc, int n, const W& w, G g) {
  const int c = cpos(j, nc, n);
  T f = mass_at<T>(c, n, w, g);
  if (c >= 2 && !(c & 1)) f = w.rl[j] * mass_at<T>(c - 1, n, w, g) + f;
  if (!(c & 1) && c < n - 2) f = f + w.rr[j] * mass_at<T>(c + 1, n, w, g);
  return f;
}

// q = sign(y) * floor(|y| + 1/2), y = c / b in float64.  |q| < R is decided on
// the rounded magnitude, so the common case converts to 32 bits only; the
// 64-bit conversion is left to escapes.
template <typename T>
__device__ inline void quant_store(T c, double inv_b, int R, uint64_t pos, uint16_t* __restrict__ sym,
                                   int64_t* __restrict__ qside) {
  const double y = (double)c * inv_b;
  const double a = floor(fabs(y) + 0.5);
  if (a < (double)R) {
    const int qa = (int)a;
    sym[pos] = (uint16_t)(y < 0.0 ? R - qa : R + qa);
  } else {
    sym[pos] = 0;
    qside[pos] = (int64_t)(y < 0.0 ? -a : a);
  }
}

template <typename T>
__device__ inline T dequant_load(const uint16_t* __restrict__ sym, const int64_t* __restrict__ qside, uint64_t pos,
                                 double b, int R) {
  const uint16_t s = sym[pos];
  const double q = s ? (double)((int)s - R) : (double)qside[pos];
  return static_cast<T>(q * b);
}

// sub-grid offset and strides of the 7 masks, staged in LDS: [m][0] offset, [m][1..3] strides
__device__ inline void load_sub(uint64_t (*subs)[4], const uint64_t* sub, uint64_t level_off) {
  for (int k = threadIdx.x; k < 8 * 4; k += blockDim.x) {
    const int m = k >> 2, e = k & 3;
    subs[m][e] = m == 0 ? 0 : (e == 0 ? level_off + sub[m] : sub[16 + 4 * m + e]);
  }
}

// Stream position of the first element of fine row (f0, f1) in the sub-grid
// of dim-2 parity e2 (0: coarse along dim 2, 1: new); a coarse-coarse-coarse
// row has none (0).  Along the row, position = base + (e2 ? f2 >> 1 : cidx(f2)),
// the last dimension of every sub-grid being contiguous.
__device__ inline uint64_t row_base(const uint64_t (*subs)[4], int f0, int n0, int f1, int n1, int e2) {
  const bool e0 = is_new(f0, n0), e1 = is_new(f1, n1);
  const int m = (e0 ? 1 : 0) | (e1 ? 2 : 0) | (e2 ? 4 : 0);
  if (!m) return 0;
  const int i0 = e0 ? (f0 >> 1) : cidx(f0);
  const int i1 = e1 ? (f1 >> 1) : cidx(f1);
  return subs[m][0] + (uint64_t)i0 * subs[m][1] + (uint64_t)i1 * subs[m][2];
}

// ------------------------------------------------------------------ decomposition
// Tile layout of the plane-marching decomposition kernel: CY x CX coarse
// outputs in (dim 1, dim 2); FY x FX fine nodes with a halo of 2 before and 1
// after; rows of the LDS arrays are PX apart.  Thread t owns fine column
// t % 128 and half of the rows (t / 128), so every column quantity is a
// per-thread constant and every row quantity is uniform across a wavefront.
constexpr int CX = 62, CY = 8;
constexpr int FX = 2 * CX + 3, FY = 2 * CY + 3;  // 127 x 19
constexpr int PX = 128;                          // LDS row pitch of the fine tile
constexpr int HR = (FY + 1) / 2;                 // rows per half (10, then 9)

// Restriction weights of one coarse index, held in registers: the mass
// stencils at fine c-1, c, c+1 and the restriction terms, applied in the
// order of mass_at / restrict_at.
template <typename T>
struct RestrictW {
  int c = 0;
  bool l = false, r = false;
  T rl = 0, rr = 0;
  T a[3] = {0, 0, 0}, b[3] = {0, 0, 0}, d[3] = {0, 0, 0};
  bool hl[3] = {false, false, false}, hr[3] = {false, false, false};

  template <typename W>
  __device__ void load(int j, int nc, int n, const W& w) {
    c = cpos(j, nc, n);
    l = c >= 2 && !(c & 1);
    r = !(c & 1) && c < n - 2;
    // every load from an index clamped into range, issued before any is
    // used, then the values that do not apply are zeroed
    const T vrl = w.rl[j], vrr = w.rr[j];
    T vb[3], va[3], vd[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int i = min(max(c - 1 + k, 0), n - 1);
      vb[k] = w.mb[i];
      va[k] = w.ma[i];
      vd[k] = w.mc[i];
    }
    rl = l ? vrl : T(0);
    rr = r ? vrr : T(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int i = c - 1 + k;
      const bool in = i >= 0 && i < n && (k == 1 || (k == 0 && l) || (k == 2 && r));
      hl[k] = in && i > 0;
      hr[k] = in && i < n - 1;
      b[k] = in ? vb[k] : T(0);
      a[k] = hl[k] ? va[k] : T(0);
      d[k] = hr[k] ? vd[k] : T(0);
    }
  }
  template <typename G>
  __device__ T apply(G g) const {
    auto M = [&](int k) {
      const int i = c - 1 + k;
      T s = b[k] * g(i);
      if (hl[k]) s = a[k] * g(i - 1) + s;
      if (hr[k]) s = s + d[k] * g(i + 1);
      return s;
    };
    T f = M(1);
    if (l) f = rl * M(0) + f;
    if (r) f = f + rr * M(2);
    return f;
  }
};

// MODE 1: quantize into sym/qside; MODE 0: write float coefficients to cstream.
template <typename T, int MODE>
__device__ __forceinline__ void k3_coeff_r21(G3 mg_bid, G3 mg_gdim, const T* __restrict__ u, T* __restrict__ ucoarse,
                                                   T* __restrict__ g1, uint16_t* __restrict__ sym,
                                                   int64_t* __restrict__ qside, T* __restrict__ cstream,
                                                   const double* __restrict__ bins, int level, int R, const Lv3<T>& p,
                                                   int seg, const T* __restrict__ d0wl, const T* __restrict__ d0wr) {
  __shared__ T U[FY * PX];
  __shared__ T BA[FY * PX];
  __shared__ T BB[FY * PX];
  __shared__ T W1s[5 * FY + 2 * CY];
  __shared__ uint64_t subs[8][4];
  __shared__ uint64_t rb[FY][2];  // stream row bases of the committed plane (dim-2 parity 0 / 1)
  __shared__ uint64_t ucb[FY];    // coarse-grid row offsets of the committed plane
  const int t = threadIdx.x;
  const int J1 = mg_bid.y * CY, J2 = mg_bid.x * CX;
  const int F1 = 2 * J1 - 2, F2 = 2 * J2 - 2;
  const int n0 = p.n0, n1 = p.n1, n2 = p.n2;
  const int cb = mg_bid.z * seg;
  const int ce = min(cb + seg, p.c0 - 1);
  const uint64_t plane = (uint64_t)n1 * n2;
  const int o1b = 2 * J1, o1e = min(2 * (J1 + CY), n1);  // owned fine rows
  double inv_b = 0.0;
  if (MODE == 1) inv_b = 1.0 / bins[level];
  load_sub(subs, p.sub, p.level_off);
  const TileW<T> w1 = stage_weights<T, FY, CY>(W1s, p.d1, F1, J1, n1, p.c1);

  // this thread's column and rows
  // h and g4 are the same for every lane of a wavefront (128 and 64 lanes per
  // value): made scalar, every row quantity below is a scalar too
  const int x = t & (PX - 1), h = __builtin_amdgcn_readfirstlane(t >> 7);
  const int r0 = h * HR, nr = h ? FY - HR : HR;
  const int f2 = F2 + x;
  const bool colok = x < FX && f2 >= 0 && f2 < n2;
  const bool e2 = colok && is_new(f2, n2);
  const T wl2 = e2 ? p.d2.wl[f2] : T(0), wr2 = e2 ? p.d2.wr[f2] : T(0);
  const bool own2 = colok && f2 >= 2 * J2 && f2 < min(2 * (J2 + CX), n2);
  const uint64_t i2 = e2 ? (uint64_t)(f2 >> 1) : (uint64_t)cidx(f2);
  const int f2c = min(max(f2, 0), n2 - 1);
  // this thread's restriction along dim 2: coarse column jx, rows g, g+4, ...
  const int jx = t & 63, g4 = __builtin_amdgcn_readfirstlane(t >> 6);
  const int j2 = J2 + jx;
  const bool ok2 = jx < CX && j2 < p.c2;
  // every lane loads the weights of a column inside the tile (its own, or the
  // tile's last for lanes past it), so the dim-2 restriction runs unguarded
  // in LDS; only the g1 store is masked by ok2
  RestrictW<T> rw2;
  rw2.load(min(J2 + min(jx, CX - 1), p.c2 - 1), p.c2, n2, p.d2);
  // Row tests as bit masks (the same for every lane of a wavefront): bit j of
  // m_in: row r0 + j lies in the grid; m_new: it is a new row along dim 1;
  // m_own: the block owns it; bit k of m_r2: restriction row g4 + 4k lies in
  // the grid.  The plane loop reads them through an empty asm that claims to
  // change them, so the tests are made where they are used instead of being
  // hoisted out of the loop as one scalar register pair each.
  uint32_t m_in = 0, m_new = 0, m_own = 0, m_r2 = 0;
#pragma unroll
  for (int j = 0; j < HR; ++j) {
    const int f1 = F1 + r0 + j;
    const bool in = j < nr && f1 >= 0 && f1 < n1;
    m_in |= in ? 1u << j : 0u;
    m_new |= in && is_new(f1, n1) ? 1u << j : 0u;
    m_own |= in && f1 >= o1b && f1 < o1e ? 1u << j : 0u;
  }
  constexpr int R2N = (FY + 3) / 4;
#pragma unroll
  for (int k = 0; k < R2N; ++k) {
    const int r = g4 + 4 * k, f1 = F1 + r;
    m_r2 |= r < FY && f1 >= 0 && f1 < n1 ? 1u << k : 0u;
  }
  m_in = __builtin_amdgcn_readfirstlane(m_in);
  m_new = __builtin_amdgcn_readfirstlane(m_new);
  m_own = __builtin_amdgcn_readfirstlane(m_own);
  m_r2 = __builtin_amdgcn_readfirstlane(m_r2);
  auto bit = [](uint32_t m, int j) { return ((m >> j) & 1u) != 0u; };

  // The next plane is loaded into registers while the current one is
  // processed: unconditional loads from clamped addresses, zeroed outside the
  // grid when committed, so no register is written between a load and its use.
  T pre[HR];
  int row0 = F1 + r0;  // first fine row of this thread (scalar)
  auto prefetch = [&](int f0) {
#pragma unroll
    for (int j = 0; j < HR; ++j) {
      const int f1 = min(max(row0 + j, 0), n1 - 1);
      pre[j] = u[(uint64_t)f0 * plane + (uint64_t)f1 * n2 + f2c];
    }
  };
  auto commit = [&](int f0) {
#pragma unroll
    for (int j = 0; j < HR; ++j)
      if (j < nr) U[(r0 + j) * PX + x] = bit(m_in, j) ? pre[j] : T(0);

    if (t < FY) {
      const int f1 = F1 + t;
      const bool in = f1 >= 0 && f1 < n1;
      rb[t][0] = in ? row_base(subs, f0, n0, f1, n1, 0) : 0;
      rb[t][1] = in ? row_base(subs, f0, n0, f1, n1, 1) : 0;
      ucb[t] = in && !is_new(f0, n0) && !is_new(f1, n1) ? ((uint64_t)cidx(f0) * p.c1 + cidx(f1)) * p.c2 : 0;
    }
    __syncthreads();
  };
  // in-plane interpolant of the coarse-coarse nodes: dim 2 on coarse rows, then dim 1
  auto build_b = [&](T* B) {
#pragma unroll
    for (int j = 0; j < HR; ++j) {
      const int r = r0 + j;
      if (!bit(m_in & ~m_new, j)) continue;
      const int k = r * PX + x;
      B[k] = e2 ? wl2 * U[k - 1] + wr2 * U[k + 1] : U[k];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < HR; ++j) {
      const int r = r0 + j, f1 = F1 + r;
      if (!bit(m_new, j)) continue;
      const int k = r * PX + x;
      B[k] = w1.wl[f1] * B[k - PX] + w1.wr[f1] * B[k + PX];
    }
    __syncthreads();
  };
  // coefficients of plane f0 into U, outputs of the owned nodes, then R2 and R1 -> g1
  auto emit = [&](int f0, const T* Bl, const T* Br) {
    const bool new0 = is_new(f0, n0);
    const T w0l = new0 ? d0wl[f0] : T(0), w0r = new0 ? d0wr[f0] : T(0);
#pragma unroll
    for (int j = 0; j < HR; ++j) {
      const int r = r0 + j;
      if (!bit(m_in, j)) continue;
      const int k = r * PX + x;
      const T v = U[k];
      const T pi = new0 ? w0l * Bl[k] + w0r * Br[k] : Bl[k];
      const T c = v - pi;
      U[k] = c;
      if (!bit(m_own, j) || !own2) continue;
      const bool e1 = bit(m_new, j);
      if (!new0 && !e1 && !e2) {
        ucoarse[ucb[r] + (uint64_t)cidx(f2)] = v;
      } else {
        const uint64_t pos = rb[r][e2 ? 1 : 0] + i2;
        if (MODE == 1)
          quant_store(c, inv_b, R, pos, sym, qside);
        else
          cstream[pos] = c;
      }
    }
    __syncthreads();
    // mass + restriction along dim 2 for every row of the tile, held in
    // registers until every lane is done reading U, then stored in U's place
    // (rows of 64: G2[r * 64 + jx])
    T g2v[R2N];
#pragma unroll
    for (int k = 0; k < R2N; ++k) {
      const int r = g4 + 4 * k;
      g2v[k] = T(0);
      if (bit(m_r2, k)) {
        const T* row = U + r * PX - F2;  // row[f2] for fine f2 inside the tile
        g2v[k] = rw2.apply([&](int i) { return row[i]; });
      }
    }
    __syncthreads();
    T* G2 = U;
#pragma unroll
    for (int k = 0; k < R2N; ++k) {
      const int r = g4 + 4 * k;
      if (bit(m_r2, k)) G2[r * 64 + jx] = g2v[k];
    }
    __syncthreads();
    // mass + restriction along dim 1 -> g1
    for (int jy = g4; jy < CY; jy += 4) {
      const int j1 = J1 + jy;
      if (j1 >= p.c1 || !ok2) continue;
      const T* col = G2 + jx - F1 * 64;  // col[f1 * 64]
      const T f = restrict_at<T>(j1, p.c1, n1, w1, [&](int i) { return col[i * 64]; });
      g1[((uint64_t)f0 * p.c1 + j1) * p.c2 + j2] = f;
    }
    __syncthreads();
  };

  // Planes of the segment in order: the first coarse plane, then per interval
  // j its closing coarse plane (kind 1) and, when the interval has one, its new
  // plane (kind 2).  Kind 1 planes build the right interpolant; a new plane
  // uses the left and right ones; the two swap when an interval is done.
  auto task_at = [&](int j, int phase, int& plane, int& kind, int& tj) -> bool {
    while (j < ce) {
      const int fcj = cpos(j, p.c0, n0), fnj = cpos(j + 1, p.c0, n0);
      if (phase == 0) {
        plane = fnj, kind = 1, tj = j;
        return true;
      }
      if (fnj - fcj == 2) {
        plane = fcj + 1, kind = 2, tj = j;
        return true;
      }
      ++j;
      phase = 0;
    }
    return false;
  };
  T* Bp = BA;
  T* Bn = BB;
  int cplane = cpos(cb, p.c0, n0), ckind = 0, cj = cb;
  int nj = cb, nph = 0;
  __syncthreads();  // subs and the staged weights are visible to all threads
  prefetch(cplane);
  commit(cplane);
  while (true) {
    asm volatile("" : "+s"(m_in), "+s"(m_new), "+s"(m_own), "+s"(m_r2), "+s"(row0));
    if (ckind != 2) build_b(ckind == 0 ? Bp : Bn);
    int xplane = 0, xkind = 0, xj = 0;
    const bool more = task_at(nj, nph, xplane, xkind, xj);
    if (more) prefetch(xplane);
    if (ckind == 0)
      emit(cplane, Bp, Bp);
    else if (ckind == 1) {
      if (cj + 1 < ce || cj + 1 == p.c0 - 1) emit(cplane, Bn, Bn);
    } else {
      emit(cplane, Bp, Bn);
    }
    const bool interval_done =
        ckind == 2 || (ckind == 1 && cpos(cj + 1, p.c0, n0) - cpos(cj, p.c0, n0) == 1);
    if (interval_done) {
      T* tmp = Bp;
      Bp = Bn;
      Bn = tmp;
    }
    if (!more) break;
    if (xkind == 1) {
      nj = xj;
      nph = 1;
    } else {
      nj = xj + 1;
      nph = 0;
    }
    commit(xplane);
    cplane = xplane, ckind = xkind, cj = xj;
  }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 2))) k3_coeff_r21_k(const T* __restrict__ u, T* __restrict__ ucoarse,
                                                   T* __restrict__ g1, uint16_t* __restrict__ sym,
                                                   int64_t* __restrict__ qside, T* __restrict__ cstream,
                                                   const double* __restrict__ bins, int level, int R, Lv3<T> p,
                                                   int seg, const T* __restrict__ d0wl, const T* __restrict__ d0wr) {
  k3_coeff_r21<T, MODE>(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, u, ucoarse, g1, sym, qside, cstream, bins, level, R, p, seg, d0wl, d0wr);
}


// ------------------------------------------------------------------ decomposition, register tiles (float)
// The float form of the plane-marching decomposition: one wavefront per tile
// and no barriers.  Lane i holds fine columns e = F2 + 2i and e + 1 (F2 =
// 2 J2 - 2) of the tile's RX fine rows in registers: the current plane, the
// next plane (in flight), and the in-plane interpolants of the two coarse
// planes around the current interval.  Neighbouring columns come from the
// adjacent lanes by DPP wavefront shifts, neighbouring rows are registers of
// the same lane.  The planes of one dim-0 segment are visited as in
// k3_coeff_r21, and the arithmetic and its order are those of k3_coeff_r21.
constexpr int RX = 11;    // fine rows per tile: 8 owned, 2 before, 1 after
constexpr int RCY = 4;    // coarse rows (dim-1 outputs) per tile
constexpr int RCX = 62;   // coarse columns (dim-2 outputs) per tile: lanes 1..62
constexpr int RWAVE = 64;

// x of lane i + 1 (0 for lane 63) and of lane i - 1 (0 for lane 0): DPP
// wavefront shifts, every lane active
__device__ inline float lane_next(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xf, 0xf, true));  // wave_shl:1
}
__device__ inline float lane_prev(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xf, 0xf, true));  // wave_shr:1
}

// Tiles in XCD order: consecutive workgroups go to the eight XCDs in turn, so
// block b takes tile (b mod 8) q + b / 8 (q = ceil(tiles / 8)): each XCD gets
// a run of tiles adjacent along dim 1, whose shared halo rows its L2 then
// holds.  Tiles are numbered dim 1 fastest, then dim 2, then the segment.
__device__ inline bool reg_tile(uint32_t b, int nt1, int nt2, int nseg, int& t1, int& t2, int& sg) {
  const uint32_t nb = (uint32_t)nt1 * (uint32_t)nt2 * (uint32_t)nseg;
  const uint32_t q8 = (nb + 7) / 8;
  const uint32_t t = (b % 8) * q8 + b / 8;
  if (t >= nb) return false;
  t1 = (int)(t % (uint32_t)nt1);
  t2 = (int)((t / (uint32_t)nt1) % (uint32_t)nt2);
  sg = (int)(t / ((uint32_t)nt1 * (uint32_t)nt2));
  return true;
}

// Column and row quantities of a register tile, and the mass + restriction
// of a plane's coefficients along dims 2 and 1 with the arithmetic of
// RestrictW::apply and restrict_at.  Wr and Wk are the tile's dim-1 weights,
// staged in LDS by init.
struct RTile {
  int n1, n2, c1, c2, J1, J2, F1, F2, lane, e, o, pc, j2;
  bool ein, oin, inner, own_e, own_o, onew, eshift, out2, rshift, full2;
  uint64_t colidx;
  float wl2, wr2;  // interpolation weights of column o (0 unless o is new)
  RestrictW<float> rw;
  uint32_t m_in, m_new, k_ok, k_odd, k_l, k_r;

  __device__ void init(const Lv3<float>& p, int tile1, int tile2, float (&Wr)[5][RX], float (&Wk)[2][RCY]) {
    n1 = p.n1, n2 = p.n2, c1 = p.c1, c2 = p.c2;
    J1 = tile1 * RCY, J2 = tile2 * RCX;
    F1 = 2 * J1 - 2, F2 = 2 * J2 - 2;
    // columns of this lane
    lane = threadIdx.x;
    e = F2 + 2 * lane, o = e + 1;
    ein = e >= 0 && e < n2;
    oin = e >= 0 && o < n2;
    inner = lane >= 1 && lane <= RCX;  // owned fine columns [2 J2, 2 J2 + 124)
    own_e = inner && ein, own_o = inner && oin;
    onew = oin && o < n2 - 1;  // o is new along dim 2 (else the last column, coarse)
    eshift = e == n2 - 1;      // e is the last column: the loaded pair starts one before
    pc = min(max(e, 0), n2 - 2);
    const int oc = min(max(o, 0), n2 - 1);
    const float wl2v = p.d2.wl[oc], wr2v = p.d2.wr[oc];
    wl2 = onew ? wl2v : 0.f, wr2 = onew ? wr2v : 0.f;
    colidx = e >= 0 ? (uint64_t)(e >> 1) : 0;  // cidx(e) = e / 2 = o >> 1
    // restriction along dim 2: this lane's coarse column j2 = J2 - 1 + lane
    j2 = J2 - 1 + lane;
    out2 = inner && j2 < c2;
    rw.load(min(max(j2, 0), c2 - 1), c2, n2, p.d2);
    rshift = out2 && rw.c == e - 1;  // the last coarse column of an even side sits at e - 1
    // the whole wavefront on the interior path: every output lane, and lane
    // 0, away from the grid's sides
    const bool interior2 = (!out2 && lane != 0) || (!rshift && rw.l && rw.r && rw.hl[0] && rw.hl[1] &&
                                                    rw.hl[2] && rw.hr[0] && rw.hr[1] && rw.hr[2]);
    full2 = __builtin_amdgcn_ballot_w64(interior2) == __builtin_amdgcn_read_exec();
    // rows of the tile (the same for every lane)
    m_in = 0, m_new = 0;
#pragma unroll
    for (int r = 0; r < RX; ++r) {
      const int f1 = F1 + r;
      const bool in = f1 >= 0 && f1 < n1;
      m_in |= in ? 1u << r : 0u;
      m_new |= in && is_new(f1, n1) ? 1u << r : 0u;
    }
    m_in = __builtin_amdgcn_readfirstlane(m_in);
    m_new = __builtin_amdgcn_readfirstlane(m_new);
    if (lane < RX) {
      const int r = lane, f1c = min(max(F1 + r, 0), n1 - 1);
      const float vl = p.d1.wl[f1c], vr = p.d1.wr[f1c], va = p.d1.ma[f1c], vb = p.d1.mb[f1c], vc = p.d1.mc[f1c];
      const bool nw = ((m_new >> r) & 1u) != 0u, in = ((m_in >> r) & 1u) != 0u;
      Wr[0][r] = nw ? vl : 0.f;
      Wr[1][r] = nw ? vr : 0.f;
      Wr[2][r] = in ? va : 0.f;
      Wr[3][r] = in ? vb : 0.f;
      Wr[4][r] = in ? vc : 0.f;
    }
    k_ok = 0, k_odd = 0, k_l = 0, k_r = 0;
#pragma unroll
    for (int k = 0; k < RCY; ++k) {
      const int j1 = J1 + k;
      const int c = cpos(min(j1, c1 - 1), c1, n1);
      const bool ok = j1 < c1;
      k_ok |= ok ? 1u << k : 0u;
      k_odd |= ok && c != 2 * j1 ? 1u << k : 0u;  // centre at tile row 2k + 1 instead of 2k + 2
      k_l |= ok && c >= 2 && !(c & 1) ? 1u << k : 0u;
      k_r |= ok && !(c & 1) && c < n1 - 2 ? 1u << k : 0u;
    }
    k_ok = __builtin_amdgcn_readfirstlane(k_ok);
    k_odd = __builtin_amdgcn_readfirstlane(k_odd);
    k_l = __builtin_amdgcn_readfirstlane(k_l);
    k_r = __builtin_amdgcn_readfirstlane(k_r);
    if (lane < RCY) {
      const int jc = min(J1 + lane, c1 - 1);
      Wk[0][lane] = p.d1.rl[jc];
      Wk[1][lane] = p.d1.rr[jc];
    }
  }
  __device__ static bool bit(uint32_t m, int j) { return ((m >> j) & 1u) != 0u; }

  // mass + restriction along dim 2 of every row of the tile: the window of
  // fine columns e - 2 .. e + 2 from this lane and its two neighbours
  __device__ void restrict2(const float (&cv)[RX][2], float (&g2)[RX]) const {
    if (full2) {  // every output lane (and lane 0) has both side terms and full stencils
#pragma unroll
      for (int r = 0; r < RX; ++r) {
        const float w1 = lane_prev(cv[r][1]), w4 = lane_next(cv[r][0]);
        const float w2 = cv[r][0], w3 = cv[r][1];
        auto M = [&](int k, float a, float b, float c) {
          float s = rw.b[k] * b;
          s = rw.a[k] * a + s;
          return s + rw.d[k] * c;
        };
        // the mass stencil at this lane's e - 1 is the one lane i - 1 takes at
        // its e + 1: same fine column, weights and values
        const float m1 = M(1, w1, w2, w3), m2 = M(2, w2, w3, w4);
        const float m0 = lane_prev(m2);
        float f = m1;
        f = rw.rl * m0 + f;
        g2[r] = f + rw.rr * m2;
      }
    } else {
#pragma unroll
      for (int r = 0; r < RX; ++r) {
        const float w0 = lane_prev(cv[r][0]), w1 = lane_prev(cv[r][1]), w4 = lane_next(cv[r][0]);
        const float w2 = cv[r][0], w3 = cv[r][1];
        const float gm = rshift ? w0 : w1, g0 = rshift ? w1 : w2, gp = rshift ? w2 : w3;
        auto M = [&](int k, float a, float b, float c) {
          float s = rw.b[k] * b;
          s = rw.hl[k] ? rw.a[k] * a + s : s;
          s = rw.hr[k] ? s + rw.d[k] * c : s;
          return s;
        };
        float f = M(1, gm, g0, gp);
        f = rw.l ? rw.rl * M(0, w0, w1, w2) + f : f;
        f = rw.r ? f + rw.rr * M(2, w2, w3, w4) : f;
        g2[r] = f;
      }
    }
  }
  // mass stencil of tile row r (fine row F1 + r inside the grid), on g
  __device__ float mass1(const float (&Wr)[5][RX], int r, const float (&g)[RX]) const {
    const int f1 = F1 + r;
    float s = Wr[3][r] * g[r];
    if (r > 0) s = f1 > 0 ? Wr[2][r] * g[r - 1] + s : s;
    if (r + 1 < RX) s = f1 < n1 - 1 ? s + Wr[4][r] * g[r + 1] : s;
    return s;
  }
  // mass + restriction along dim 1: coarse row J1 + k (k_ok bit set)
  __device__ float restrict1(const float (&Wr)[5][RX], const float (&Wk)[2][RCY], const float (&g2)[RX],
                             int k) const {
    float f;
    if (!bit(k_odd, k)) {
      const int c = 2 * k + 2;
      f = mass1(Wr, c, g2);
      if (bit(k_l, k)) f = Wk[0][k] * mass1(Wr, c - 1, g2) + f;
      if (bit(k_r, k)) f = f + Wk[1][k] * mass1(Wr, c + 1, g2);
    } else {
      f = mass1(Wr, 2 * k + 1, g2);  // an odd centre has neither side term
    }
    return f;
  }
};

template <int MODE>
__device__ __forceinline__ void k3_coeff_reg(G3 mg_bid, G3 mg_gdim, const float* __restrict__ u,
                                             float* __restrict__ ucoarse, float* __restrict__ g1,
                                             uint16_t* __restrict__ sym, int64_t* __restrict__ qside,
                                             float* __restrict__ cstream, const double* __restrict__ bins, int level,
                                             int R, const Lv3<float>& p, int seg, int nt1, int nt2, int nseg,
                                             const float* __restrict__ d0wl, const float* __restrict__ d0wr) {
  // in-plane interpolants of the interval's two coarse planes, lane-private
  // slots [plane][row][column][lane]; row weights of the tile
  __shared__ float Bs[2][RX][2][RWAVE];
  __shared__ float Wr[5][RX];   // dim 1: interpolation left/right (new rows), mass a/b/c (rows in the grid)
  __shared__ float Wk[2][RCY];  // dim 1: restriction left/right of coarse row J1 + k
  // stream positions: sub-grid m (bit 0: new along dim 0, bit 1: dim 1, bit 2:
  // dim 2) starts at row part + i0 * S0[m] for owned row r: Rb[r - 2][m]
  // holds its offset + i1 * (stride of i1); S0[m] the stride of i0
  __shared__ uint64_t Rb[2 * RCY][8];
  __shared__ uint64_t S0[8];
  int tile1, tile2, sgi;
  if (!reg_tile(mg_bid.x, nt1, nt2, nseg, tile1, tile2, sgi)) return;
  RTile T;
  T.init(p, tile1, tile2, Wr, Wk);
  const int n0 = p.n0, n1 = T.n1, n2 = T.n2, c1 = T.c1, c2 = T.c2;
  const int J1 = T.J1, F1 = T.F1;
  const int cb = sgi * seg;
  const int ce = min(cb + seg, p.c0 - 1);
  const uint64_t plane = (uint64_t)n1 * n2;
  double inv_b = 0.0;
  if (MODE == 1) inv_b = 1.0 / bins[level];
  const int lane = T.lane;
  const bool ein = T.ein, oin = T.oin, own_e = T.own_e, own_o = T.own_o, onew = T.onew, eshift = T.eshift;
  const int pc = T.pc;
  const float wl2 = T.wl2, wr2 = T.wr2;
  const uint64_t colidx = T.colidx;
  uint32_t m_in = T.m_in, m_new = T.m_new;
  auto bit = [](uint32_t m, int j) { return ((m >> j) & 1u) != 0u; };
  {
    // lane = 8 (r - 2) + m: the row part of owned row r in sub-grid m
    const int r = 2 + (lane >> 3), m = lane & 7;
    const int f1 = F1 + r;
    const bool e1 = is_new(min(max(f1, 0), n1 - 1), n1);
    const int i1 = e1 ? (f1 >> 1) : cidx(f1);
    const uint64_t off = m == 0 ? 0 : p.level_off + p.sub[m];
    const uint64_t s1 = p.sub[16 + 4 * m + 2];
    Rb[r - 2][m] = m == 0 ? 0 : off + (uint64_t)max(i1, 0) * s1;
    if (lane < 8) S0[lane] = lane == 0 ? 0 : p.sub[16 + 4 * lane + 1];
  }
  __syncthreads();

  // ---- plane registers
  float pre[RX][2];  // next plane, in flight
  float cur[RX][2];  // current plane (u), then its coefficients
  auto prefetch = [&](int f0) {
    const float* base = u + (uint64_t)f0 * plane + pc;
    // the clamped rows are recomputed here (scalar work), not held across
    // the plane loop in scalar registers
    int f1a = F1;
    asm volatile("" : "+s"(f1a));
#pragma unroll
    for (int r = 0; r < RX; ++r) {
      float2 v;
      const int rc = min(max(f1a + r, 0), n1 - 1);
      __builtin_memcpy(&v, base + (uint64_t)rc * n2, 8);
      pre[r][0] = v.x;
      pre[r][1] = v.y;
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int r = 0; r < RX; ++r) {
      const bool in = bit(m_in, r);
      cur[r][0] = in && ein ? (eshift ? pre[r][1] : pre[r][0]) : 0.f;
      cur[r][1] = in && oin ? pre[r][1] : 0.f;
    }
  };
  // quantization as in quant_store: the symbol is computed and stored by
  // every lane without a branch; only an escape takes one
  auto qstore = [&](float c, uint64_t pos) {
    if (MODE == 1) {
      const double y = (double)c * inv_b;
      const double a = floor(fabs(y) + 0.5);
      const bool esc = !(a < (double)R);
      const int qa = (int)fmin(a, (double)R);
      int sv = y < 0.0 ? R - qa : R + qa;
      sv = esc ? 0 : sv;
      asm volatile("" : "+v"(sv));
      sym[pos] = (uint16_t)sv;
      if (esc) qside[pos] = (int64_t)(y < 0.0 ? -a : a);
    } else {
      cstream[pos] = c;
    }
  };
  int bp = 0, bn = 1;  // slots of the left and right coarse planes' interpolants
  // Coarse plane: in-plane interpolant (dim 2 on the coarse rows, then dim 1)
  // into slot bn, and the coefficients u - interpolant in place of u.
  auto coarse_coeffs = [&](float (&cv)[RX][2]) {
    float B[RX][2];
#pragma unroll
    for (int r = 0; r < RX; ++r) {
      if (r % 2 == 1 && bit(m_new, r)) continue;
      const float nx = lane_next(cur[r][0]);
      B[r][0] = cur[r][0];
      B[r][1] = onew ? wl2 * cur[r][0] + wr2 * nx : cur[r][1];
    }
#pragma unroll
    for (int r = 1; r < RX; r += 2) {
      if (!bit(m_new, r)) continue;
      B[r][0] = Wr[0][r] * B[r - 1][0] + Wr[1][r] * B[r + 1][0];
      B[r][1] = Wr[0][r] * B[r - 1][1] + Wr[1][r] * B[r + 1][1];
    }
#pragma unroll
    for (int r = 0; r < RX; ++r) {
      Bs[bn][r][0][lane] = B[r][0];
      Bs[bn][r][1][lane] = B[r][1];
      cv[r][0] = cur[r][0] - B[r][0];
      cv[r][1] = cur[r][1] - B[r][1];
    }
  };
  // Outputs of the owned nodes of plane f0 (cur: u; cv: coefficients), then
  // mass + restriction along dims 2 and 1 of the coefficients -> g1.
  auto emit = [&](int f0, const float (&cv)[RX][2]) {
    const bool e0 = is_new(f0, n0);
    const int i0 = e0 ? (f0 >> 1) : cidx(f0);
    const uint64_t ucplane = (uint64_t)cidx(f0) * c1 * c2;
    // i0 * stride for the four sub-grids of this plane's dim-0 parity
    const int m0 = e0 ? 1 : 0;
    const uint64_t P00 = (uint64_t)i0 * S0[m0], P10 = (uint64_t)i0 * S0[m0 | 2];
    const uint64_t P01 = (uint64_t)i0 * S0[m0 | 4], P11 = (uint64_t)i0 * S0[m0 | 6];
#pragma unroll
    for (int r = 2; r < 2 + 2 * RCY; ++r) {
      if (!bit(m_in, r)) continue;
      const int f1 = F1 + r;
      const bool e1 = bit(m_new, r);
      const int m01 = m0 | (e1 ? 2 : 0);
      const uint64_t rb1 = Rb[r - 2][m01 | 4] + (e1 ? P11 : P01);
      if (!e0 && !e1) {  // coarse row of a coarse plane: e is a coarse node
        const uint64_t ucb = ucplane + (uint64_t)cidx(f1) * c2 + colidx;
        if (own_e) ucoarse[ucb] = cur[r][0];
        if (own_o) {
          if (onew)
            qstore(cv[r][1], rb1 + colidx);
          else
            ucoarse[ucb + 1] = cur[r][1];
        }
      } else {
        const uint64_t rb0 = Rb[r - 2][m01] + (e1 ? P10 : P00);
        if (own_e) qstore(cv[r][0], rb0 + colidx);
        if (own_o) qstore(cv[r][1], onew ? rb1 + colidx : rb0 + colidx + 1);
      }
    }
    // mass + restriction along dims 2 and 1 -> g1
    float g2[RX];
    T.restrict2(cv, g2);
    const uint64_t gplane = (uint64_t)f0 * c1;
#pragma unroll
    for (int k = 0; k < RCY; ++k) {
      if (!bit(T.k_ok, k)) continue;
      const float f = T.restrict1(Wr, Wk, g2, k);
      if (T.out2) g1[(gplane + (uint64_t)(J1 + k)) * c2 + T.j2] = f;
    }
  };

  // Planes of the segment, as in k3_coeff_r21: the first coarse plane, then
  // per interval j its closing coarse plane (kind 1) and, when the interval
  // has one, its new plane (kind 2).
  auto task_at = [&](int j, int phase, int& pl, int& kind, int& tj) -> bool {
    while (j < ce) {
      const int fcj = cpos(j, p.c0, n0), fnj = cpos(j + 1, p.c0, n0);
      if (phase == 0) {
        pl = fnj, kind = 1, tj = j;
        return true;
      }
      if (fnj - fcj == 2) {
        pl = fcj + 1, kind = 2, tj = j;
        return true;
      }
      ++j;
      phase = 0;
    }
    return false;
  };
  int cplane = cpos(cb, p.c0, n0), ckind = 0, cj = cb;
  int nj = cb, nph = 0;
  prefetch(cplane);
  commit();
  while (true) {
    asm volatile("" : "+s"(m_in), "+s"(m_new));
    int xplane = 0, xkind = 0, xj = 0;
    const bool more = task_at(nj, nph, xplane, xkind, xj);
    if (more) prefetch(xplane);
    float cv[RX][2];
    if (ckind != 2) {
      coarse_coeffs(cv);
    } else {
      const float w0l = d0wl[cplane], w0r = d0wr[cplane];
#pragma unroll
      for (int r = 0; r < RX; ++r)
#pragma unroll
        for (int k = 0; k < 2; ++k) cv[r][k] = cur[r][k] - (w0l * Bs[bp][r][k][lane] + w0r * Bs[bn][r][k][lane]);
    }
    // a closing coarse plane that opens the next segment is that segment's
    // (except the grid's last plane); the interval is done after its new
    // plane, or after its closing plane when it has none, and the segment's
    // first plane is the left plane of its first interval
    const bool mine = ckind != 1 || cj + 1 < ce || cj + 1 == p.c0 - 1;
    const bool done = ckind != 1 || cpos(cj + 1, p.c0, n0) - cpos(cj, p.c0, n0) == 1;
    if (mine) emit(cplane, cv);
    if (done) {
      const int t = bp;
      bp = bn;
      bn = t;
    }
    if (!more) break;
    if (xkind == 1) {
      nj = xj;
      nph = 1;
    } else {
      nj = xj + 1;
      nph = 0;
    }
    commit();
    cplane = xplane, ckind = xkind, cj = xj;
  }
}

template <int MODE>
__global__ void __launch_bounds__(RWAVE) k3_coeff_reg_k(const float* __restrict__ u, float* __restrict__ ucoarse,
                                                        float* __restrict__ g1, uint16_t* __restrict__ sym,
                                                        int64_t* __restrict__ qside, float* __restrict__ cstream,
                                                        const double* __restrict__ bins, int level, int R, Lv3<float> p,
                                                        int seg, int nt1, int nt2, int nseg,
                                                        const float* __restrict__ d0wl,
                                                        const float* __restrict__ d0wr) {
  k3_coeff_reg<MODE>(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, u, ucoarse, g1, sym,
                     qside, cstream, bins, level, R, p, seg, nt1, nt2, nseg, d0wl, d0wr);
}

// mass + restriction along dim 0 of g1 (n0 x c1 x c2), then Thomas along dim 0 -> z (c0 x c1 x c2).
// One lane per (j1, j2) line.  Both sweeps run in groups of SWEEP coarse
// indices whose loads are all issued before the group's recurrence, so a
// lane waits for memory once per group rather than once per index; the
// arithmetic and its order are those of the plain loops.  Eight indices per
// group measured fastest: longer groups hold more rows in registers and, on
// the short lines of the coarse levels, load more clamped rows that no index
// uses; shorter ones wait for memory more often.
constexpr int SWEEP = 8;

// The weights come as separate restrict pointers: the compiler then knows the
// stores to z leave them alone and reads them with scalar loads.
template <typename T>
__device__ __forceinline__ void k3_r0_thomas0(G3 mg_bid, G3 mg_gdim, const T* __restrict__ g1, T* __restrict__ z, int n0, int c0,
                                                    uint64_t lines, const T* __restrict__ w_ma,
                                                    const T* __restrict__ w_mb, const T* __restrict__ w_mc,
                                                    const T* __restrict__ w_rl, const T* __restrict__ w_rr,
                                                    const T* __restrict__ w_ta, const T* __restrict__ w_tr,
                                                    const T* __restrict__ w_tcp) {
  struct {
    const T *ma, *mb, *mc, *rl, *rr, *ta, *tr, *tcp;
  } w{w_ma, w_mb, w_mc, w_rl, w_rr, w_ta, w_tr, w_tcp};
  const uint64_t t = (uint64_t)mg_bid.x * NT + threadIdx.x;
  if (t >= lines) return;
  const T* g = g1 + t;
  T* zz = z + t;
  T prev = T(0);
  // coarse j < c0 - 1 sits at fine 2j: it reads fine rows 2j-2 .. 2j+2
  const int jend = c0 - 1;
  // fine rows of the group starting at coarse j0, from row indices clamped
  // into the grid: every load is unconditional, so the wait before a group
  // covers only the older group's loads (a load under a branch makes the
  // compiler wait for all of them).  The sweeps read only rows whose fine
  // index lies in the grid, so the clamped copies are never used.
  auto load_rows = [&](int j0, T* rows) {
    const int r0 = 2 * j0 - 2;
#pragma unroll
    for (int q = 0; q < 2 * SWEEP + 3; ++q) {
      const int r = min(max(r0 + q, 0), n0 - 1);
      rows[q] = g[(uint64_t)r * lines];
    }
  };
  auto forward = [&](int j0, const T* rows) {
    // interior group: every neighbour exists, so the group is one straight
    // block whose weight loads can be issued together (same arithmetic)
    if (j0 >= 1 && j0 + SWEEP - 1 < jend && 2 * (j0 + SWEEP - 1) < n0 - 2) {
#pragma unroll
      for (int u = 0; u < SWEEP; ++u) {
        const int j = j0 + u;
        auto M = [&](int d) -> T {
          const int i = 2 * j + d;
          T s = w.mb[i] * rows[2 * u + 2 + d];
          s = w.ma[i] * rows[2 * u + 1 + d] + s;
          return s + w.mc[i] * rows[2 * u + 3 + d];
        };
        T f = M(0);
        f = w.rl[j] * M(-1) + f;
        f = f + w.rr[j] * M(1);
        prev = (f - w.ta[j] * prev) * w.tr[j];
        zz[(uint64_t)j * lines] = prev;
      }
      return;
    }
#pragma unroll
    for (int u = 0; u < SWEEP; ++u) {
      const int j = j0 + u;
      if (j < jend) {
        // mass_at and restrict_at for c = 2j, rows[q] holding fine row 2*j0 - 2 + q
        auto M = [&](int d) -> T {
          const int i = 2 * j + d;
          T s = w.mb[i] * rows[2 * u + 2 + d];
          if (i > 0) s = w.ma[i] * rows[2 * u + 1 + d] + s;
          if (i < n0 - 1) s = s + w.mc[i] * rows[2 * u + 3 + d];
          return s;
        };
        T f = M(0);
        if (j >= 1) f = w.rl[j] * M(-1) + f;
        if (2 * j < n0 - 2) f = f + w.rr[j] * M(1);
        prev = j == 0 ? f * w.tr[0] : (f - w.ta[j] * prev) * w.tr[j];
        zz[(uint64_t)j * lines] = prev;
      }
    }
  };
  // two row buffers: the next group's loads are issued before this group's recurrence
  {
    T ra[2 * SWEEP + 3], rb[2 * SWEEP + 3];
    load_rows(0, ra);
    for (int j0 = 0; j0 < jend; j0 += 2 * SWEEP) {
      load_rows(j0 + SWEEP, rb);
      forward(j0, ra);
      load_rows(j0 + 2 * SWEEP, ra);
      forward(j0 + SWEEP, rb);
    }
  }
  {
    const int j = jend;
    auto G = [&](int i) { return g[(uint64_t)i * lines]; };
    DimConsts<T> dc{};
    dc.ma = w.ma;
    dc.mb = w.mb;
    dc.mc = w.mc;
    dc.rl = w.rl;
    dc.rr = w.rr;
    const T f = restrict_at<T>(j, c0, n0, dc, G);
    prev = j == 0 ? f * w.tr[0] : (f - w.ta[j] * prev) * w.tr[j];
    zz[(uint64_t)j * lines] = prev;
  }
  T x = prev;
  auto load_z = [&](int j1, T* v) {  // clamped and unconditional, as above
#pragma unroll
    for (int u = 0; u < SWEEP; ++u) {
      const int j = max(j1 - u, 0);
      v[u] = zz[(uint64_t)j * lines];
    }
  };
  auto backward = [&](int j1, const T* v) {
    if (j1 - (SWEEP - 1) >= 0) {
#pragma unroll
      for (int u = 0; u < SWEEP; ++u) {
        const int j = j1 - u;
        x = v[u] - w.tcp[j] * x;
        zz[(uint64_t)j * lines] = x;
      }
      return;
    }
#pragma unroll
    for (int u = 0; u < SWEEP; ++u) {
      const int j = j1 - u;
      if (j >= 0) {
        x = v[u] - w.tcp[j] * x;
        zz[(uint64_t)j * lines] = x;
      }
    }
  };
  {
    T va[SWEEP], vb[SWEEP];
    load_z(c0 - 2, va);
    for (int j1 = c0 - 2; j1 >= 0; j1 -= 2 * SWEEP) {
      load_z(j1 - SWEEP, vb);
      backward(j1, va);
      load_z(j1 - 2 * SWEEP, va);
      backward(j1 - SWEEP, vb);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(NT) k3_r0_thomas0_k(const T* __restrict__ g1, T* __restrict__ z, int n0, int c0,
                                                    uint64_t lines, const T* __restrict__ w_ma,
                                                    const T* __restrict__ w_mb, const T* __restrict__ w_mc,
                                                    const T* __restrict__ w_rl, const T* __restrict__ w_rr,
                                                    const T* __restrict__ w_ta, const T* __restrict__ w_tr,
                                                    const T* __restrict__ w_tcp) {
  k3_r0_thomas0<T>(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, g1, z, n0, c0, lines, w_ma, w_mb, w_mc, w_rl, w_rr, w_ta, w_tr, w_tcp);
}


// Thomas along the contiguous dimension on `rows` rows per block, then out = a +/- z.
// The weights are restrict pointers (scalar loads); the sweeps are unrolled
// so that their LDS reads and weight loads are issued ahead of the recurrence.
// Each lane loads all of its EPT elements of the block's rows (clamped
// indices, unconditional) before it stores any, so a block waits for memory
// once per phase; LDSB bytes of LDS per block (32 KB lets five blocks share a
// CU, whose memory phases then overlap the serial solves of the others).
template <typename T, bool ADD, int LDSB>
__device__ __forceinline__ void k3_thomas2_axpy(G3 mg_bid, G3 mg_gdim, const T* z, const T* a, T* out, uint64_t nrows, int n, int rows,
                                                      const T* __restrict__ ta, const T* __restrict__ tr,
                                                      const T* __restrict__ tcp) {
  constexpr int CAP = LDSB / (int)sizeof(T);
  constexpr int EPT = CAP / NT;
  __shared__ T tile[CAP];
  const uint64_t r0 = (uint64_t)mg_bid.x * rows;
  const int nr = (int)min((uint64_t)rows, nrows - r0);
  const uint64_t base = r0 * (uint64_t)n;
  const int cnt = nr * n;
  const unsigned last = (unsigned)cnt - 1;
  // uniform row-block bases and 32-bit lane offsets
  const T* zb = z + base;
  const T* ab = a + base;
  T* ob = out + base;
  {
    T v[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) v[u] = zb[min(threadIdx.x + (unsigned)(u * NT), last)];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const unsigned k = threadIdx.x + (unsigned)(u * NT);
      if (k < (unsigned)cnt) tile[k] = v[u];
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nr) {
    T* line = tile + threadIdx.x * n;
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
  {
    T v[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) v[u] = ab[min(threadIdx.x + (unsigned)(u * NT), last)];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      const unsigned k = threadIdx.x + (unsigned)(u * NT);
      if (k < (unsigned)cnt) ob[k] = ADD ? v[u] + tile[k] : v[u] - tile[k];
    }
  }
}

template <typename T, bool ADD, int LDSB>
__global__ void __launch_bounds__(NT) k3_thomas2_axpy_k(const T* z, const T* a, T* out, uint64_t nrows, int n, int rows,
                                                      const T* __restrict__ ta, const T* __restrict__ tr,
                                                      const T* __restrict__ tcp) {
  k3_thomas2_axpy<T, ADD, LDSB>(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, z, a, out, nrows, n, rows, ta, tr, tcp);
}


// Launch of k3_thomas2_axpy over the c0 * c1 rows of length c2: 32 KB of LDS
// per block when a row fits, else 64 KB.
template <typename T, bool ADD>
void launch_thomas2_axpy(const T* z, const T* a, T* out, uint64_t nrows, int n, const T* ta, const T* tr,
                         const T* tcp, hipStream_t st) {
  if ((uint64_t)n * sizeof(T) <= (uint64_t)AXPY_LDS / 2) {
    const int rows = std::max(1, std::min(64, (int)(AXPY_LDS / 2 / sizeof(T) / n)));
    MG_LAUNCH((&k3_thomas2_axpy<T, ADD, AXPY_LDS / 2>), (k3_thomas2_axpy_k<T, ADD, AXPY_LDS / 2>), (NT), (0), (dim3((unsigned)((nrows + rows - 1) / rows))), st, z, a, out, nrows, n, rows, ta, tr, tcp);
  } else {
    const int rows = std::max(1, std::min(64, (int)(AXPY_LDS / sizeof(T) / n)));
    MG_LAUNCH((&k3_thomas2_axpy<T, ADD, AXPY_LDS>), (k3_thomas2_axpy_k<T, ADD, AXPY_LDS>), (NT), (0), (dim3((unsigned)((nrows + rows - 1) / rows))), st, z, a, out, nrows, n, rows, ta, tr, tcp);
  }
}

// ------------------------------------------------------------------ recomposition
// Coefficients of each fine plane from the stream (zeros at coarse nodes),
// then mass + restriction along dim 2 and dim 1 -> g1.  Same tile layout as
// the decomposition kernel: thread t owns fine column t % 128 and half of the
// rows (scalar per wavefront); the symbols of the next plane are loaded into
// registers while the current one is restricted.
template <typename T, int MODE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : 2)))
k3_scatter_r21(const uint16_t* __restrict__ sym, const int64_t* __restrict__ qside, const T* __restrict__ cstream,
               const double* __restrict__ bins, int level, int R, T* __restrict__ g1, Lv3<T> p, int planes_per) {
  __shared__ T U[FY * PX];
  __shared__ T W1s[5 * FY + 2 * CY];
  __shared__ uint64_t subs[8][4];
  __shared__ uint64_t rb[2][FY][2];
  const int t = threadIdx.x;
  const int J1 = blockIdx.y * CY, J2 = blockIdx.x * CX;
  const int F1 = 2 * J1 - 2, F2 = 2 * J2 - 2;
  const int n0 = p.n0, n1 = p.n1, n2 = p.n2;
  const double b = MODE == 1 ? bins[level] : 0.0;
  load_sub(subs, p.sub, p.level_off);
  const TileW<T> w1 = stage_weights<T, FY, CY>(W1s, p.d1, F1, J1, n1, p.c1);
  const int x = t & (PX - 1), h = __builtin_amdgcn_readfirstlane(t >> 7);
  const int r0 = h * HR, nr = h ? FY - HR : HR;
  const int f2 = F2 + x;
  const bool colok = x < FX && f2 >= 0 && f2 < n2;
  const bool e2 = colok && is_new(f2, n2);
  const uint64_t i2 = e2 ? (uint64_t)(f2 >> 1) : (uint64_t)cidx(f2);
  const int jx = t & 63, g4 = __builtin_amdgcn_readfirstlane(t >> 6);
  const int j2 = J2 + jx;
  const bool ok2 = jx < CX && j2 < p.c2;
  RestrictW<T> rw2;
  if (ok2) rw2.load(j2, p.c2, n2, p.d2);
  __syncthreads();  // subs and the staged weights

  // Stream row bases of a plane (dim-2 parity 0 / 1), two planes in flight:
  // rb[slot][r][e2] for fine row F1 + r, 0 outside the grid.
  const int fb = blockIdx.z * planes_per, fe = min(fb + planes_per, n0);
  auto bases = [&](int f0, int slot) {
    if (t < 2 * FY && f0 < fe) {
      const int f1 = F1 + (t >> 1);
      rb[slot][t >> 1][t & 1] = (f1 >= 0 && f1 < n1) ? row_base(subs, f0, n0, f1, n1, t & 1) : 0;
    }
  };
  // The coefficients of the next plane are loaded into registers while the
  // current one is restricted: unconditional loads (position 0 stands in for
  // nodes without a coefficient: outside the grid, or coarse in every
  // dimension); their positions and presence stay in registers for the commit.
  uint16_t sv[HR];
  T cv[HR];
  uint64_t pv[HR];
  uint32_t hasm = 0;
  auto prefetch = [&](int f0, int slot) {
    hasm = 0;
    const bool e0 = is_new(f0, n0);
#pragma unroll
    for (int j = 0; j < HR; ++j) {
      const int r = r0 + j, f1 = F1 + r;
      const bool rowok = j < nr && f1 >= 0 && f1 < n1;
      const bool has = rowok && colok && (e0 || is_new(f1, n1) || e2);
      const uint64_t pos = has ? rb[slot][rowok ? r : 0][e2 ? 1 : 0] + i2 : 0;
      hasm |= has ? 1u << j : 0u;
      pv[j] = pos;
      if (MODE == 1)
        sv[j] = sym[pos];
      else
        cv[j] = cstream[pos];
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int j = 0; j < HR; ++j) {
      if (j >= nr) continue;
      T c = T(0);
      if ((hasm >> j) & 1) {
        if (MODE == 1) {
          const double q = sv[j] ? (double)((int)sv[j] - R) : (double)qside[pv[j]];
          c = static_cast<T>(q * b);
        } else {
          c = cv[j];
        }
      }
      U[(r0 + j) * PX + x] = c;
    }
  };
  bases(fb, 0);
  __syncthreads();
  if (fb < fe) prefetch(fb, 0);
  for (int f0 = fb; f0 < fe; ++f0) {
    const int slot = (f0 - fb) & 1;
    commit();
    bases(f0 + 1, slot ^ 1);
    __syncthreads();
    if (f0 + 1 < fe) prefetch(f0 + 1, slot ^ 1);
    // mass + restriction along dim 2 for every row of the tile, held in
    // registers until every lane is done reading U, then stored in U's place
    constexpr int R2N = (FY + 3) / 4;
    T g2v[R2N];
#pragma unroll
    for (int k = 0; k < R2N; ++k) {
      const int r = g4 + 4 * k, f1 = F1 + r;
      g2v[k] = T(0);
      if (r < FY && f1 >= 0 && f1 < n1 && ok2) {
        const T* row = U + r * PX - F2;  // row[f2] for fine f2 inside the tile
        g2v[k] = rw2.apply([&](int i) { return row[i]; });
      }
    }
    __syncthreads();
    T* G2 = U;
#pragma unroll
    for (int k = 0; k < R2N; ++k) {
      const int r = g4 + 4 * k, f1 = F1 + r;
      if (r < FY && f1 >= 0 && f1 < n1 && ok2) G2[r * 64 + jx] = g2v[k];
    }
    __syncthreads();
    // mass + restriction along dim 1 -> g1
    for (int jy = g4; jy < CY; jy += 4) {
      const int j1 = J1 + jy;
      if (j1 >= p.c1 || !ok2) continue;
      const T* col = G2 + jx - F1 * 64;  // col[f1 * 64]
      const T f = restrict_at<T>(j1, p.c1, n1, w1, [&](int i) { return col[i * 64]; });
      g1[((uint64_t)f0 * p.c1 + j1) * p.c2 + j2] = f;
    }
    __syncthreads();
  }
}

// u_l = c + Pi(uc) at new nodes, uc at coarse nodes; Pi nested with dim 2 innermost.
// A block covers IA_ROWS fine rows of one plane and IA_XP column pairs
// (2q, 2q+1) with 2q+1 < n2: column 2q is coarse along dim 2 and column 2q+1
// is new (or, for an even side, the last coarse column).  Lane t owns pair
// X0 + t for every row, so its dim-2 weights are registers and every row
// quantity is the same across a wavefront; for an odd side the lane with the
// last pair also writes the last column (coarse, unpaired).  The coarse rows
// the block interpolates from (at most IA_CR per coarse plane, at most two
// planes) are staged in LDS; each lane loads the symbols of all its rows
// before any arithmetic.
constexpr int IA_ROWS = 8;
constexpr int IA_CR = IA_ROWS / 2 + 1;
constexpr int IA_XP = NT;  // column pairs per block

// Loads that are issued under a branch, or whose result is merged with a
// default right away, make the compiler wait for every outstanding memory
// operation (stores included) before going on.  So every load below is
// unconditional, from an index clamped into its array (position 0 stands in
// for a node without a coefficient), and conditions are applied where the
// values are used; the coarse rows are loaded into registers first, while the
// row tables are set up; escape symbols (whose values live in the side array)
// are patched after every row has been stored, so no row waits for the
// stores of the rows before it.
constexpr int IA_CS = (2 * IA_CR * (IA_XP + 1) + NT - 1) / NT;  // coarse values per thread

template <typename T, int MODE>
__global__ void __launch_bounds__(NT) k3_interp_add(T* __restrict__ out, const T* __restrict__ uc,
                                                    const uint16_t* __restrict__ sym, const int64_t* __restrict__ qside,
                                                    const T* __restrict__ cstream, const double* __restrict__ bins,
                                                    int level, int R, Lv3<T> p) {
  __shared__ T Cs[2][IA_CR][IA_XP + 1];
  __shared__ uint64_t subs[8][4];
  __shared__ uint64_t rb0[IA_ROWS], rb1[IA_ROWS], obs[IA_ROWS];
  __shared__ T w1s[IA_ROWS][2];
  __shared__ int kbs[IA_ROWS];
  const int n0 = p.n0, n1 = p.n1, n2 = p.n2, c1 = p.c1, c2 = p.c2;
  const int t = threadIdx.x;
  const int f0 = blockIdx.z;
  const int R0 = blockIdx.y * IA_ROWS;
  const int nrow = min(IA_ROWS, n1 - R0);
  const int npairs = n2 >> 1;
  const int X0 = blockIdx.x * IA_XP;           // first pair (= first coarse column) of the tile
  const int np = min(IA_XP, npairs - X0);
  const int ncol = min(np + 1, c2 - X0);       // coarse columns X0 .. X0 + ncol - 1
  const bool e0 = is_new(f0, n0);
  const int q0 = e0 ? (f0 >> 1) : cidx(f0);
  const int lo = cidx(R0);                     // R0 is even: a coarse row
  const int last = R0 + nrow - 1;
  const int hi = is_new(last, n1) ? (last >> 1) + 1 : cidx(last);
  const int ncr = hi - lo + 1;
  // coarse rows lo..hi of planes q0 (and q0 + 1 for a new plane), columns of the tile
  const int npl = e0 ? 2 : 1;
  const int per = ncr * ncol;
  T cvals[IA_CS];
#pragma unroll
  for (int it = 0; it < IA_CS; ++it) {
    const int k = min(t + it * NT, npl * per - 1);
    const int a = k / per, rem = k - a * per;
    const int rr = rem / ncol, j = rem - rr * ncol;
    cvals[it] = uc[((uint64_t)(q0 + a) * c1 + (uint64_t)(lo + rr)) * c2 + (uint64_t)(X0 + j)];
  }
  load_sub(subs, p.sub, p.level_off);
  __syncthreads();
  // this lane's pair, its dim-2 weights (read only where fb is new), and
  // whether it also owns the last column
  const int q = t, qq = X0 + q;
  const bool live = q < np;
  const int fa = 2 * qq, fb = fa + 1;
  const bool nb = live && is_new(fb, n2);
  const int fbc = min(fb, n2 - 1);
  const T wl2 = p.d2.wl[fbc], wr2 = p.d2.wr[fbc];
  const bool extra = live && (n2 & 1) && qq == npairs - 1;  // column n2 - 1 = fb + 1
  if (t < nrow) {
    const int f1 = R0 + t;
    const bool e1 = is_new(f1, n1);
    const T a1 = p.d1.wl[f1], b1 = p.d1.wr[f1];
    rb0[t] = row_base(subs, f0, n0, f1, n1, 0);
    rb1[t] = row_base(subs, f0, n0, f1, n1, 1);
    obs[t] = ((uint64_t)f0 * n1 + f1) * n2;
    w1s[t][0] = e1 ? a1 : T(0);
    w1s[t][1] = e1 ? b1 : T(0);
    kbs[t] = (e1 ? (f1 >> 1) : cidx(f1)) - lo;
  }
  __syncthreads();
  // stream positions of row r's coefficients in columns fa, fb and the extra
  // column (0 where there is none)
  auto positions = [&](int r, uint64_t& pa, uint64_t& pb, uint64_t& px) {
    const bool rowok = r < nrow && live;
    const bool e1 = is_new(R0 + r, n1);
    const uint64_t base0 = rb0[min(r, nrow - 1)], base1 = rb1[min(r, nrow - 1)];
    pa = rowok && (e0 || e1) ? base0 + (uint64_t)qq : 0;
    px = rowok && (e0 || e1) && extra ? base0 + (uint64_t)(qq + 1) : 0;
    pb = rowok && (nb || e0 || e1) ? (nb ? base1 + (uint64_t)qq : base0 + (uint64_t)(qq + 1)) : 0;
  };
  // the symbols (or float coefficients) of every row
  uint16_t sa[IA_ROWS], sb[IA_ROWS], sx[IA_ROWS];
  T ca[IA_ROWS], cb[IA_ROWS], cx[IA_ROWS];
#pragma unroll
  for (int r = 0; r < IA_ROWS; ++r) {
    uint64_t pa, pb, px;
    positions(r, pa, pb, px);
    if (MODE == 1) {
      sa[r] = sym[pa];
      sb[r] = sym[pb];
      sx[r] = sym[px];
    } else {
      ca[r] = cstream[pa];
      cb[r] = cstream[pb];
      cx[r] = cstream[px];
    }
  }
#pragma unroll
  for (int it = 0; it < IA_CS; ++it) {
    const int k = t + it * NT;
    if (k < npl * per) {
      const int a = k / per, rem = k - a * per;
      const int rr = rem / ncol, j = rem - rr * ncol;
      Cs[a][rr][j] = cvals[it];
    }
  }
  __syncthreads();
  if (!live) return;
  const double b = MODE == 1 ? bins[level] : 0.0;
  const T w0l = e0 ? p.d0.wl[f0] : T(0), w0r = e0 ? p.d0.wr[f0] : T(0);
  // the coefficient of a symbol; an escape (0) reads the side array only when
  // `side` is set (the patch pass) and stands in as 0 otherwise
  auto coef = [&](uint16_t s, T cf, uint64_t pos, bool side) -> T {
    if (MODE == 0) return cf;
    const double qv = s ? (double)((int)s - R) : side ? (double)qside[pos] : 0.0;
    return static_cast<T>(qv * b);
  };
  auto row = [&](int r, bool side) {
    const bool e1 = is_new(R0 + r, n1);
    const int kb = kbs[r];
    const T w1l = w1s[r][0], w1r = w1s[r][1];
    // coarse value of plane choice a, row choice bb, coarse column qc (tile-relative)
    auto V = [&](int a, int bb, int qc) -> T { return Cs[a][kb + bb][qc]; };
    auto Va = [&](int a, int bb) -> T { return V(a, bb, q); };
    auto Vb = [&](int a, int bb) -> T {
      if (nb) return wl2 * V(a, bb, q) + wr2 * V(a, bb, q + 1);
      return V(a, bb, q + 1);
    };
    auto Vx = [&](int a, int bb) -> T { return V(a, bb, q + 1); };
    auto W = [&](auto&& Vf, int a) -> T { return e1 ? w1l * Vf(a, 0) + w1r * Vf(a, 1) : Vf(a, 0); };
    auto PI = [&](auto&& Vf) -> T { return e0 ? w0l * W(Vf, 0) + w0r * W(Vf, 1) : W(Vf, 0); };
    const uint64_t o = obs[r] + fa;
    uint64_t pa = 0, pb = 0, px = 0;
    if (side) positions(r, pa, pb, px);
    // column fa: coarse along dim 2; column fb: new along dim 2, or the last
    // (coarse) column of an even side; the pair is one 2-element store
    T pair[2];
    pair[0] = (!e0 && !e1) ? Cs[0][kb][q] : coef(sa[r], ca[r], pa, side) + PI(Va);
    pair[1] = (!nb && !e0 && !e1) ? Cs[0][kb][q + 1] : coef(sb[r], cb[r], pb, side) + PI(Vb);
    __builtin_memcpy(out + o, pair, sizeof(pair));
    // the last column of an odd side (coarse along dim 2)
    if (extra) {
      if (!e0 && !e1)
        out[o + 2] = Cs[0][kb][q + 1];
      else
        out[o + 2] = coef(sx[r], cx[r], px, side) + PI(Vx);
    }
  };
  uint32_t esc = 0;  // rows of this lane with an escape among its coefficients
#pragma unroll
  for (int r = 0; r < IA_ROWS; ++r) {
    if (r >= nrow) continue;
    row(r, false);
    if (MODE == 1) {
      const bool e1 = is_new(R0 + r, n1);
      const bool has = (e0 || e1) && (sa[r] == 0 || (extra && sx[r] == 0));
      const bool hasb = (nb || e0 || e1) && sb[r] == 0;
      esc |= has || hasb ? 1u << r : 0u;
    }
  }
  // rewrite the rows that hold an escape, now with their side values
  if (MODE == 1 && esc) {
    for (int r = 0; r < IA_ROWS; ++r)
      if ((esc >> r) & 1u) row(r, true);
  }
}

// ------------------------------------------------------------------ small levels
// The levels whose three sides are all at most TAIL_N, and the coarsest grid,
// in one workgroup with every intermediate grid in LDS: the same arithmetic as
// the per-level kernels above (the same interpolation nest, mass_at /
// restrict_at, Thomas recurrences and quantizer), one barrier between steps
// instead of one launch per step.
constexpr int TAIL_N = 17;
constexpr int TAIL_F = TAIL_N * TAIL_N * TAIL_N;                  // fine grid of a tail level
constexpr int TAIL_H = TAIL_N / 2 + 1;                            // its coarse side
constexpr int TAIL_C = TAIL_H * TAIL_H * TAIL_H;                  // coarse grid
constexpr int TAIL_G2 = TAIL_N * TAIL_N * TAIL_H;                 // after the dim-2 restriction
constexpr int TAIL_G1 = TAIL_N * TAIL_H * TAIL_H;                 // after the dim-1 restriction
constexpr int TAIL_T = 1024;
constexpr int TAIL_LMAX = 6;

template <typename T>
struct TailLevels {
  int nl;               // levels in the tail
  Lv3<T> lv[TAIL_LMAX];  // decomposition: finest first; recomposition: coarsest first
};

// A level's weights in LDS: ws[d][a][i] holds array a of dimension d (wl, wr,
// ma, mb, mc over fine indices; rl, rr, ta, tr, tcp over coarse ones); the
// returned constants point into it.
template <typename T>
struct TailW {
  DimConsts<T> d[3];
};
template <typename T>
__device__ inline const T* tail_arr(const DimConsts<T>& w, int a) {
  switch (a) {
    case 0: return w.wl;
    case 1: return w.wr;
    case 2: return w.ma;
    case 3: return w.mb;
    case 4: return w.mc;
    case 5: return w.rl;
    case 6: return w.rr;
    case 7: return w.ta;
    case 8: return w.tr;
    default: return w.tcp;
  }
}
template <typename T>
__device__ inline TailW<T> tail_stage_weights(T (*ws)[10][TAIL_N], const Lv3<T>& p) {
  for (int e = threadIdx.x; e < 3 * 10 * TAIL_N; e += TAIL_T) {
    const int d = e / (10 * TAIL_N), a = (e / TAIL_N) % 10, i = e % TAIL_N;
    const DimConsts<T>& w = d == 0 ? p.d0 : d == 1 ? p.d1 : p.d2;
    const int nf = d == 0 ? p.n0 : d == 1 ? p.n1 : p.n2, nc = d == 0 ? p.c0 : d == 1 ? p.c1 : p.c2;
    if (i < (a < 5 ? nf : nc)) ws[d][a][i] = tail_arr(w, a)[i];
  }
  TailW<T> r;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    r.d[d] = DimConsts<T>{ws[d][0], ws[d][1], ws[d][2], ws[d][3], ws[d][4],
                          ws[d][5], ws[d][6], ws[d][7], ws[d][8], ws[d][9]};
  return r;
}

// Every level's weights and sub-grid table in LDS at once (ws[k], subs[k] for
// a.lv[k]): one batch of loads, from indices clamped into their arrays, for
// the whole kernel, so no level waits on loads issued after the previous
// level's stores.
constexpr int TAIL_WPL = 3 * 10 * TAIL_N;                          // weights per level
constexpr int TAIL_WIT = (TAIL_LMAX * TAIL_WPL + TAIL_T - 1) / TAIL_T;
template <typename T>
__device__ inline void tail_stage_all(T (*ws)[3][10][TAIL_N], uint64_t (*subs)[8][4], const TailLevels<T>& a) {
  const int t = threadIdx.x;
  const int total = a.nl * TAIL_WPL;
  auto where = [&](int e, int& k, int& d, int& q, int& i, int& lim) {
    k = e / TAIL_WPL;
    const int r = e - k * TAIL_WPL;
    d = r / (10 * TAIL_N);
    q = (r / TAIL_N) % 10;
    i = r % TAIL_N;
    const Lv3<T>& p = a.lv[k];
    const int nf = d == 0 ? p.n0 : d == 1 ? p.n1 : p.n2, nc = d == 0 ? p.c0 : d == 1 ? p.c1 : p.c2;
    lim = q < 5 ? nf : nc;
  };
  T v[TAIL_WIT];
#pragma unroll
  for (int it = 0; it < TAIL_WIT; ++it) {
    int k, d, q, i, lim;
    where(min(t + it * TAIL_T, total - 1), k, d, q, i, lim);
    const Lv3<T>& p = a.lv[k];
    const DimConsts<T>& w = d == 0 ? p.d0 : d == 1 ? p.d1 : p.d2;
    v[it] = tail_arr(w, q)[min(i, lim - 1)];
  }
  uint64_t sv = 0;
  int sk = 0, sm = 0, se = 0;
  if (t < a.nl * 32) {
    sk = t >> 5;
    sm = (t >> 2) & 7;
    se = t & 3;
    const Lv3<T>& p = a.lv[sk];
    sv = sm == 0 ? 0 : (se == 0 ? p.level_off + p.sub[sm] : p.sub[16 + 4 * sm + se]);
  }
#pragma unroll
  for (int it = 0; it < TAIL_WIT; ++it) {
    const int e = t + it * TAIL_T;
    if (e >= total) continue;
    int k, d, q, i, lim;
    where(e, k, d, q, i, lim);
    if (i < lim) ws[k][d][q][i] = v[it];
  }
  if (t < a.nl * 32) subs[sk][sm][se] = sv;
}
template <typename T>
__device__ inline TailW<T> tail_weights(T (*ws)[10][TAIL_N]) {
  TailW<T> r;
#pragma unroll
  for (int d = 0; d < 3; ++d)
    r.d[d] = DimConsts<T>{ws[d][0], ws[d][1], ws[d][2], ws[d][3], ws[d][4],
                          ws[d][5], ws[d][6], ws[d][7], ws[d][8], ws[d][9]};
  return r;
}
constexpr int TAIL_PER = (TAIL_F + TAIL_T - 1) / TAIL_T;  // fine nodes per thread

// Thomas along one line (n values `stride` apart), as k_thomas
template <typename T>
__device__ inline void tail_thomas(T* base, int n, int stride, const DimConsts<T>& w) {
  T prev = base[0] * w.tr[0];
  base[0] = prev;
  for (int i = 1; i < n; ++i) {
    prev = (base[i * stride] - w.ta[i] * prev) * w.tr[i];
    base[i * stride] = prev;
  }
  T x = prev;
  for (int i = n - 2; i >= 0; --i) {
    x = base[i * stride] - w.tcp[i] * x;
    base[i * stride] = x;
  }
}

// c (n0 x n1 x n2, zeros at coarse nodes) -> z (c0 x c1 x c2): restrictions
// along dims 2, 1, 0 (g2, g1 scratch; z may alias g2), then the three solves.
template <typename T>
__device__ inline void tail_correction(const Lv3<T>& p, const TailW<T>& w, const T* c, T* g2, T* g1, T* z) {
  const int t = threadIdx.x;
  const int n0 = p.n0, n1 = p.n1, n2 = p.n2, c0 = p.c0, c1 = p.c1, c2 = p.c2;
  for (int e = t; e < n0 * n1 * c2; e += TAIL_T) {
    const int f01 = e / c2, j2 = e - f01 * c2;
    g2[e] = restrict_at<T>(j2, c2, n2, w.d[2], [&](int i) { return c[f01 * n2 + i]; });
  }
  __syncthreads();
  for (int e = t; e < n0 * c1 * c2; e += TAIL_T) {
    const int f0 = e / (c1 * c2), j12 = e - f0 * (c1 * c2), j1 = j12 / c2, j2 = j12 - j1 * c2;
    g1[e] = restrict_at<T>(j1, c1, n1, w.d[1], [&](int i) { return g2[(f0 * n1 + i) * c2 + j2]; });
  }
  __syncthreads();
  for (int e = t; e < c0 * c1 * c2; e += TAIL_T) {
    const int j0 = e / (c1 * c2), j12 = e - j0 * (c1 * c2);
    z[e] = restrict_at<T>(j0, c0, n0, w.d[0], [&](int i) { return g1[i * (c1 * c2) + j12]; });
  }
  __syncthreads();
  for (int e = t; e < c1 * c2; e += TAIL_T) tail_thomas(z + e, c0, c1 * c2, w.d[0]);
  __syncthreads();
  for (int e = t; e < c0 * c2; e += TAIL_T) {
    const int j0 = e / c2, j2 = e - j0 * c2;
    tail_thomas(z + j0 * c1 * c2 + j2, c1, c2, w.d[1]);
  }
  __syncthreads();
  for (int e = t; e < c0 * c1; e += TAIL_T) tail_thomas(z + e * c2, c2, 1, w.d[2]);
  __syncthreads();
}

// stream position of fine node (f0, f1, f2) of a level with mask m != 0
__device__ inline uint64_t tail_pos(const uint64_t (*subs)[4], int f0, int n0, int f1, int n1, int f2, int n2) {
  const bool e0 = is_new(f0, n0), e1 = is_new(f1, n1), e2 = is_new(f2, n2);
  const int m = (e0 ? 1 : 0) | (e1 ? 2 : 0) | (e2 ? 4 : 0);
  const uint64_t i0 = e0 ? (uint64_t)(f0 >> 1) : (uint64_t)cidx(f0);
  const uint64_t i1 = e1 ? (uint64_t)(f1 >> 1) : (uint64_t)cidx(f1);
  const uint64_t i2 = e2 ? (uint64_t)(f2 >> 1) : (uint64_t)cidx(f2);
  return subs[m][0] + i0 * subs[m][1] + i1 * subs[m][2] + i2;
}

// Decomposition of levels lt .. lt - nl + 1 (a.lv[k] = level lt - k) and the
// coarsest grid; u is the fine grid of level lt.  MODE 1: symbols; MODE 0:
// float coefficients in cstream.
template <typename T, int MODE>
__device__ __forceinline__ void k3_tail_decompose(G3 mg_bid, G3 mg_gdim, const T* __restrict__ u, uint16_t* __restrict__ sym,
                                                           int64_t* __restrict__ qside, T* __restrict__ cstream,
                                                           const double* __restrict__ bins, int R, int lt,
                                                           const TailLevels<T>& a) {
  __shared__ T A[TAIL_F], B[TAIL_C], C[TAIL_F], G[TAIL_G2];
  __shared__ T WS[TAIL_LMAX][3][10][TAIL_N];
  __shared__ uint64_t SUBS[TAIL_LMAX][8][4];
  const int t = threadIdx.x;
  {
    // the fine grid: every load issued (clamped index) before any store
    const Lv3<T>& p = a.lv[0];
    const int nf = p.n0 * p.n1 * p.n2;
    T v[TAIL_PER];
#pragma unroll
    for (int it = 0; it < TAIL_PER; ++it) v[it] = u[min(t + it * TAIL_T, nf - 1)];
    tail_stage_all<T>(WS, SUBS, a);
#pragma unroll
    for (int it = 0; it < TAIL_PER; ++it)
      if (t + it * TAIL_T < nf) A[t + it * TAIL_T] = v[it];
  }
  T* U = A;   // fine grid of the current level
  T* UC = B;  // its coarse grid
  int ncoarse = 0;
  for (int k = 0; k < a.nl; ++k) {
    const Lv3<T>& p = a.lv[k];
    const int level = lt - k;
    const int n0 = p.n0, n1 = p.n1, n2 = p.n2, c1 = p.c1, c2 = p.c2;
    const uint64_t (*subs)[4] = SUBS[k];
    const TailW<T> w = tail_weights<T>(WS[k]);
    __syncthreads();
    const double inv_b = MODE == 1 ? 1.0 / bins[level] : 0.0;
    // coefficients (interpolant nested with dim 2 innermost), quantization, coarse copy
    for (int e = t; e < n0 * n1 * n2; e += TAIL_T) {
      const int f0 = e / (n1 * n2), f12 = e - f0 * (n1 * n2), f1 = f12 / n2, f2 = f12 - f1 * n2;
      const bool e0 = is_new(f0, n0), e1 = is_new(f1, n1), e2 = is_new(f2, n2);
      if (!e0 && !e1 && !e2) {
        UC[(cidx(f0) * c1 + cidx(f1)) * c2 + cidx(f2)] = U[e];
        C[e] = T(0);
        continue;
      }
      auto Y = [&](int g0, int g1) -> T {
        const T* row = U + (g0 * n1 + g1) * n2;
        return e2 ? w.d[2].wl[f2] * row[f2 - 1] + w.d[2].wr[f2] * row[f2 + 1] : row[f2];
      };
      auto X = [&](int g0) -> T {
        return e1 ? w.d[1].wl[f1] * Y(g0, f1 - 1) + w.d[1].wr[f1] * Y(g0, f1 + 1) : Y(g0, f1);
      };
      const T pi = e0 ? w.d[0].wl[f0] * X(f0 - 1) + w.d[0].wr[f0] * X(f0 + 1) : X(f0);
      const T c = U[e] - pi;
      C[e] = c;
      const uint64_t pos = tail_pos(subs, f0, n0, f1, n1, f2, n2);
      if (MODE == 1)
        quant_store(c, inv_b, R, pos, sym, qside);
      else
        cstream[pos] = c;
    }
    __syncthreads();
    // z = M^-1 P^T M c (g1 over the coefficients, which are done), then u_{l-1} = u_l|coarse + z
    tail_correction<T>(p, w, C, G, C, G);
    ncoarse = p.c0 * c1 * c2;
    for (int e = t; e < ncoarse; e += TAIL_T) UC[e] = UC[e] + G[e];
    __syncthreads();
    T* tmp = U;
    U = UC;
    UC = tmp;
  }
  // the coarsest grid opens the stream
  const double inv_b0 = MODE == 1 ? 1.0 / bins[0] : 0.0;
  for (int e = t; e < ncoarse; e += TAIL_T) {
    if (MODE == 1)
      quant_store(U[e], inv_b0, R, (uint64_t)e, sym, qside);
    else
      cstream[e] = U[e];
  }
}

template <typename T, int MODE>
__global__ void __launch_bounds__(TAIL_T) k3_tail_decompose_k(const T* __restrict__ u, uint16_t* __restrict__ sym,
                                                           int64_t* __restrict__ qside, T* __restrict__ cstream,
                                                           const double* __restrict__ bins, int R, int lt,
                                                           TailLevels<T> a) {
  k3_tail_decompose<T, MODE>(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, u, sym, qside, cstream, bins, R, lt, a);
}


// Recomposition of levels lt - nl + 1 .. lt (a.lv[k] = level lt - nl + 1 + k)
// from the coarsest grid in the stream; writes the fine grid of level lt to out.
template <typename T, int MODE>
__global__ void __launch_bounds__(TAIL_T) k3_tail_recompose(T* __restrict__ out, const uint16_t* __restrict__ sym,
                                                           const int64_t* __restrict__ qside,
                                                           const T* __restrict__ cstream,
                                                           const double* __restrict__ bins, int R, int lt,
                                                           TailLevels<T> a) {
  __shared__ T P0[TAIL_C], P1[TAIL_C], C[TAIL_F], G[TAIL_G2], G1[TAIL_G1];
  __shared__ T WS[TAIL_LMAX][3][10][TAIL_N];
  __shared__ uint64_t SUBS[TAIL_LMAX][8][4];
  const int t = threadIdx.x;
  T* UC = P0;  // coarse grid of the current level
  T* UF = P1;  // its fine grid (below the last level)
  tail_stage_all<T>(WS, SUBS, a);
  {
    const Lv3<T>& p = a.lv[0];
    const double b0 = MODE == 1 ? bins[0] : 0.0;
    for (int e = t; e < p.c0 * p.c1 * p.c2; e += TAIL_T)
      UC[e] = MODE == 1 ? dequant_load<T>(sym, qside, (uint64_t)e, b0, R) : cstream[e];
  }
  for (int k = 0; k < a.nl; ++k) {
    const Lv3<T>& p = a.lv[k];
    const int level = lt - a.nl + 1 + k;
    const bool last = k == a.nl - 1;
    const int n0 = p.n0, n1 = p.n1, n2 = p.n2, c1 = p.c1, c2 = p.c2;
    const uint64_t (*subs)[4] = SUBS[k];
    const TailW<T> w = tail_weights<T>(WS[k]);
    __syncthreads();
    const double b = MODE == 1 ? bins[level] : 0.0;
    // coefficients of the level (zeros at coarse nodes): every load issued
    // (position 0 for nodes without one) before any is used
    const int nf = n0 * n1 * n2;
    uint64_t pos[TAIL_PER];
    uint16_t sv[TAIL_PER];
    T cv[TAIL_PER];
#pragma unroll
    for (int it = 0; it < TAIL_PER; ++it) {
      const int e = t + it * TAIL_T;
      const int ec = min(e, nf - 1);
      const int f0 = ec / (n1 * n2), f12 = ec - f0 * (n1 * n2), f1 = f12 / n2, f2 = f12 - f1 * n2;
      const bool any = is_new(f0, n0) || is_new(f1, n1) || is_new(f2, n2);
      pos[it] = e < nf && any ? tail_pos(subs, f0, n0, f1, n1, f2, n2) : 0;
      if (MODE == 1)
        sv[it] = sym[pos[it]];
      else
        cv[it] = cstream[pos[it]];
    }
#pragma unroll
    for (int it = 0; it < TAIL_PER; ++it) {
      const int e = t + it * TAIL_T;
      if (e >= nf) continue;
      const int f0 = e / (n1 * n2), f12 = e - f0 * (n1 * n2), f1 = f12 / n2, f2 = f12 - f1 * n2;
      const bool any = is_new(f0, n0) || is_new(f1, n1) || is_new(f2, n2);
      T c = T(0);
      if (any) {
        if (MODE == 1) {
          const double q = sv[it] ? (double)((int)sv[it] - R) : (double)qside[pos[it]];
          c = static_cast<T>(q * b);
        } else {
          c = cv[it];
        }
      }
      C[e] = c;
    }
    __syncthreads();
    tail_correction<T>(p, w, C, G, G1, G);
    // uc = u_{l-1} - z
    for (int e = t; e < p.c0 * c1 * c2; e += TAIL_T) UC[e] = UC[e] - G[e];
    __syncthreads();
    // u_l = c + Pi(uc) at new nodes, uc at coarse nodes (dim 2 innermost)
    T* dst = last ? out : UF;
    for (int e = t; e < n0 * n1 * n2; e += TAIL_T) {
      const int f0 = e / (n1 * n2), f12 = e - f0 * (n1 * n2), f1 = f12 / n2, f2 = f12 - f1 * n2;
      const bool e0 = is_new(f0, n0), e1 = is_new(f1, n1), e2 = is_new(f2, n2);
      const int q0 = e0 ? (f0 >> 1) : cidx(f0), q1 = e1 ? (f1 >> 1) : cidx(f1), q2 = e2 ? (f2 >> 1) : cidx(f2);
      auto V = [&](int a0, int a1, int a2) -> T { return UC[(a0 * c1 + a1) * c2 + a2]; };
      if (!e0 && !e1 && !e2) {
        dst[e] = V(q0, q1, q2);
        continue;
      }
      auto Y = [&](int a0, int a1) -> T {
        return e2 ? w.d[2].wl[f2] * V(a0, a1, q2) + w.d[2].wr[f2] * V(a0, a1, q2 + 1) : V(a0, a1, q2);
      };
      auto X = [&](int a0) -> T {
        return e1 ? w.d[1].wl[f1] * Y(a0, q1) + w.d[1].wr[f1] * Y(a0, q1 + 1) : Y(a0, q1);
      };
      const T pi = e0 ? w.d[0].wl[f0] * X(q0) + w.d[0].wr[f0] * X(q0 + 1) : X(q0);
      dst[e] = C[e] + pi;
    }
    __syncthreads();
    T* tmp = UC;
    UC = UF;
    UF = tmp;
  }
}

inline unsigned blocks1(uint64_t n) { return (unsigned)std::max<uint64_t>(1, (n + NT - 1) / NT); }

}  // namespace

template <typename T>
bool fused3d_ok(const Hierarchy& h) {
  if (h.D != 3) return false;
  for (int s = 1; s < MAXD; ++s)
    if (!h.active[s]) return false;
  if (h.shape[1] > 65535 || h.shape[2] > 65535 || h.shape[3] > (1 << 24)) return false;
  // the contiguous-dimension solve stages at least one coarse row in LDS
  return (uint64_t)h.sizes[h.L > 0 ? h.L - 1 : 0][3] * sizeof(T) <= (uint64_t)AXPY_LDS;
}

template <typename T>
static Lv3<T> lv3(const Hierarchy& h, int l, const T* table) {
  Lv3<T> p;
  p.n0 = (int)h.sizes[l][1];
  p.n1 = (int)h.sizes[l][2];
  p.n2 = (int)h.sizes[l][3];
  p.c0 = (int)h.sizes[l - 1][1];
  p.c1 = (int)h.sizes[l - 1][2];
  p.c2 = (int)h.sizes[l - 1][3];
  p.d0 = dim_consts<T>(h, l, 1, table);
  p.d1 = dim_consts<T>(h, l, 2, table);
  p.d2 = dim_consts<T>(h, l, 3, table);
  p.level_off = h.level_off[l];
  p.sub = static_cast<const uint64_t*>(h.dev_itab) + 80 * (uint64_t)l;
  return p;
}

// g1 buffer: n0 * c1 * c2; z buffer: c0 * c1 * c2
template <typename T>
uint64_t fused3d_scratch_elems(const Hierarchy& h) {
  uint64_t g = 0;
  for (int l = 1; l <= h.L; ++l)
    g = std::max<uint64_t>(g, (uint64_t)h.sizes[l][1] * h.sizes[l - 1][2] * h.sizes[l - 1][3]);
  return g;
}

// Decomposition of level l: writes the coefficients (sym/qside or cstream), the
// coarse grid u_{l-1} into `ucoarse`, using g1 and z scratch.
template <typename T>
void fused3d_decompose_level(const Hierarchy& h, int l, const T* table, const T* u, T* ucoarse, T* g1, T* z,
                             const QuantOut* q, T* cstream, hipStream_t st,
                             const std::function<void()>* coeff_written) {
  Lv3<T> p = lv3<T>(h, l, table);
  const bool fine = l == h.L;
  {
    KernelTimer kt(fine ? "coeff_r21_fine" : "coeff_r21_coarse", st);
    if constexpr (sizeof(T) == 4) {
      // register tiles, one wavefront each: coarse intervals of dim 0 per
      // wavefront so that about 8192 wavefronts run, at most 16, unless tuned
      const int nt1 = (p.c1 + RCY - 1) / RCY, nt2 = (p.c2 + RCX - 1) / RCX;
      const uint64_t tiles = (uint64_t)nt1 * nt2;
      const int guess = (int)std::max<uint64_t>(1, std::min<uint64_t>(16, ((uint64_t)(p.c0 - 1) * tiles + 8191) / 8192));
      const int seg = std::max(1, tune_get(TUNE_COEFF_SEG, false, p.n0, p.n1, p.n2, guess));
      const int nseg = (p.c0 - 1 + seg - 1) / seg;
      const uint64_t nb = tiles * (uint64_t)nseg;
      if (nb > 0x7fffffffull) fail(MGARD_ERR_SHAPE, "level too large for one launch");
      const dim3 grid((unsigned)(8 * ((nb + 7) / 8)));
      if (q)
        MG_LAUNCH((&k3_coeff_reg<1>), (k3_coeff_reg_k<1>), (RWAVE), (0), (grid), st, u, ucoarse, g1, q->sym, q->qside,
                  (float*)nullptr, q->bins, l, q->R, p, seg, nt1, nt2, nseg, p.d0.wl, p.d0.wr);
      else
        MG_LAUNCH((&k3_coeff_reg<0>), (k3_coeff_reg_k<0>), (RWAVE), (0), (grid), st, u, ucoarse, g1, (uint16_t*)nullptr,
                  (int64_t*)nullptr, cstream, (const double*)nullptr, l, 0, p, seg, nt1, nt2, nseg, p.d0.wl, p.d0.wr);
    } else {
    // coarse intervals of dim 0 per block: enough blocks to fill the chip, at most 16
    const uint64_t tiles = (uint64_t)((p.c2 + CX - 1) / CX) * ((p.c1 + CY - 1) / CY);
    const int guess = (int)std::max<uint64_t>(1, std::min<uint64_t>(16, ((uint64_t)(p.c0 - 1) * tiles + 4095) / 4096));
    const int seg = std::max(1, tune_get(TUNE_COEFF_SEG, sizeof(T) == 8, p.n0, p.n1, p.n2, guess));
    dim3 grid((p.c2 + CX - 1) / CX, (p.c1 + CY - 1) / CY, (p.c0 - 1 + seg - 1) / seg);
    if (q)
      MG_LAUNCH((&k3_coeff_r21<T, 1>), (k3_coeff_r21_k<T, 1>), (NT), (sizeof(T) == 4 ? 5 : 2), (grid), st, u, ucoarse, g1, q->sym, q->qside,
                         (T*)nullptr, q->bins, l, q->R, p, seg, p.d0.wl, p.d0.wr);
    else
      MG_LAUNCH((&k3_coeff_r21<T, 0>), (k3_coeff_r21_k<T, 0>), (NT), (sizeof(T) == 4 ? 5 : 2), (grid), st, u, ucoarse, g1, (uint16_t*)nullptr, (int64_t*)nullptr, cstream, (const double*)nullptr, l, 0, p, seg, p.d0.wl, p.d0.wr);
    }
  }
  if (coeff_written) (*coeff_written)();
  const uint64_t lines = (uint64_t)p.c1 * p.c2;
  {
    KernelTimer kt(fine ? "r0_thomas0_fine" : "r0_thomas0_coarse", st);
    MG_LAUNCH((&k3_r0_thomas0<T>), (k3_r0_thomas0_k<T>), (NT), (0), (dim3(blocks1(lines))), st, g1, z, p.n0, p.c0, lines, p.d0.ma, p.d0.mb, p.d0.mc, p.d0.rl, p.d0.rr, p.d0.ta, p.d0.tr, p.d0.tcp);
  }
  {
    KernelTimer kt(fine ? "thomas1_fine" : "thomas1_coarse", st);
    launch_thomas_strided<T>(z, (uint64_t)p.c0, p.c1, (uint64_t)p.c2, dim_consts<T>(h, l, 2, table), st);
  }
  {
    KernelTimer kt(fine ? "thomas2_add_fine" : "thomas2_add_coarse", st);
    launch_thomas2_axpy<T, true>(z, ucoarse, ucoarse, (uint64_t)p.c0 * p.c1, p.c2, p.d2.ta, p.d2.tr, p.d2.tcp, st);
  }
  MG_HIP(hipGetLastError());
}

// Recomposition of level l: from the coefficients and u_{l-1} (cur) to u_l (out).
template <typename T>
void fused3d_recompose_correction(const Hierarchy& h, int l, const T* table, T* g1, T* z, const QuantOut* q,
                                  const T* cstream, hipStream_t st) {
  Lv3<T> p = lv3<T>(h, l, table);
  const bool fine = l == h.L;
  // fine planes per block: about 2048 blocks, at most 8 planes each, unless tuned
  const uint64_t tiles = (uint64_t)((p.c2 + CX - 1) / CX) * ((p.c1 + CY - 1) / CY);
  const int guess = (int)std::max<uint64_t>(1, std::min<uint64_t>(8, (uint64_t)p.n0 * tiles / 2048));
  const int planes_per = std::max(1, tune_get(TUNE_SCATTER_PLANES, sizeof(T) == 8, p.n0, p.n1, p.n2, guess));
  {
    KernelTimer kt(fine ? "scatter_r21_fine" : "scatter_r21_coarse", st);
    dim3 grid((p.c2 + CX - 1) / CX, (p.c1 + CY - 1) / CY, (p.n0 + planes_per - 1) / planes_per);
    if (q)
      hipLaunchKernelGGL((k3_scatter_r21<T, 1>), grid, dim3(NT), 0, st, q->sym, q->qside, (const T*)nullptr, q->bins,
                         l, q->R, g1, p, planes_per);
    else
      hipLaunchKernelGGL((k3_scatter_r21<T, 0>), grid, dim3(NT), 0, st, (const uint16_t*)nullptr,
                         (const int64_t*)nullptr, cstream, (const double*)nullptr, l, 0, g1, p, planes_per);
  }
  const uint64_t lines = (uint64_t)p.c1 * p.c2;
  {
    KernelTimer kt(fine ? "rec_r0_thomas0_fine" : "rec_r0_thomas0_coarse", st);
    MG_LAUNCH((&k3_r0_thomas0<T>), (k3_r0_thomas0_k<T>), (NT), (0), (dim3(blocks1(lines))), st, g1, z, p.n0, p.c0, lines, p.d0.ma, p.d0.mb, p.d0.mc, p.d0.rl, p.d0.rr, p.d0.ta, p.d0.tr, p.d0.tcp);
  }
  {
    KernelTimer kt(fine ? "rec_thomas1_fine" : "rec_thomas1_coarse", st);
    launch_thomas_strided<T>(z, (uint64_t)p.c0, p.c1, (uint64_t)p.c2, dim_consts<T>(h, l, 2, table), st);
  }
  MG_HIP(hipGetLastError());
}

template <typename T>
void fused3d_recompose_finish(const Hierarchy& h, int l, const T* table, const T* cur, T* out, T* z,
                              const QuantOut* q, const T* cstream, hipStream_t st) {
  Lv3<T> p = lv3<T>(h, l, table);
  const bool fine = l == h.L;
  {
    KernelTimer kt(fine ? "rec_thomas2_sub_fine" : "rec_thomas2_sub_coarse", st);
    // uc = u_{l-1} - z, written over z
    launch_thomas2_axpy<T, false>(z, cur, z, (uint64_t)p.c0 * p.c1, p.c2, p.d2.ta, p.d2.tr, p.d2.tcp, st);
  }
  {
    KernelTimer kt(fine ? "interp_add3_fine" : "interp_add3_coarse", st);
    const int npairs = p.n2 / 2;
    dim3 grid((unsigned)((npairs + IA_XP - 1) / IA_XP), (unsigned)((p.n1 + IA_ROWS - 1) / IA_ROWS), (unsigned)p.n0);
    if (q)
      hipLaunchKernelGGL((k3_interp_add<T, 1>), grid, dim3(NT), 0, st, out, z, q->sym, q->qside, (const T*)nullptr,
                         q->bins, l, q->R, p);
    else
      hipLaunchKernelGGL((k3_interp_add<T, 0>), grid, dim3(NT), 0, st, out, z, (const uint16_t*)nullptr,
                         (const int64_t*)nullptr, cstream, (const double*)nullptr, l, 0, p);
  }
  MG_HIP(hipGetLastError());
}

template <typename T>
void fused3d_recompose_level(const Hierarchy& h, int l, const T* table, const T* cur, T* out, T* g1, T* z,
                             const QuantOut* q, const T* cstream, hipStream_t st) {
  fused3d_recompose_correction<T>(h, l, table, g1, z, q, cstream, st);
  fused3d_recompose_finish<T>(h, l, table, cur, out, z, q, cstream, st);
}

// Levels handled by the small-level kernels: every level l <= lt has all
// three sides <= TAIL_N (0: none).
template <typename T>
int fused3d_tail_levels(const Hierarchy& h) {
  if (!fused3d_ok<T>(h)) return 0;
  int lt = 0;
  for (int l = 1; l <= h.L && l <= TAIL_LMAX; ++l) {
    bool small = true;
    for (int s = 1; s < MAXD; ++s) small = small && h.sizes[l][s] <= TAIL_N;
    if (!small) break;
    lt = l;
  }
  return lt;
}

template <typename T>
void fused3d_tail_decompose(const Hierarchy& h, int lt, const T* table, const T* u, const QuantOut* q, T* cstream,
                            hipStream_t st) {
  TailLevels<T> a{};
  a.nl = lt;
  for (int k = 0; k < lt; ++k) a.lv[k] = lv3<T>(h, lt - k, table);
  KernelTimer kt("tail_decompose", st);
  if (q)
    MG_LAUNCH((&k3_tail_decompose<T, 1>), (k3_tail_decompose_k<T, 1>), (TAIL_T), (0), (dim3(1)), st, u, q->sym, q->qside, (T*)nullptr,
                       q->bins, q->R, lt, a);
  else
    MG_LAUNCH((&k3_tail_decompose<T, 0>), (k3_tail_decompose_k<T, 0>), (TAIL_T), (0), (dim3(1)), st, u, (uint16_t*)nullptr, (int64_t*)nullptr, cstream, (const double*)nullptr, 0, lt, a);
  MG_HIP(hipGetLastError());
}

template <typename T>
void fused3d_tail_recompose(const Hierarchy& h, int lt, const T* table, T* out, const QuantOut* q, const T* cstream,
                            hipStream_t st) {
  TailLevels<T> a{};
  a.nl = lt;
  for (int k = 0; k < lt; ++k) a.lv[k] = lv3<T>(h, k + 1, table);
  KernelTimer kt("tail_recompose", st);
  if (q)
    hipLaunchKernelGGL((k3_tail_recompose<T, 1>), dim3(1), dim3(TAIL_T), 0, st, out, q->sym, q->qside,
                       (const T*)nullptr, q->bins, q->R, lt, a);
  else
    hipLaunchKernelGGL((k3_tail_recompose<T, 0>), dim3(1), dim3(TAIL_T), 0, st, out, (const uint16_t*)nullptr,
                       (const int64_t*)nullptr, cstream, (const double*)nullptr, 0, lt, a);
  MG_HIP(hipGetLastError());
}

#define MG_INST3(T)                                                                                             \
  template bool fused3d_ok<T>(const Hierarchy&);                                                               \
  template uint64_t fused3d_scratch_elems<T>(const Hierarchy&);                                                \
  template void fused3d_decompose_level<T>(const Hierarchy&, int, const T*, const T*, T*, T*, T*, const QuantOut*, \
                                           T*, hipStream_t, const std::function<void()>*);                     \
  template void fused3d_recompose_level<T>(const Hierarchy&, int, const T*, const T*, T*, T*, T*, const QuantOut*, \
                                           const T*, hipStream_t);                                             \
  template void fused3d_recompose_correction<T>(const Hierarchy&, int, const T*, T*, T*, const QuantOut*,      \
                                                const T*, hipStream_t);                                        \
  template void fused3d_recompose_finish<T>(const Hierarchy&, int, const T*, const T*, T*, T*, const QuantOut*, \
                                            const T*, hipStream_t);                                            \
  template int fused3d_tail_levels<T>(const Hierarchy&);                                                       \
  template void fused3d_tail_decompose<T>(const Hierarchy&, int, const T*, const T*, const QuantOut*, T*,      \
                                          hipStream_t);                                                        \
  template void fused3d_tail_recompose<T>(const Hierarchy&, int, const T*, T*, const QuantOut*, const T*,      \
                                          hipStream_t);
MG_INST3(float)
MG_INST3(double)
#undef MG_INST3

}  // namespace mg
