// Lossless stage: histogram, canonical Huffman codebook, chunked encode and
// decode (gfx950).
//
// Paper Sec. 2: the quantized integers are losslessly encoded before being
// written.  The code is a canonical Huffman code over a fixed dictionary:
//   * lengths from the two-queue merge of leaves sorted by (count, symbol),
//     the leaf queue winning ties (computed in place on the sorted weights,
//     which gives the same tree as the explicit two queues);
//   * canonical codes in (length, symbol) order;
//   * the symbol stream is cut into chunks; each chunk is packed MSB-first into
//     32-bit words starting word-aligned, so chunks decode independently.
#include <algorithm>
#include <mutex>

#include "internal.hpp"

namespace mg {

namespace {

constexpr int TPB = 256;
constexpr int MAXLEN = 64;
constexpr int MAXDICT = 8192;  // largest dictionary; all LDS below is static
constexpr int CB_T = 1024, CB_KPT = MAXDICT / CB_T;  // codebook block; sort keys per thread
// Encoder tables: codes of at most ENC_PACKLEN bits are packed with their
// length into one word (code << 6 | length); longer codes up to ENC_MAXLEN
// bits (the wave encoder's limit) are entered as ENC_LONG, and the encoder
// reads them from the full code and length tables.
constexpr int ENC_PACKLEN = 26;
constexpr int ENC_MAXLEN = 32;
constexpr uint32_t ENC_LONG = 63;

// ------------------------------------------------------------------ histogram
// Blocks of 1024 threads with a private LDS histogram; each wave takes whole
// chunks (chunk is a multiple of 256), four symbols per lane per step with
// 8-byte loads, and counts the chunk's escapes with a wave reduction.  Each
// block adds its nonzero bins to the global histogram once.
constexpr int WAVE_T = 1024;              // threads of the wave-per-chunk kernels
constexpr int WAVES = WAVE_T / 64;

// Symbols i .. i+3 of a chunk ending at `end` (i is a multiple of 4); lanes
// past the end get 0xffffffff.
__device__ inline void load4_symbols(const uint16_t* __restrict__ sym, uint64_t i, uint64_t end, uint32_t* s) {
  if (i + 4 <= end) {
    const uint2 v = *reinterpret_cast<const uint2*>(sym + i);
    s[0] = v.x & 0xffffu;
    s[1] = v.x >> 16;
    s[2] = v.y & 0xffffu;
    s[3] = v.y >> 16;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = i + j < end ? (uint32_t)sym[i + j] : 0xffffffffu;
  }
}

// The full chunks kb, kb + stride, ... below kfull of one wavefront (chunk a
// multiple of 256, at most 1024): each lane holds four 8-byte groups of a
// chunk (step s: symbols beg + 256 s + 4 lane .. + 3).  The next chunk's
// loads are issued before the current chunk is processed and its result
// stored, and no load is under a branch (steps past the chunk's end re-read
// its last step and are not used; the chunk index past the end is clamped),
// so a wait covers only loads issued one chunk earlier and never a store.
// body(k, v) handles chunk k from v and stores its result from every lane.
template <typename F>
__device__ inline void walk_full_chunks(const uint16_t* __restrict__ sym, int chunk, uint64_t kb, uint64_t kfull,
                                        uint64_t stride, int lane, F&& body) {
  if (kb >= kfull) return;
  auto load = [&](uint64_t k, uint2 (&v)[4]) {
    const uint64_t beg = min(k, kfull - 1) * (uint64_t)chunk + 4 * (uint64_t)lane;
#pragma unroll
    for (int st = 0; st < 4; ++st)
      v[st] = *reinterpret_cast<const uint2*>(sym + beg + (uint64_t)min(256 * st, chunk - 256));
  };
  uint2 va[4], vb[4];
  load(kb, va);
  for (uint64_t k = kb; k < kfull; k += 2 * stride) {
    load(k + stride, vb);
    body(k, va);
    if (k + stride >= kfull) break;
    load(k + 2 * stride, va);
    body(k + stride, vb);
  }
}

// A value the same on every lane of the wavefront, made scalar: loads indexed
// by it become scalar loads, which do not share the vector-memory counter.
__device__ inline uint64_t wave_uniform(uint64_t x) {
  return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(x >> 32)) << 32) |
         (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)x);
}

// symbol j (0..3) of an 8-byte group
// Inclusive prefix sum over the 64 lanes of a wavefront with DPP moves:
// shifts by 1, 2, 4 and 8 lanes within each row of 16, then lane 15 of a row
// added to the row after it (rows 1 and 3) and lane 31 to rows 2 and 3.
// Lanes without a source read 0.
__device__ inline uint32_t wave_inclusive_sum(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

// Lane shuffle of a 64-bit value: lane l reads lane l ^ m (m < 64).
__device__ inline uint64_t shfl_xor_u64(uint64_t x, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, m), hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), m);
  return (uint64_t)hi << 32 | lo;
}

// Sum over the 64 lanes of a wavefront, the same in every lane.
__device__ inline uint32_t wave_sum(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readlane((int)wave_inclusive_sum(x), 63);
}

__device__ inline uint32_t group_sym(uint2 g, int j) {
  const uint32_t w = j < 2 ? g.x : g.y;
  return (j & 1) ? (w >> 16) : (w & 0xffffu);
}

__device__ __forceinline__ void k_histogram(G3 mg_bid, G3 mg_gdim, const uint16_t* __restrict__ sym, uint64_t n, int dict,
                                                      int chunk, uint64_t k0, uint64_t nch,
                                                      unsigned long long* __restrict__ hist,
                                                      uint32_t* __restrict__ chunk_esc,
                                                      uint32_t* __restrict__ status) {
  __shared__ uint32_t sh[MAXDICT];
  for (int b = threadIdx.x; b < dict; b += WAVE_T) sh[b] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)mg_gdim.x * WAVES;
  const uint64_t wave = (uint64_t)mg_bid.x * WAVES + (threadIdx.x >> 6);
  bool bad = false;
  // full chunks of at most 1024 symbols: batched, prefetched loads
  uint64_t kslow = k0 + wave;  // first chunk left to the per-step loop below
  if (chunk <= 1024) {
    const uint64_t kfull = min(nch, n / (uint64_t)chunk);
    const int steps = chunk / 256;
    walk_full_chunks(sym, chunk, k0 + wave, kfull, stride, lane, [&](uint64_t k, const uint2 (&v)[4]) {
      uint32_t e = 0;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        if (st >= steps) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t x = group_sym(v[st], j);
          if (x < (uint32_t)dict)
            atomicAdd(&sh[x], 1u);
          else
            bad = true;  // symbol outside the dictionary
          e += x == 0;
        }
      }
      chunk_esc[k] = wave_sum(e);
    });
    // the ragged last chunk, if any, goes to the wave whose turn it is
    kslow = k0 + wave;
    if (kslow < kfull) kslow += ((kfull - kslow + stride - 1) / stride) * stride;
  }
  for (uint64_t k = kslow; k < nch; k += stride) {
    const uint64_t beg = k * (uint64_t)chunk;
    const uint64_t end = min(beg + (uint64_t)chunk, n);
    uint32_t e = 0;
    for (uint64_t i = beg + 4 * (uint64_t)lane; i < end; i += 256) {
      uint32_t s4[4];
      load4_symbols(sym, i, end, s4);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t v = s4[j];
        if (v == 0xffffffffu) continue;
        if (v < (uint32_t)dict)
          atomicAdd(&sh[v], 1u);
        else
          bad = true;  // symbol outside the dictionary
        e += v == 0;
      }
    }
#pragma unroll
    for (int d = 32; d; d >>= 1) e += __shfl_xor(e, d);
    if (lane == 0) chunk_esc[k] = e;
  }
  if (bad) atomicOr(status, 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < dict; b += WAVE_T)
    if (sh[b]) atomicAdd(&hist[b], (unsigned long long)sh[b]);
}

__global__ void __launch_bounds__(WAVE_T) k_histogram_k(const uint16_t* __restrict__ sym, uint64_t n, int dict,
                                                      int chunk, uint64_t k0, uint64_t nch,
                                                      unsigned long long* __restrict__ hist,
                                                      uint32_t* __restrict__ chunk_esc,
                                                      uint32_t* __restrict__ status) {
  k_histogram(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, sym, n, dict, chunk, k0, nch, hist, chunk_esc, status);
}


// ------------------------------------------------------------------ wave helpers
// The encoder's table entry of a code of length L (0: unused symbol or a code
// longer than ENC_MAXLEN, which the generic encoder handles).
__device__ inline uint32_t pack_code(uint32_t L, uint64_t c) {
  if (!L || L > (uint32_t)ENC_MAXLEN) return 0u;
  return L <= (uint32_t)ENC_PACKLEN ? (uint32_t)((c << 6) | L) : ENC_LONG;
}

__device__ inline uint64_t lanes_below(int lane) { return lane ? (~0ull >> (64 - lane)) : 0ull; }

// Mask of the lanes whose `v` (7 bits) equals this lane's.
__device__ inline uint64_t match7(uint32_t v) {
  uint64_t m = __ballot(1);
#pragma unroll
  for (int b = 0; b < 7; ++b) {
    const bool bit = (v >> b) & 1u;
    const uint64_t bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

// Canonical ranks, for a block of 1024 threads: for every symbol s with
// lens[s] in 1..MAXLEN, rank[s] = the number of symbols t < s of the same
// length; cnt[L] = the number of symbols of length L (cnt[0] counts the unused
// ones).  Wave w owns a contiguous range of 64-symbol groups, so ranks are
// per-wave counts plus the counts of the waves before it.
__device__ void canonical_ranks(const uint8_t* lens, int dict, uint16_t* rank,
                                uint32_t (*wcnt)[MAXLEN + 1], uint32_t* cnt) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int ngroups = (dict + 63) / 64;
  const int gpw = (ngroups + 15) / 16;
  const int g0 = min(w * gpw, ngroups), g1 = min(g0 + gpw, ngroups);
  for (int i = t; i < 16 * (MAXLEN + 1); i += blockDim.x) wcnt[i / (MAXLEN + 1)][i % (MAXLEN + 1)] = 0;
  __syncthreads();
  for (int g = g0; g < g1; ++g) {
    const int s = g * 64 + lane;
    if (s < dict) atomicAdd(&wcnt[w][lens[s]], 1u);
  }
  __syncthreads();
  if (t <= MAXLEN) {
    uint32_t run = 0;
    for (int v = 0; v < 16; ++v) {
      const uint32_t x = wcnt[v][t];
      wcnt[v][t] = run;
      run += x;
    }
    cnt[t] = run;
  }
  __syncthreads();
  volatile uint32_t* mine = wcnt[w];
  const uint64_t below = lanes_below(lane);
  for (int g = g0; g < g1; ++g) {
    const int s = g * 64 + lane;
    const uint32_t L = s < dict ? lens[s] : 0u;
    const uint64_t m = match7(L);
    const uint32_t r = (uint32_t)__popcll(m & below);
    const uint32_t base = mine[L];
    if (L) rank[s] = (uint16_t)(base + r);
    __builtin_amdgcn_wave_barrier();
    if (r == 0) mine[L] = base + (uint32_t)__popcll(m);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
}

// ------------------------------------------------------------------ codebook
constexpr int MERGE_SEQ_MIN = 8;    // smaller batches are built by one thread ...
constexpr int MERGE_SEQ_RUN = 64;   // ... this many nodes at a time
constexpr int MERGE_PER = MAXDICT / 1024;  // batch nodes per thread

// Number of leaves among the first p items of the stable merge (ties to the
// leaf) of leaves keys[K..n) (sorted) and internal nodes keys[0..K), p >= 2K:
// every leaf below slot K is among them, and no internal node from K on is.
__device__ inline int merge_split(const uint64_t* keys, int n, int K, int p) {
  int lo = max(0, p - K), hi = min(p, n);
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (keys[mid] <= keys[p - mid - 1])
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// First x in [lo, hi) with pred(x) true (hi when there is none), for a pred
// that is false and then true along the range: the 64 lanes of one wavefront
// test 64 evenly spaced points per step, so a range of 8192 takes three steps.
// Every lane returns the same x.
template <typename P>
__device__ inline int wave_first(int lo, int hi, P pred) {
  const int lane = threadIdx.x & 63;
  while (lo < hi) {
    const int step = (hi - lo + 63) >> 6;
    const int x = lo + lane * step;
    const uint64_t m = __ballot(x >= hi || pred(x));
    if (m == 0) {  // every point tested is false, the last one below hi
      lo += 63 * step + 1;
      continue;
    }
    const int f = __ffsll((unsigned long long)m) - 1;
    if (f == 0) return lo;
    hi = min(lo + f * step, hi);
    lo += (f - 1) * step + 1;
  }
  return lo;
}

// One workgroup of 1024 threads; everything stays in LDS.  keys: (count << 16
// | symbol), empty bins sort last.  The merge builds internal nodes in
// batches (see below); internal-node depths come from pointer jumping, leaf
// lengths from the number of leaves per depth (deepest for the smallest
// weights), canonical codes from per-length ranks in symbol order.
// When enc is given, the encoder's packed table (code << 6 | length, 0 for an
// unused symbol or a code longer than ENC_MAXLEN) and the longest length go to
// enc and *maxlen_out as well.
__device__ __forceinline__ void codebook_block(const uint64_t* __restrict__ hist, int dict,
                                               uint8_t* __restrict__ len_out, uint64_t* __restrict__ codes,
                                               uint32_t* __restrict__ enc, uint32_t* __restrict__ maxlen_out) {
  __shared__ uint64_t keys[MAXDICT];
  __shared__ uint16_t syms[MAXDICT];
  __shared__ uint16_t par[MAXDICT];  // parents, then canonical ranks
  __shared__ uint8_t dep[MAXDICT];
  __shared__ uint8_t lens[MAXDICT];
  __shared__ uint32_t wcnt[16][MAXLEN + 1];
  __shared__ int nleaf;
  __shared__ int merge_k, merge_b;
  __shared__ uint32_t icount[MAXLEN + 2];
  __shared__ uint32_t lstart[MAXLEN + 2];
  __shared__ uint64_t first[MAXLEN + 1];
  __shared__ uint32_t lcount[MAXLEN + 1];
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  if (t == 0) nleaf = 0;
  for (int i = t; i <= MAXLEN + 1; i += nt) icount[i] = 0;
  __syncthreads();
  // Used symbols only, as keys (count << 16 | symbol), packed in any order
  // (one LDS atomic per wavefront); the keys are distinct, so the sort below
  // fixes their order.
  {
    const int lane = t & 63;
    for (int s0 = 0; s0 < dict; s0 += nt) {
      const int s = s0 + t;
      const uint64_t c = s < dict ? hist[s] : 0;
      if (s < dict) lens[s] = 0;
      const uint64_t m = __ballot(c != 0);
      int base = 0;
      if (lane == 0 && m) base = atomicAdd(&nleaf, __popcll(m));
      base = __shfl(base, 0);
      if (c) keys[base + __popcll(m & lanes_below(lane))] = (c << 16) | (uint64_t)s;
    }
  }
  __syncthreads();
  const int n = nleaf;
  // Bitonic sort of the next power of two P >= n keys (padding sorts last).
  // Thread t holds positions 8t .. 8t+7 in registers: partners closer than 8
  // are exchanged in registers, partners 8 .. 256 apart sit in the same
  // wavefront and come through lane shuffles, and only partners 512 or more
  // apart go through LDS (two barriers a pass).  Positions at or past P never
  // meet a real key in a stage k <= P, so every thread runs every pass.
  {
    int P = 1;
    while (P < n) P <<= 1;
    const int e0 = t * CB_KPT;
    uint64_t v[CB_KPT];
#pragma unroll
    for (int r = 0; r < CB_KPT; ++r) v[r] = e0 + r < n ? keys[e0 + r] : ~0ull;
    for (int k = 2; k <= P; k <<= 1) {
      for (int j = k >> 1; j >= CB_KPT; j >>= 1) {
        uint64_t o[CB_KPT];
        if (j >= CB_KPT * 64) {
          __syncthreads();
#pragma unroll
          for (int r = 0; r < CB_KPT; ++r) keys[e0 + r] = v[r];
          __syncthreads();
#pragma unroll
          for (int r = 0; r < CB_KPT; ++r) o[r] = keys[(e0 + r) ^ j];
        } else {
#pragma unroll
          for (int r = 0; r < CB_KPT; ++r) o[r] = shfl_xor_u64(v[r], j / CB_KPT);
        }
        // the partner shares bit k, so the pair's direction is known here
        const bool up = (e0 & k) == 0, lower = (e0 & j) == 0;
#pragma unroll
        for (int r = 0; r < CB_KPT; ++r) v[r] = lower == up ? min(v[r], o[r]) : max(v[r], o[r]);
      }
#pragma unroll
      for (int J = CB_KPT / 2; J; J >>= 1) {
        if (J >= k) continue;
#pragma unroll
        for (int r = 0; r < CB_KPT; ++r) {
          if (r & J) continue;
          const bool up = ((e0 + r) & k) == 0;
          const uint64_t a = v[r], b = v[r | J];
          const bool sw = (a > b) == up;
          v[r] = sw ? b : a;
          v[r | J] = sw ? a : b;
        }
      }
    }
    __syncthreads();  // the last LDS pass's reads are done
#pragma unroll
    for (int r = 0; r < CB_KPT; ++r) {
      const int e = e0 + r;
      if (e < n) {
        syms[e] = (uint16_t)(v[r] & 0xffff);
        keys[e] = v[r] >> 16;
      } else if (e < P) {
        keys[e] = ~0ull;
      }
    }
  }
  __syncthreads();
  if (n == 1) {
    if (t == 0) lens[syms[0]] = 1;
  } else if (n > 1) {
    // The two-queue merge consumes the stable merge (ties to the leaf) of the
    // sorted leaves and the internal nodes in creation order, and internal
    // node k joins that merge's items 2k and 2k+1.  So, with K nodes built,
    // nodes K .. K+B-1 follow from the merge of the leaves with nodes < K, as
    // long as their items lie before the point where node K itself enters
    // (after every leaf of weight <= its own): they are built in parallel.
    // When B is small a single thread builds a sequential stretch instead.
    // Node k is stored in slot k (its leaf is consumed by then); parents of
    // internal nodes go to par[].
    if (t == 0) merge_k = 0;
    __syncthreads();
    for (;;) {
      const int K = merge_k;
      if (K >= n - 1) break;
      if (t < 64) {
        // the first wavefront finds where node K enters the merge
        const int p = 2 * K;
        int a = wave_first(max(0, p - K), min(p, n), [&](int x) { return keys[x] > keys[p - x - 1]; }), b = p - a;
        uint64_t w = 0;
        for (int pick = 0; pick < 2; ++pick) {
          if (a < n && (b >= K || keys[a] <= keys[b]))
            w += keys[a++];
          else
            w += keys[b++];
        }
        // leaves of weight <= w: those below slot K all are (they come before node K)
        const int lo = wave_first(K, n, [&](int x) { return keys[x] > w; });
        const int enter = K + lo;  // merge position of node K
        const int B = min(max(1, (enter - 2 * K) / 2), n - 1 - K);
        if (B >= MERGE_SEQ_MIN) {
          if (t == 0) merge_b = B;
        } else if (t == 0) {
          a = merge_split(keys, n, K, p);
          b = p - a;
          const int end = min(K + MERGE_SEQ_RUN, n - 1);
          for (int node = K; node < end; ++node) {
            uint64_t v = 0;
            for (int pick = 0; pick < 2; ++pick) {
              if (a < n && (b >= node || keys[a] <= keys[b])) {
                v += keys[a++];
              } else {
                par[b] = (uint16_t)node;
                v += keys[b++];
              }
            }
            keys[node] = v;
          }
          merge_b = -(end - K);
        }
      }
      __syncthreads();
      const int B = merge_b;
      if (B > 0) {
        // thread t builds nodes K + j0 .. K + j0 + m - 1: one split search for
        // the first, then the next 2m merge items in order
        const int m = (B + nt - 1) / nt;
        const int j0 = t * m;
        uint64_t w[MERGE_PER];
        if (j0 < B) {
          const int p = 2 * (K + j0);
          int a = merge_split(keys, n, K, p), b = p - a;
#pragma unroll
          for (int q = 0; q < MERGE_PER; ++q) {
            w[q] = 0;
            if (q < m && j0 + q < B) {
              for (int pick = 0; pick < 2; ++pick) {
                if (a < n && (b >= K || keys[a] <= keys[b])) {
                  w[q] += keys[a++];
                } else {
                  par[b] = (uint16_t)(K + j0 + q);
                  w[q] += keys[b++];
                }
              }
            }
          }
        }
        __syncthreads();
        if (j0 < B) {
#pragma unroll
          for (int q = 0; q < MERGE_PER; ++q)
            if (q < m && j0 + q < B) keys[K + j0 + q] = w[q];
        }
      }
      if (t == 0) merge_k = K + (B > 0 ? B : -B);
      __syncthreads();
    }
    // internal node k < n-1: parent in par[k]; the root n-2 is its own parent
    const int ni = n - 1;
    for (int k = t; k < ni; k += nt) {
      if (k == ni - 1) par[k] = (uint16_t)k;
      dep[k] = k == ni - 1 ? 0 : 1;
    }
    __syncthreads();
    for (int step = 1; step < ni; step <<= 1) {  // pointer jumping: depth = hops to the root
      int nd[8], np[8];
      int c = 0;
      for (int k = t; k < ni; k += nt, ++c) {
        const int p = par[k];
        nd[c] = dep[k] + dep[p];
        np[c] = par[p];
      }
      __syncthreads();
      c = 0;
      for (int k = t; k < ni; k += nt, ++c) {
        dep[k] = (uint8_t)nd[c];
        par[k] = (uint16_t)np[c];
      }
      __syncthreads();
    }
    for (int k = t; k < ni; k += nt) atomicAdd(&icount[dep[k]], 1u);
    __syncthreads();
    if (t == 0) {
      // leaves at depth d: 2 * (internal nodes at depth d-1) - (internal nodes at depth d);
      // the smallest weights take the deepest leaves
      uint32_t start = 0;
      for (int d = MAXLEN; d >= 1; --d) {
        const uint32_t leaves = 2 * icount[d - 1] - icount[d];
        lstart[d] = start;
        start += leaves;
      }
      lstart[0] = start;
    }
    __syncthreads();
    for (int i = t; i < n; i += nt) {
      // leaf i has length d with lstart[d] <= i < lstart[d-1]; lstart does not
      // rise with d, so d is the smallest depth with lstart[d] <= i
      int lo = 1, hi = MAXLEN;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (lstart[mid] <= (uint32_t)i)
          hi = mid;
        else
          lo = mid + 1;
      }
      lens[syms[i]] = (uint8_t)lo;
    }
  }
  __syncthreads();
  // canonical codes: consecutive codes per length in symbol order
  canonical_ranks(lens, dict, par, wcnt, lcount);
  if (t == 0) {
    uint64_t code = 0;
    for (int b = 1; b <= MAXLEN; ++b) {
      code = (code + (b > 1 ? lcount[b - 1] : 0)) << 1;
      first[b] = code;
    }
  }
  __syncthreads();
  uint32_t mine = 0;
  for (int s = t; s < dict; s += nt) {
    const int L = lens[s];
    const uint64_t c = L ? first[L] + (uint64_t)par[s] : 0ull;
    len_out[s] = (uint8_t)L;
    codes[s] = c;
    if (enc) enc[s] = pack_code(L, c);
    mine = max(mine, (uint32_t)L);
  }
  if (enc) {
    __shared__ uint32_t mx;
    if (t == 0) mx = 0;
    __syncthreads();
    if (mine) atomicMax(&mx, mine);
    __syncthreads();
    if (t == 0) *maxlen_out = mx;
  }
}

__device__ __forceinline__ void k_codebook(G3 mg_bid, G3 mg_gdim, const uint64_t* __restrict__ hist, int dict,
                                                   uint8_t* __restrict__ len_out, uint64_t* __restrict__ codes,
                                                   uint32_t* __restrict__ enc, uint32_t* __restrict__ maxlen_out) {
  codebook_block(hist, dict, len_out, codes, enc, maxlen_out);
}

__global__ void __launch_bounds__(CB_T) k_codebook_k(const uint64_t* __restrict__ hist, int dict,
                                                   uint8_t* __restrict__ len_out, uint64_t* __restrict__ codes,
                                                   uint32_t* __restrict__ enc, uint32_t* __restrict__ maxlen_out) {
  k_codebook(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, hist, dict, len_out, codes, enc, maxlen_out);
}


// One codebook per block: the codebooks of a batch's fields in one launch.

// ------------------------------------------------------------------ chunk sizes
// Bits of each chunk: one wave per chunk, code lengths in LDS.
__device__ __forceinline__ void k_chunk_bits(G3 mg_bid, G3 mg_gdim, const uint16_t* __restrict__ sym, uint64_t n, int chunk,
                                                       uint64_t nch, uint32_t mask, const uint8_t* __restrict__ len,
                                                       uint32_t* __restrict__ chunk_bits) {
  __shared__ uint8_t lens[MAXDICT];
  for (uint32_t s = threadIdx.x; s <= mask; s += WAVE_T) lens[s] = len[s];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)mg_gdim.x * WAVES;
  const uint64_t wave = (uint64_t)mg_bid.x * WAVES + (threadIdx.x >> 6);
  // full chunks of at most 1024 symbols: batched, prefetched loads
  uint64_t kslow = wave;
  if (chunk <= 1024) {
    const uint64_t kfull = min(nch, n / (uint64_t)chunk);
    const int steps = chunk / 256;
    walk_full_chunks(sym, chunk, wave, kfull, stride, lane, [&](uint64_t k, const uint2 (&v)[4]) {
      uint32_t b = 0;
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        if (st >= steps) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) b += lens[group_sym(v[st], j) & mask];
      }
      chunk_bits[k] = wave_sum(b);
    });
    if (kslow < kfull) kslow += ((kfull - kslow + stride - 1) / stride) * stride;
  }
  for (uint64_t k = kslow; k < nch; k += stride) {
    const uint64_t beg = k * (uint64_t)chunk;
    const uint64_t end = min(beg + (uint64_t)chunk, n);
    uint32_t b = 0;
    for (uint64_t i = beg + 4 * (uint64_t)lane; i < end; i += 256) {
      uint32_t s4[4];
      load4_symbols(sym, i, end, s4);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (s4[j] != 0xffffffffu) b += lens[s4[j] & mask];
    }
#pragma unroll
    for (int d = 32; d; d >>= 1) b += __shfl_xor(b, d);
    if (lane == 0) chunk_bits[k] = b;
  }
}

__global__ void __launch_bounds__(WAVE_T) k_chunk_bits_k(const uint16_t* __restrict__ sym, uint64_t n, int chunk,
                                                       uint64_t nch, uint32_t mask, const uint8_t* __restrict__ len,
                                                       uint32_t* __restrict__ chunk_bits) {
  k_chunk_bits(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, sym, n, chunk, nch, mask, len, chunk_bits);
}


// ------------------------------------------------------------------ scans
// Exclusive scan of n values (the words of chunk bit counts when WORDS) into
// off[0..n], off[n] the total, in three launches: tile sums parked in the
// first output slot of each tile, a one-block scan of those, and a per-tile
// scan that adds its tile's base.
constexpr int SCAN_T = 256, SCAN_PER = 16, SCAN_TILE = SCAN_T * SCAN_PER;

template <bool WORDS>
__device__ inline uint64_t scan_value(uint32_t x) {
  return WORDS ? (((uint64_t)x + 31u) >> 5) : (uint64_t)x;
}

__device__ inline uint64_t block_exclusive_scan(uint64_t v, uint64_t* sh, uint64_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < (int)blockDim.x; d <<= 1) {
    const uint64_t a = t >= d ? sh[t - d] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const uint64_t incl = sh[t];
  *total = sh[blockDim.x - 1];
  __syncthreads();
  return incl - v;
}

template <bool WORDS>
__global__ void __launch_bounds__(SCAN_T) k_scan_tiles(const uint32_t* __restrict__ v, uint64_t n,
                                                       uint64_t* __restrict__ off) {
  __shared__ uint64_t sh[SCAN_T];
  const uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
  // every load from an index clamped into [0, n), issued before any is used
  uint32_t raw[SCAN_PER];
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) raw[j] = v[min(base + (uint64_t)j * SCAN_T + threadIdx.x, n - 1)];
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    const uint64_t i = base + (uint64_t)j * SCAN_T + threadIdx.x;
    if (i < n) s += scan_value<WORDS>(raw[j]);
  }
  uint64_t total;
  block_exclusive_scan(s, sh, &total);
  if (threadIdx.x == 0) off[base] = total;
}

__global__ void __launch_bounds__(1024) k_scan_top(uint64_t* __restrict__ off, uint64_t n) {
  __shared__ uint64_t sh[1024];
  const uint64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
  uint64_t carry = 0;
  for (uint64_t g = 0; g < nt; g += blockDim.x) {
    const uint64_t b = g + threadIdx.x;
    const uint64_t x = b < nt ? off[b * SCAN_TILE] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(x, sh, &total);
    if (b < nt) off[b * SCAN_TILE] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) off[n] = carry;
}

template <bool WORDS>
__global__ void __launch_bounds__(SCAN_T) k_scan_apply(const uint32_t* __restrict__ v, uint64_t n,
                                                       uint64_t* __restrict__ off) {
  __shared__ uint64_t sh[SCAN_T];
  __shared__ uint64_t tbase_sh;
  const uint64_t tile = (uint64_t)blockIdx.x * SCAN_TILE;
  // only thread 0 reads the parked base: it is also the thread that overwrites it
  if (threadIdx.x == 0) tbase_sh = off[tile];
  const uint64_t mine = tile + (uint64_t)threadIdx.x * SCAN_PER;
  uint32_t raw[SCAN_PER];
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) raw[j] = v[min(mine + j, n - 1)];
  uint64_t x[SCAN_PER];
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    x[j] = mine + j < n ? scan_value<WORDS>(raw[j]) : 0;
    s += x[j];
  }
  uint64_t total;
  uint64_t run = block_exclusive_scan(s, sh, &total);  // its barriers publish tbase_sh
  run += tbase_sh;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    if (mine + j < n) off[mine + j] = run;
    run += x[j];
  }
}

// Both scans of the compression path in one sequence of launches: blockIdx.y
// 0 scans the chunk word counts (ceil(bits / 32)) of a into oa, 1 the values
// of b into ob.
struct ScanPair {
  const uint32_t* v[2];
  uint64_t* off[2];
};

__device__ __forceinline__ void k_scan_tiles2(G3 mg_bid, G3 mg_gdim, const ScanPair& p, uint64_t n) {
  __shared__ uint64_t sh[SCAN_T];
  const int y = mg_bid.y;
  const uint32_t* __restrict__ v = p.v[y];
  const uint64_t base = (uint64_t)mg_bid.x * SCAN_TILE;
  // every load from an index clamped into [0, n), issued before any is used
  uint32_t raw[SCAN_PER];
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) raw[j] = v[min(base + (uint64_t)j * SCAN_T + threadIdx.x, n - 1)];
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    const uint64_t i = base + (uint64_t)j * SCAN_T + threadIdx.x;
    if (i < n) s += y == 0 ? scan_value<true>(raw[j]) : scan_value<false>(raw[j]);
  }
  uint64_t total;
  block_exclusive_scan(s, sh, &total);
  if (threadIdx.x == 0) p.off[y][base] = total;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_tiles2_k(ScanPair p, uint64_t n) {
  k_scan_tiles2(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, p, n);
}


__device__ __forceinline__ void k_scan_top2(G3 mg_bid, G3 mg_gdim, const ScanPair& p, uint64_t n) {
  __shared__ uint64_t sh[1024];
  uint64_t* __restrict__ off = p.off[mg_bid.y];
  const uint64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
  uint64_t carry = 0;
  for (uint64_t g = 0; g < nt; g += blockDim.x) {
    const uint64_t b = g + threadIdx.x;
    const uint64_t x = b < nt ? off[b * SCAN_TILE] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(x, sh, &total);
    if (b < nt) off[b * SCAN_TILE] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) off[n] = carry;
}

__global__ void __launch_bounds__(1024) k_scan_top2_k(ScanPair p, uint64_t n) {
  k_scan_top2(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, p, n);
}


__device__ __forceinline__ void k_scan_apply2(G3 mg_bid, G3 mg_gdim, const ScanPair& p, uint64_t n) {
  __shared__ uint64_t sh[SCAN_T];
  __shared__ uint64_t tbase_sh;
  const int y = mg_bid.y;
  const uint32_t* __restrict__ v = p.v[y];
  uint64_t* __restrict__ off = p.off[y];
  const uint64_t tile = (uint64_t)mg_bid.x * SCAN_TILE;
  if (threadIdx.x == 0) tbase_sh = off[tile];
  const uint64_t mine = tile + (uint64_t)threadIdx.x * SCAN_PER;
  uint32_t raw[SCAN_PER];
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) raw[j] = v[min(mine + j, n - 1)];
  uint64_t x[SCAN_PER];
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    x[j] = mine + j < n ? (y == 0 ? scan_value<true>(raw[j]) : scan_value<false>(raw[j])) : 0;
    s += x[j];
  }
  uint64_t total;
  uint64_t run = block_exclusive_scan(s, sh, &total);  // its barriers publish tbase_sh
  run += tbase_sh;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    if (mine + j < n) off[mine + j] = run;
    run += x[j];
  }
}

__global__ void __launch_bounds__(SCAN_T) k_scan_apply2_k(ScanPair p, uint64_t n) {
  k_scan_apply2(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, p, n);
}


template <bool WORDS>
void launch_scan(const uint32_t* v, uint64_t n, uint64_t* off, hipStream_t st) {
  const uint64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nt) hipLaunchKernelGGL(k_scan_tiles<WORDS>, dim3((unsigned)nt), dim3(SCAN_T), 0, st, v, n, off);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, off, n);
  if (nt) hipLaunchKernelGGL(k_scan_apply<WORDS>, dim3((unsigned)nt), dim3(SCAN_T), 0, st, v, n, off);
  MG_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ encode
// Codes of at most ENC_MAXLEN bits are packed with their length into one word
// (code << 6 | length), by the codebook kernel or by k_pack_codes, which also
// record the longest length: it decides on the device which encode kernel
// does the work.
constexpr int ENC_CHUNK = 1024;                          // largest chunk of the wave kernel
constexpr int ENC_WORDS = ENC_CHUNK * ENC_MAXLEN / 32;   // its LDS words per wave
constexpr int ENC_T = 512;

// The stored code of an escaped value (|q| >= R): 2 (|q| - R) + [q < 0].
__device__ inline uint64_t escape_code(int64_t q, int R) {
  const uint64_t a = q < 0 ? (uint64_t)0 - (uint64_t)q : (uint64_t)q;
  return 2 * (a - (uint64_t)R) + (q < 0 ? 1u : 0u);
}

__global__ void __launch_bounds__(1024) k_pack_codes(const uint8_t* __restrict__ len, const uint64_t* __restrict__ codes,
                                                     int dict, uint32_t* __restrict__ enc,
                                                     uint32_t* __restrict__ maxlen_out) {
  __shared__ uint32_t mx;
  if (threadIdx.x == 0) mx = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < dict; s += blockDim.x) {
    const uint32_t L = len[s];
    if (L) atomicMax(&mx, L);
    enc[s] = pack_code(L, codes[s]);
  }
  __syncthreads();
  if (threadIdx.x == 0) *maxlen_out = mx;
}

// One wave per chunk (chunk <= ENC_CHUNK, codes <= ENC_MAXLEN bits): each lane
// takes four consecutive symbols per step, a wave scan gives its bit offset,
// and its codes pass through a 64-bit accumulator into the wave's LDS words
// (word-granular atomics: only the first and last word of a lane are shared);
// the finished chunk is copied out coalesced.
__device__ __forceinline__ void k_encode_wave(G3 mg_bid, G3 mg_gdim, const uint16_t* __restrict__ sym, uint64_t n, int chunk,
                                                      uint64_t nch, uint32_t mask, const uint32_t* __restrict__ enc_g,
                                                      const uint32_t* __restrict__ maxlen,
                                                      const uint8_t* __restrict__ len_g,
                                                      const uint64_t* __restrict__ codes_g,
                                                      const uint64_t* __restrict__ word_off,
                                                      uint32_t* __restrict__ payload,
                                                      const uint64_t* __restrict__ esc_off,
                                                      const int64_t* __restrict__ qside,
                                                      uint64_t* __restrict__ ecodes, int R) {
  if (*maxlen > (uint32_t)ENC_MAXLEN) return;  // the generic kernel encodes instead
  __shared__ uint32_t enc[MAXDICT];
  __shared__ uint32_t words[ENC_T / 64][ENC_WORDS];
  for (uint32_t s = threadIdx.x; s <= mask; s += ENC_T) enc[s] = enc_g[s];
  __syncthreads();
  uint64_t* outliers = ecodes;
  const int lane = threadIdx.x & 63;
  uint32_t* wb = words[threadIdx.x >> 6];
  const uint64_t stride = (uint64_t)mg_gdim.x * (ENC_T / 64);
  const uint64_t wave = (uint64_t)mg_bid.x * (ENC_T / 64) + (threadIdx.x >> 6);
  // chunk k: clear its LDS words; per step of 256 symbols (first symbol i of
  // this lane, s4 its four symbols, 0xffffffff past the end) pack the codes;
  // then copy the words out
  uint64_t w0 = 0, eo = 0;
  uint32_t nw = 0, base = 0;  // base: chunk bit offset of the step's first symbol
  auto open_chunk = [&](uint64_t kk) {
    const uint64_t k = wave_uniform(kk);
    w0 = word_off[k];
    nw = (uint32_t)min(word_off[k + 1] - w0, (uint64_t)ENC_WORDS);
    for (uint32_t i = lane; i < nw; i += 64) wb[i] = 0;
    __builtin_amdgcn_wave_barrier();
    base = 0;
    eo = outliers ? esc_off[k] : 0;
  };
  auto close_chunk = [&]() {
    __builtin_amdgcn_wave_barrier();
    for (uint32_t i = lane; i < nw; i += 64) payload[w0 + i] = wb[i];
    __builtin_amdgcn_wave_barrier();
  };
  auto step = [&](uint64_t i, const uint32_t (&s4)[4]) {
    uint32_t L4[4], c4[4];
    uint32_t bits = 0, esc = 0, longc = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t e = s4[j] != 0xffffffffu ? enc[s4[j] & mask] : 0u;
      L4[j] = e & 63u;
      c4[j] = e >> 6;
      longc |= L4[j] == ENC_LONG ? 1u : 0u;
      esc += s4[j] == 0;
    }
    if (longc) {  // codes longer than ENC_PACKLEN bits (rare): the full tables
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (L4[j] == ENC_LONG) {
          const uint32_t s = s4[j] & mask;
          L4[j] = len_g[s];
          c4[j] = (uint32_t)codes_g[s];
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) bits += L4[j];
    const uint32_t bi = wave_inclusive_sum(bits), ei = wave_inclusive_sum(esc);
    const uint32_t off = base + bi - bits;
    uint32_t wi = off >> 5;
    int fill = (int)(off & 31u);
    uint64_t acc = 0;  // left-aligned at word wi
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int L = (int)L4[j];
      if (L) {
        acc |= (uint64_t)c4[j] << (64 - fill - L);
        fill += L;
        if (fill >= 32) {
          if (wi < ENC_WORDS) atomicOr(&wb[wi], (uint32_t)(acc >> 32));
          acc <<= 32;
          fill -= 32;
          ++wi;
        }
      }
    }
    if (fill > 0 && wi < ENC_WORDS) atomicOr(&wb[wi], (uint32_t)(acc >> 32));
    if (outliers && esc) {
      uint64_t o = eo + (ei - esc);
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (s4[j] == 0) outliers[o++] = escape_code(qside[i + j], R);
    }
    eo += (uint32_t)__builtin_amdgcn_readlane(ei, 63);
    base += (uint32_t)__builtin_amdgcn_readlane(bi, 63);
  };
  // full chunks: batched, prefetched loads (every chunk here is at most 1024)
  const uint64_t kfull = min(nch, n / (uint64_t)chunk);
  const int steps = chunk / 256;
  walk_full_chunks(sym, chunk, wave, kfull, stride, lane, [&](uint64_t k, const uint2 (&v)[4]) {
    open_chunk(k);
    const uint64_t beg = k * (uint64_t)chunk + 4 * (uint64_t)lane;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      if (st >= steps) break;
      const uint32_t s4[4] = {group_sym(v[st], 0), group_sym(v[st], 1), group_sym(v[st], 2), group_sym(v[st], 3)};
      step(beg + 256 * (uint64_t)st, s4);
    }
    close_chunk();
  });
  // the ragged last chunk, if any
  uint64_t kslow = wave;
  if (kslow < kfull) kslow += ((kfull - kslow + stride - 1) / stride) * stride;
  for (uint64_t k = kslow; k < nch; k += stride) {
    const uint64_t beg = k * (uint64_t)chunk;
    const uint64_t end = min(beg + (uint64_t)chunk, n);
    open_chunk(k);
    for (uint64_t i0 = beg; i0 < end; i0 += 256) {
      const uint64_t i = i0 + 4 * (uint64_t)lane;
      uint32_t s4[4];
      load4_symbols(sym, i, end, s4);
      step(i, s4);
    }
    close_chunk();
  }
}

__global__ void __launch_bounds__(ENC_T) k_encode_wave_k(const uint16_t* __restrict__ sym, uint64_t n, int chunk,
                                                      uint64_t nch, uint32_t mask, const uint32_t* __restrict__ enc_g,
                                                      const uint32_t* __restrict__ maxlen,
                                                      const uint8_t* __restrict__ len_g,
                                                      const uint64_t* __restrict__ codes_g,
                                                      const uint64_t* __restrict__ word_off,
                                                      uint32_t* __restrict__ payload,
                                                      const uint64_t* __restrict__ esc_off,
                                                      const int64_t* __restrict__ qside,
                                                      uint64_t* __restrict__ ecodes, int R) {
  k_encode_wave(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, sym, n, chunk, nch, mask, enc_g, maxlen, len_g, codes_g, word_off, payload, esc_off, qside, ecodes, R);
}


__device__ inline void put_code(uint32_t* words, uint64_t b, int L, uint64_t code) {
  // code occupies chunk bits [b, b+L), MSB-first
  const uint64_t e = b + (uint64_t)L;
  for (uint64_t w = b >> 5; (w << 5) < e; ++w) {
    const uint64_t ws = w << 5, we = ws + 32;
    const uint64_t s0 = b > ws ? b : ws;
    const uint64_t s1 = e < we ? e : we;
    const int nb = (int)(s1 - s0);
    uint64_t part = code >> (e - s1);
    part &= (nb >= 64) ? ~0ull : ((1ull << nb) - 1ull);
    atomicOr(&words[w], (uint32_t)(part << (we - s1)));
  }
}

// MAXW: LDS words of one chunk, chunk * MAXLEN / 32 for the largest chunk of the instantiation.
// Generic encoder (any chunk size and code length); it stands aside when the
// wave kernel handles the call (chunk <= ENC_CHUNK and codes <= ENC_MAXLEN bits).
template <int MAXW>
__device__ __forceinline__ void k_encode(G3 mg_bid, G3 mg_gdim, const uint16_t* __restrict__ sym, uint64_t n, int chunk,
                                                uint64_t nch, uint32_t mask, const uint8_t* __restrict__ len,
                                                const uint32_t* __restrict__ maxlen,
                                                const uint64_t* __restrict__ codes,
                                                const uint64_t* __restrict__ word_off,
                                                uint32_t* __restrict__ payload,
                                                const uint64_t* __restrict__ esc_off,
                                                const int64_t* __restrict__ qside,
                                                uint64_t* __restrict__ ecodes, int R) {
  if (chunk <= ENC_CHUNK && *maxlen <= (uint32_t)ENC_MAXLEN) return;
  __shared__ uint32_t words[MAXW];  // chunk * MAXLEN / 32 words
  uint64_t* outliers = ecodes;
  __shared__ uint64_t scan[TPB];
  __shared__ uint32_t escan[TPB];
  const int t = threadIdx.x;
  const int per = chunk / TPB;
  for (uint64_t k = mg_bid.x; k < nch; k += mg_gdim.x) {
    const uint64_t beg = k * (uint64_t)chunk;
    const uint64_t w0 = word_off[k], nw = word_off[k + 1] - w0;
    for (uint64_t i = t; i < nw; i += TPB) words[i] = 0;
    const uint64_t mine = beg + (uint64_t)t * per;
    uint64_t bits = 0;
    uint32_t esc = 0;
    for (int j = 0; j < per; ++j) {
      const uint64_t i = mine + j;
      if (i < n) {
        const uint32_t s = sym[i] & mask;
        bits += len[s];
        esc += (s == 0);
      }
    }
    scan[t] = bits;
    escan[t] = esc;
    __syncthreads();
    for (int d = 1; d < TPB; d <<= 1) {
      uint64_t a = t >= d ? scan[t - d] : 0;
      uint32_t b = t >= d ? escan[t - d] : 0;
      __syncthreads();
      scan[t] += a;
      escan[t] += b;
      __syncthreads();
    }
    uint64_t pos = scan[t] - bits;
    uint64_t eo = (outliers ? esc_off[k] : 0) + (escan[t] - esc);
    for (int j = 0; j < per; ++j) {
      const uint64_t i = mine + j;
      if (i < n) {
        const uint32_t s = sym[i] & mask;
        const int L = len[s];
        put_code(words, pos, L, codes[s]);
        pos += L;
        if (s == 0 && outliers) outliers[eo++] = escape_code(qside[i], R);
      }
    }
    __syncthreads();
    for (uint64_t i = t; i < nw; i += TPB) payload[w0 + i] = words[i];
    __syncthreads();
  }
}

template <int MAXW>
__global__ void __launch_bounds__(TPB) k_encode_k(const uint16_t* __restrict__ sym, uint64_t n, int chunk,
                                                uint64_t nch, uint32_t mask, const uint8_t* __restrict__ len,
                                                const uint32_t* __restrict__ maxlen,
                                                const uint64_t* __restrict__ codes,
                                                const uint64_t* __restrict__ word_off,
                                                uint32_t* __restrict__ payload,
                                                const uint64_t* __restrict__ esc_off,
                                                const int64_t* __restrict__ qside,
                                                uint64_t* __restrict__ ecodes, int R) {
  k_encode<MAXW>(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, sym, n, chunk, nch, mask, len, maxlen, codes, word_off, payload, esc_off, qside, ecodes, R);
}


// ------------------------------------------------------------------ decode
// Canonical decoding tables: per length L, the first code, the count and the
// offset into the symbols sorted by (length, symbol); lim1[L] is the
// left-aligned (64-bit) end of the codes of length <= L, minus one, so the
// length of the next code is the smallest L with window <= lim1[L].  The code
// ranges of successive lengths are contiguous from 0, so only windows above
// lim1[maxlen] are invalid.
//
// Fast path (every length <= 32): for the j-th distinct length flen[j],
// flim[j] = the top 32 bits of its lim1 (whose low 32 bits are all ones, so
// comparing the top 32 bits of the window decides) and fdelta[j] = offset -
// first (mod 2^32); entry nfast (the number of distinct lengths) has length 0
// (an invalid code), limit 2^32 - 1, so no window passes it, and delta
// 2^32 - 1, so the symbol index it gives is out of range.
constexpr int FASTN = 33;
// Prefix table of the fast path: entry v describes the 32-bit windows that
// start with the LUT_BITS bits v.  Its low 6 bits are j, the index of the
// shortest length whose interval meets them; bit 6 set: the windows meet the
// intervals of lengths j and j + 1 (the window's comparison with flim[j]
// decides); bit 7 set: they meet three or more (comparisons from j on decide);
// neither: every such window has length j.
constexpr int LUT_BITS = 12;
constexpr uint32_t LUT_SPLIT = 1u << 22;

struct DecTables {
  uint64_t first[MAXLEN + 1];
  uint64_t lim1[MAXLEN + 1];
  uint32_t count[MAXLEN + 1];
  uint32_t offset[MAXLEN + 1];
  uint32_t minlen, maxlen, bad, used;
  uint32_t nfast, pad;
  uint32_t flen[FASTN], flim[FASTN], fdelta[FASTN];
  // entry v: bits 0-15 the symbol-table index of the first code in the
  // windows starting with v, bits 16-21 their length (0: no code starts with
  // these bits), when the windows meet one length; else bit 22 set and bits
  // 24-29 the first length index j whose limit decides (flim, fld).
  uint32_t lut[1 << LUT_BITS];
};

__global__ void __launch_bounds__(1024) k_decode_tables(const uint8_t* __restrict__ len, int dict, DecTables* tab,
                                                        uint16_t* __restrict__ sorted) {
  __shared__ uint8_t lens[MAXDICT];
  __shared__ uint16_t rank[MAXDICT];
  __shared__ uint32_t wcnt[16][MAXLEN + 1];
  __shared__ uint32_t cnt[MAXLEN + 1];
  __shared__ uint32_t offs[MAXLEN + 1];
  __shared__ uint32_t bad;
  __shared__ uint32_t sflim[FASTN], snfast;
  __shared__ uint32_t sflen[FASTN];
  __shared__ uint64_t sfirst[MAXLEN + 1];
  const int t = threadIdx.x, nt = blockDim.x;
  if (t == 0) bad = 0;
  __syncthreads();
  for (int s = t; s < dict; s += nt) {
    const uint8_t L = len[s];
    if (L > MAXLEN) atomicOr(&bad, 1u);
    lens[s] = L > MAXLEN ? 0 : L;
  }
  __syncthreads();
  canonical_ranks(lens, dict, rank, wcnt, cnt);
  if (t == 0) {
    uint64_t code = 0;
    uint32_t off = 0, minlen = 0, maxlen = 0, nd = 0;
    for (int b = 1; b <= MAXLEN; ++b) {
      code = (code + (b > 1 ? cnt[b - 1] : 0)) << 1;
      tab->first[b] = code;
      tab->count[b] = cnt[b];
      tab->offset[b] = off;
      offs[b] = off;
      off += cnt[b];
      if (cnt[b]) {
        if (!minlen) minlen = b;
        maxlen = b;
        ++nd;
      }
    }
    uint32_t flag = bad;
    // Kraft: the codes of the longest length must fit in that length
    if (maxlen && maxlen < 64 && tab->first[maxlen] + cnt[maxlen] > (1ull << maxlen)) flag = 1;
    // left-aligned limits, saturating at 2^64 - 1
    for (int b = 1; b <= MAXLEN; ++b) {
      const uint64_t e = tab->first[b] + tab->count[b];
      uint64_t lim;
      if (b == 64)
        lim = e ? e - 1 : 0;
      else if (e >= (1ull << b))
        lim = ~0ull;
      else
        lim = e ? (e << (64 - b)) - 1 : 0;
      tab->lim1[b] = lim;
    }
    tab->first[0] = 0;
    tab->count[0] = 0;
    tab->offset[0] = 0;
    tab->lim1[0] = 0;
    tab->minlen = minlen;
    tab->maxlen = maxlen;
    tab->bad = flag;
    tab->used = off;
    const bool fast = maxlen && maxlen <= 32;  // then nd <= 32 < FASTN
    int j = 0;
    if (fast)
      for (int b = minlen; b <= (int)maxlen; ++b) {
        if (!cnt[b]) continue;
        tab->flen[j] = b;
        tab->flim[j] = (uint32_t)(tab->lim1[b] >> 32);
        tab->fdelta[j] = offs[b] - (uint32_t)tab->first[b];
        ++j;
      }
    for (; j < FASTN; ++j) {  // the end entry (an invalid code) and unused ones
      tab->flen[j] = 0;
      tab->flim[j] = 0xffffffffu;
      tab->fdelta[j] = 0xffffffffu;
    }
    tab->nfast = fast ? nd : 0;
    for (int j = 0; j < FASTN; ++j) {
      sflim[j] = tab->flim[j];
      sflen[j] = tab->flen[j];
    }
    for (int b = 0; b <= MAXLEN; ++b) sfirst[b] = tab->first[b];
    snfast = fast ? nd : 0;
  }
  __syncthreads();
  for (int s = t; s < dict; s += nt) {
    const int L = lens[s];
    if (L) sorted[offs[L] + rank[s]] = (uint16_t)s;
  }
  // windows starting with prefix v run from v << (32 - LUT_BITS) to that plus
  // 2^(32 - LUT_BITS) - 1; the index of a window's length is the number of
  // limits below it, between its value at the two ends.  When both ends give
  // the same length L, every window's code is its top L bits, the first of
  // them v's bits (L <= LUT_BITS: v's top L bits; else v followed by zeros),
  // so the symbol-table index of the first is offset[L] + that - first[L].
  for (int v = t; v < (1 << LUT_BITS); v += nt) {
    uint32_t e = 0xffffu;  // no code: length 0, an index past every table
    if (snfast) {
      const uint32_t lo = (uint32_t)v << (32 - LUT_BITS), hi = lo | ((1u << (32 - LUT_BITS)) - 1u);
      uint32_t clo = 0, chi = 0;
      for (uint32_t j = 0; j < snfast; ++j) {
        clo += lo > sflim[j] ? 1u : 0u;
        chi += hi > sflim[j] ? 1u : 0u;
      }
      if (chi == clo) {
        const uint32_t L = sflen[clo];
        if (L) {
          const uint64_t c0 = L <= (uint32_t)LUT_BITS ? ((uint64_t)v >> (LUT_BITS - L)) : ((uint64_t)v << (L - LUT_BITS));
          e = (offs[L] + (uint32_t)(c0 - sfirst[L])) | (L << 16);
        }
      } else {
        e = LUT_SPLIT | (clo << 24) | 0xffffu;
      }
    }
    tab->lut[v] = e;
  }
}

constexpr uint32_t RING = 32;         // words per lane (a power of two)
constexpr uint32_t RING_STRIDE = 33;  // odd stride: lanes reading the same slot hit different banks

// Four payload words from min(at, words - 4) on (words >= 4): the load is
// unconditional so it can land in its destination registers while earlier
// words are decoded; the shift that puts word `at` first is applied when the
// group is used.
__device__ inline uint4 load_group(const uint32_t* __restrict__ payload, uint64_t at, uint64_t words,
                                   uint32_t* shift) {
  const uint64_t a = min(at, words - 4);
  *shift = (uint32_t)min(at - a, (uint64_t)4);
  uint4 v;
  __builtin_memcpy(&v, payload + a, 16);
  return v;
}

// Word i of the result is word i + sh of v; zeros past the payload's end.
__device__ inline uint4 shift_group(uint4 v, uint32_t sh) {
  uint4 r;
  r.x = sh == 0 ? v.x : sh == 1 ? v.y : sh == 2 ? v.z : sh == 3 ? v.w : 0u;
  r.y = sh == 0 ? v.y : sh == 1 ? v.z : sh == 2 ? v.w : 0u;
  r.z = sh == 0 ? v.z : sh == 1 ? v.w : 0u;
  r.w = sh == 0 ? v.w : 0u;
  return r;
}

// One thread per chunk.  status[0] is set to 1 on malformed input.  When
// esc_off is given, the stream position of the j-th escape symbol is written
// to epos[j] (chunk k owns entries [esc_off[k], esc_off[k+1]), which must lie
// inside the n_out entries of epos, and esc_off[nch] must equal n_out); the loop
// itself issues no loads besides the payload, so it never waits on them early.
// BT: lanes per block (the launch picks it so that every block is resident at once).
template <int BT>
__global__ void __launch_bounds__(BT) k_decode(const uint32_t* __restrict__ payload, uint64_t payload_words,
                                               const uint64_t* __restrict__ word_off,
                                               const uint32_t* __restrict__ chunk_bits, uint64_t n, int chunk,
                                               uint64_t nch, const DecTables* __restrict__ tab,
                                               const uint16_t* __restrict__ sorted_g, int dict,
                                               uint16_t* __restrict__ sym, const uint64_t* __restrict__ esc_off,
                                               uint64_t n_out, uint64_t* __restrict__ epos,
                                               uint32_t* __restrict__ status) {
  __shared__ uint64_t first[MAXLEN + 1], lim1[MAXLEN + 1];
  __shared__ uint32_t offs[MAXLEN + 1];
  __shared__ uint16_t sorted[MAXDICT];
  __shared__ uint32_t ring[BT * RING_STRIDE];
  __shared__ uint32_t lut_s[1 << LUT_BITS];  // the prefix table
  __shared__ uint2 fld_s[FASTN];                   // (fdelta, flen) of each distinct length
  __shared__ uint32_t flim_s[FASTN];
  const uint32_t used = min(tab->used, (uint32_t)dict);
  for (int b = threadIdx.x; b <= MAXLEN; b += blockDim.x) {
    first[b] = tab->first[b];
    lim1[b] = tab->lim1[b];
    offs[b] = tab->offset[b];
  }
  {
    for (int i = threadIdx.x; i < (1 << LUT_BITS); i += blockDim.x) lut_s[i] = tab->lut[i];
    if (threadIdx.x < FASTN) {
      fld_s[threadIdx.x] = make_uint2(tab->fdelta[threadIdx.x], tab->flen[threadIdx.x]);
      flim_s[threadIdx.x] = tab->flim[threadIdx.x];
    }
  }
  // symbols in code order: eight loads per lane in flight before the LDS stores
  for (uint32_t s0 = threadIdx.x; s0 < used; s0 += 8 * blockDim.x) {
    uint16_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t s = s0 + u * blockDim.x;
      v[u] = s < used ? sorted_g[s] : (uint16_t)0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t s = s0 + u * blockDim.x;
      if (s < used) sorted[s] = v[u];
    }
  }
  __syncthreads();
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nch) return;
  if (tab->bad || tab->maxlen == 0) {
    atomicOr(status, 1u);
    return;
  }
  const uint64_t w0 = word_off[k], w1 = word_off[k + 1];
  const uint64_t nbits = chunk_bits[k];
  if (w1 > payload_words || w1 < w0 || nbits > 32 * (w1 - w0)) {
    atomicOr(status, 1u);
    return;
  }
  const uint64_t beg = k * (uint64_t)chunk;
  const uint64_t cntk = min((uint64_t)chunk, n - beg);
  const bool escapes = esc_off != nullptr;
  uint64_t eo = escapes ? esc_off[k] : 0;
  const uint64_t eo_end = escapes ? esc_off[k + 1] : 0;
  // epos holds n_out entries: a chunk whose escape range (from the buffer's
  // own per-chunk counts) leaves it, or escape totals that disagree with
  // n_out, are malformed input and nothing is written
  if (escapes && (eo > eo_end || eo_end > n_out || (k + 1 == nch && eo_end != n_out))) {
    atomicOr(status, 1u);
    return;
  }
  uint64_t consumed = 0;
  if (tab->nfast && payload_words >= 4) {
    // The length of each code comes from the prefix table.  The chunk's words
    // pass through a per-lane ring in LDS: every 8 symbols (wave-uniform) the
    // 8 words fetched 8 symbols earlier are written to the ring and the next 8
    // are fetched if the ring has room, so no load is waited for soon after it
    // is issued.  The ring never holds fewer than 8 unread words at a refill
    // point, and at most 8 words are read between two refill points.
    uint32_t* myring = ring + threadIdx.x * RING_STRIDE;
    uint64_t fetch_at = w0;
    uint32_t wr = 0, rd = 0;
    for (int g = 0; g < 4; ++g) {
      uint32_t sh;
      const uint4 v = shift_group(load_group(payload, fetch_at, payload_words, &sh), sh);
      myring[wr] = v.x;
      myring[wr + 1] = v.y;
      myring[wr + 2] = v.z;
      myring[wr + 3] = v.w;
      wr += 4;
      fetch_at += 4;
    }
    uint32_t sha, shb;
    uint4 pa = load_group(payload, fetch_at, payload_words, &sha);
    uint4 pb = load_group(payload, fetch_at + 4, payload_words, &shb);
    fetch_at += 8;
    bool pend = true;
    uint32_t nextw = myring[0];
    uint64_t buf = 0;  // left-aligned bits
    int have = 0;
    // bits consumed and the largest symbol-table index met: malformed input
    // when either exceeds its bound, acted on every 8 symbols (both only grow)
    uint32_t cons = 0, imax = 0;
    const uint32_t nb32 = (uint32_t)nbits;
    // A trip's eight symbols go to eight registers; two symbols make a word
    // two steps after the second one's lookup was issued, and the trip's four
    // words are stored at the start of the next trip, so no step waits for
    // its own lookup.  Escapes and malformed input are checked at the stores.
    auto store8 = [&](uint64_t j0, uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3) -> bool {
      *reinterpret_cast<uint4*>(sym + beg + j0) = make_uint4(x0, x1, x2, x3);
      if (imax >= used || cons > nb32) {
        atomicOr(status, 1u);
        return false;
      }
      // escape symbols (value 0) among the eight, in order; the test flags
      // every zero (and at times a neighbour of one)
      const uint32_t m = 0x00010001u, h = 0x80008000u;
      if (escapes && (((x0 - m) & ~x0 & h) | ((x1 - m) & ~x1 & h) | ((x2 - m) & ~x2 & h) | ((x3 - m) & ~x3 & h))) {
        const uint32_t xs[4] = {x0, x1, x2, x3};
        for (int k = 0; k < 8; ++k) {
          const uint16_t x = (uint16_t)(xs[k >> 1] >> (16 * (k & 1)));
          if (x) continue;
          if (eo >= eo_end) {
            atomicOr(status, 1u);
            return false;
          }
          epos[eo++] = beg + j0 + k;
        }
      }
      return true;
    };
    // the words fetched one refill point earlier go to the ring; the next
    // eight are fetched when the ring has room (every eighth symbol, before
    // symbol i with i % 8 == 4)
    auto refill = [&]() {
      if (pend) {
          const uint4 va = shift_group(pa, sha), vb = shift_group(pb, shb);
          myring[wr & (RING - 1)] = va.x;
          myring[(wr + 1) & (RING - 1)] = va.y;
          myring[(wr + 2) & (RING - 1)] = va.z;
          myring[(wr + 3) & (RING - 1)] = va.w;
          myring[(wr + 4) & (RING - 1)] = vb.x;
          myring[(wr + 5) & (RING - 1)] = vb.y;
          myring[(wr + 6) & (RING - 1)] = vb.z;
          myring[(wr + 7) & (RING - 1)] = vb.w;
          wr += 8;
          pend = false;
        }
        if (wr - rd <= RING - 8) {
          pa = load_group(payload, fetch_at, payload_words, &sha);
          pb = load_group(payload, fetch_at + 4, payload_words, &shb);
          fetch_at += 8;
          pend = true;
        }
          };
    // one symbol: length, bit buffer, lookup into s
    auto step = [&](uint32_t& s) {
      // top up the buffer to at least 32 bits (branch-free; the ring slot is
      // re-read when no word was taken)
      {
        const bool need = have < 32;
        const uint32_t sh = need ? (uint32_t)(32 - have) : 0u;
        buf |= need ? ((uint64_t)nextw << sh) : 0ull;
        have += need ? 32 : 0;
        rd += need ? 1u : 0u;
        nextw = myring[rd & (RING - 1)];
      }
      const uint32_t top = (uint32_t)(buf >> 32);
      // length and symbol index from the prefix table: the window's first
      // index plus the code's bits past the prefix (none when L <= LUT_BITS:
      // the shift is then 32 or more); comparisons with the limits only for
      // windows that meet two or more lengths (rare)
      const uint32_t e = lut_s[top >> (32 - LUT_BITS)];
      uint32_t L = (e >> 16) & 63u;
      uint32_t idx = (e & 0xffffu) + (uint32_t)((uint64_t)(top << LUT_BITS) >> (32 + LUT_BITS - L));
      if (e & LUT_SPLIT) {
        uint32_t jj = e >> 24;
        while (top > flim_s[jj]) ++jj;  // flim_s[nfast] = 2^32 - 1 ends it
        const uint2 ld = fld_s[jj];
        L = ld.y;
        // L = 0 (no code of the table starts with these bits) leaves idx =
        // fdelta of the end entry, 2^32 - 1
        idx = ld.x + (uint32_t)((uint64_t)top >> (32 - L));
      }
      buf <<= L;
      have -= (int)L;
      cons += L;
      imax = max(imax, idx);  // checked with the bit count every 8 symbols
      s = sorted[min(idx, used - 1u)];
    };
    uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0, a6 = 0, a7 = 0;
    uint32_t w0 = 0, w1 = 0, w2 = 0;  // the trip's first three words
    uint64_t i0 = 0;
    for (; i0 + 8 <= cntk; i0 += 8) {
      step(a0);
      if (i0 > 0 && !store8(i0 - 8, w0, w1, w2, a6 | (a7 << 16))) return;
      step(a1);
      step(a2);
      w0 = a0 | (a1 << 16);
      step(a3);
      refill();
      step(a4);
      w1 = a2 | (a3 << 16);
      step(a5);
      step(a6);
      w2 = a4 | (a5 << 16);
      step(a7);
    }
    if (i0 > 0 && !store8(i0 - 8, w0, w1, w2, a6 | (a7 << 16))) return;
    // fewer than eight left (the stream's last chunk): one symbol at a time
    for (uint64_t i = i0; i < cntk; ++i) {
      if ((i & 7) == 4) refill();
      uint32_t t;
      step(t);
      sym[beg + i] = (uint16_t)t;
      if (t == 0 && escapes) {
        if (eo >= eo_end) {
          atomicOr(status, 1u);
          return;
        }
        epos[eo++] = beg + i;
      }
    }
    if (imax >= used || cons > nb32) {
      atomicOr(status, 1u);
      return;
    }
    consumed = cons;
  } else {
    const int minlen = (int)tab->minlen, maxlen = (int)tab->maxlen;
    const uint32_t* src = payload + w0;
    const uint64_t nw = w1 - w0;
    uint64_t buf = 0;  // left-aligned bits
    int have = 0;
    uint64_t next_word = 0;
    for (uint64_t i = 0; i < cntk; ++i) {
      int s;
      if (maxlen <= 32) {
        while (have <= 32) {
          const uint64_t w = next_word < nw ? (uint64_t)src[next_word] : 0ull;
          ++next_word;
          buf |= w << (32 - have);
          have += 32;
        }
        // code length: the smallest L in [minlen, maxlen] with buf <= lim1[L]
        int lo = minlen, hi = maxlen;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (buf <= lim1[mid])
            hi = mid;
          else
            lo = mid + 1;
        }
        const int L = lo;
        const uint64_t v = buf >> (64 - L);
        if (buf > lim1[L] || v < first[L] || offs[L] + (v - first[L]) >= used) {
          atomicOr(status, 1u);
          return;
        }
        s = sorted[offs[L] + (uint32_t)(v - first[L])];
        buf <<= L;
        have -= L;
        consumed += L;
      } else {
        // codes longer than 32 bits exist: decode one bit at a time
        uint64_t code = 0;
        s = -1;
        for (int L = 1; L <= maxlen; ++L) {
          if (have == 0) {
            buf = (next_word < nw ? (uint64_t)src[next_word] : 0ull) << 32;
            ++next_word;
            have = 32;
          }
          code = (code << 1) | (buf >> 63);
          buf <<= 1;
          --have;
          ++consumed;
          if (L >= minlen && code >= first[L] && code - first[L] < tab->count[L] &&
              offs[L] + (code - first[L]) < used) {
            s = sorted[offs[L] + (uint32_t)(code - first[L])];
            break;
          }
        }
        if (s < 0) {
          atomicOr(status, 1u);
          return;
        }
      }
      if (consumed > nbits) {
        atomicOr(status, 1u);
        return;
      }
      sym[beg + i] = (uint16_t)s;
      if (s == 0 && escapes) {
        if (eo >= eo_end) {
          atomicOr(status, 1u);
          return;
        }
        epos[eo++] = beg + i;
      }
    }
  }
  if (consumed != nbits || eo != eo_end) atomicOr(status, 1u);
}

// Lanes per decoding block.  A lane decodes a whole chunk, so every chunk of
// a stream takes about as long; the kernel ends when the CU with the most
// wavefronts is done.  Of 192, 256 and 320 lanes (three, two and two blocks
// per CU by their LDS), the one whose blocks are all resident at once with
// the fewest wavefronts on the busiest CU is used.
struct DecodeShape {
  int bt;
};
DecodeShape decode_shape(uint64_t nch) {
  static int ncu = 0, per[3] = {0, 0, 0};
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess)
      ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per[0], k_decode<192>, 192, 0) != hipSuccess) per[0] = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per[1], k_decode<256>, 256, 0) != hipSuccess) per[1] = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per[2], k_decode<320>, 320, 0) != hipSuccess) per[2] = 0;
    (void)hipGetLastError();
  });
  const int bts[3] = {192, 256, 320};
  int best = 1;
  uint64_t best_cost = ~0ull;
  for (int c = 0; c < 3; ++c) {
    if (ncu <= 0 || per[c] <= 0) continue;
    const uint64_t blocks = (nch + bts[c] - 1) / bts[c];
    const uint64_t slots = (uint64_t)per[c] * (uint64_t)ncu;
    const uint64_t rounds = (blocks + slots - 1) / slots;
    const uint64_t on_busiest = rounds == 1 ? (blocks + ncu - 1) / ncu : rounds * (uint64_t)per[c];
    const uint64_t cost = on_busiest * (uint64_t)(bts[c] / 64);
    if (cost < best_cost) {
      best_cost = cost;
      best = c;
    }
  }
  return DecodeShape{bts[best]};
}

inline unsigned blocks_for(uint64_t nch, unsigned cap) {
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(nch, cap));
}

}  // namespace

void launch_histogram_chunks(const uint16_t* sym, uint64_t n, int dict, int chunk, uint64_t k0, uint64_t k1,
                             uint64_t* hist, uint32_t* chunk_esc, uint32_t* status, hipStream_t st) {
  const uint64_t nch = (n + chunk - 1) / chunk;
  k1 = std::min(k1, nch);
  if (k0 >= k1) return;
  KernelTimer kt("histogram", st);
  MG_LAUNCH((&k_histogram), (k_histogram_k), (WAVE_T), (0), (dim3(blocks_for((k1 - k0 + WAVES - 1) / WAVES, 256))), st, sym, n, dict, chunk, k0, k1, (unsigned long long*)hist, chunk_esc, status);
  MG_HIP(hipGetLastError());
}

void launch_histogram(const uint16_t* sym, uint64_t n, int dict, int chunk, uint64_t* hist,
                      uint32_t* chunk_esc, uint32_t* status, hipStream_t st) {
  launch_fill_u64(hist, (uint64_t)dict, 0, st);
  launch_histogram_chunks(sym, n, dict, chunk, 0, (n + chunk - 1) / chunk, hist, chunk_esc, status, st);
}

void encode_tables(void* scratch, int dict, uint32_t** enc, uint32_t** maxlen) {
  Carver cv(scratch);
  *enc = cv.take<uint32_t>((uint64_t)dict);
  *maxlen = cv.take<uint32_t>(4);
}

void launch_codebook(const uint64_t* hist, int dict, uint8_t* len, uint64_t* codes, void* enc_scratch,
                     hipStream_t st) {
  uint32_t *enc = nullptr, *maxlen = nullptr;
  if (enc_scratch) encode_tables(enc_scratch, dict, &enc, &maxlen);
  KernelTimer kt("codebook", st);
  MG_LAUNCH((&k_codebook), (k_codebook_k), (CB_T), (0), (dim3(1)), st, hist, dict, len, codes, enc, maxlen);
  MG_HIP(hipGetLastError());
}


void launch_chunk_bits(const uint16_t* sym, uint64_t n, int dict, int chunk, const uint8_t* len,
                       uint32_t* chunk_bits, hipStream_t st) {
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (nch == 0) return;
  KernelTimer kt("chunk_bits", st);
  MG_LAUNCH((&k_chunk_bits), (k_chunk_bits_k), (WAVE_T), (0), (dim3(blocks_for((nch + WAVES - 1) / WAVES, 256))), st, sym, n, chunk, nch, (uint32_t)(dict - 1), len, chunk_bits);
  MG_HIP(hipGetLastError());
}

void launch_scan_words(const uint32_t* chunk_bits, uint64_t nch, uint64_t* word_off, hipStream_t st) {
  KernelTimer kt("scan", st);
  launch_scan<true>(chunk_bits, nch, word_off, st);
}

void launch_scan_u32(const uint32_t* v, uint64_t n, uint64_t* off, hipStream_t st) {
  KernelTimer kt("scan", st);
  launch_scan<false>(v, n, off, st);
}

void launch_scan_pair(const uint32_t* chunk_bits, const uint32_t* esc, uint64_t nch, uint64_t* word_off,
                      uint64_t* esc_off, hipStream_t st) {
  KernelTimer kt("scan", st);
  ScanPair p{{chunk_bits, esc}, {word_off, esc_off}};
  const uint64_t nt = (nch + SCAN_TILE - 1) / SCAN_TILE;
  if (nt) MG_LAUNCH((&k_scan_tiles2), (k_scan_tiles2_k), (SCAN_T), (0), (dim3((unsigned)nt, 2)), st, p, nch);
  MG_LAUNCH((&k_scan_top2), (k_scan_top2_k), (1024), (0), (dim3(1, 2)), st, p, nch);
  if (nt) MG_LAUNCH((&k_scan_apply2), (k_scan_apply2_k), (SCAN_T), (0), (dim3((unsigned)nt, 2)), st, p, nch);
  MG_HIP(hipGetLastError());
}

uint64_t encode_scratch_bytes(int dict) { return carve_size<uint32_t>((uint64_t)dict) + carve_size<uint32_t>(4); }

void launch_encode(const uint16_t* sym, uint64_t n, int dict, int chunk, const uint8_t* len,
                   const uint64_t* codes, const uint64_t* word_off, uint32_t* payload,
                   const uint64_t* esc_off, const int64_t* qside, uint64_t* ecodes, void* scratch,
                   bool packed, hipStream_t st) {
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (nch == 0) return;
  uint32_t *enc = nullptr, *maxlen = nullptr;
  encode_tables(scratch, dict, &enc, &maxlen);
  KernelTimer kt("encode", st);
  // the codebook kernel may have written the packed table already
  if (!packed) hipLaunchKernelGGL(k_pack_codes, dim3(1), dim3(1024), 0, st, len, codes, dict, enc, maxlen);
  const uint32_t mask = (uint32_t)(dict - 1);
  if (chunk <= ENC_CHUNK)
    MG_LAUNCH((&k_encode_wave), (k_encode_wave_k), (ENC_T), (0), (dim3(blocks_for((nch + ENC_T / 64 - 1) / (ENC_T / 64), 512))), st, sym, n, chunk, nch, mask, enc, maxlen, len, codes, word_off, payload, esc_off, qside, ecodes, dict / 2);
  // The generic kernel does the work for chunks above ENC_CHUNK; for smaller
  // chunks only when some code is longer than ENC_MAXLEN (rare), and its
  // blocks return at once otherwise, so that grid is kept small.
  const unsigned gen_blocks = blocks_for(nch, chunk <= ENC_CHUNK ? 256 : 4096);
  if (chunk <= 4096)
    MG_LAUNCH((&k_encode<4096 * MAXLEN / 32>), (k_encode_k<4096 * MAXLEN / 32>), (TPB), (0), (dim3(gen_blocks)), st, sym, n, chunk, nch, mask, len, maxlen, codes, word_off, payload, esc_off, qside, ecodes, dict / 2);
  else
    MG_LAUNCH((&k_encode<8192 * MAXLEN / 32>), (k_encode_k<8192 * MAXLEN / 32>), (TPB), (0), (dim3(gen_blocks)), st, sym, n, chunk, nch, mask, len, maxlen, codes, word_off, payload, esc_off, qside, ecodes, dict / 2);
  MG_HIP(hipGetLastError());
}

uint64_t decode_table_bytes(int dict) {
  return carve_size<DecTables>(1) + carve_size<uint16_t>((uint64_t)dict) + carve_size<uint32_t>(4);
}

// Full decode entry used by the API: builds the tables, decodes, then places
// the outliers (when given; epos has room for n_out positions).
void launch_decode_full(const uint32_t* payload, uint64_t payload_words, const uint64_t* word_off,
                        const uint32_t* chunk_bits, uint64_t n, int dict, int chunk,
                        const uint8_t* len, uint16_t* sym, const uint64_t* esc_off, uint64_t n_out,
                        uint64_t* epos, void* table_scratch, uint32_t* d_status, hipStream_t st) {
  Carver cv(table_scratch);
  DecTables* tab = cv.take<DecTables>(1);
  uint16_t* sorted = cv.take<uint16_t>((uint64_t)dict);
  hipLaunchKernelGGL(k_decode_tables, dim3(1), dim3(1024), 0, st, len, dict, tab, sorted);
  const uint64_t nch = (n + chunk - 1) / chunk;
  const bool escapes = esc_off && epos;
  if (nch) {
    KernelTimer kt("decode", st);
    const DecodeShape sh = decode_shape(nch);
    auto go = [&](auto kernel, int bt) {
      hipLaunchKernelGGL(kernel, dim3((unsigned)((nch + bt - 1) / bt)), dim3(bt), 0, st, payload, payload_words,
                         word_off, chunk_bits, n, chunk, nch, tab, sorted, dict, sym, escapes ? esc_off : nullptr,
                         n_out, escapes ? epos : nullptr, d_status);
    };
    if (sh.bt == 192)
      go(k_decode<192>, 192);
    else if (sh.bt == 256)
      go(k_decode<256>, 256);
    else
      go(k_decode<320>, 320);
  }
  MG_HIP(hipGetLastError());
}

}  // namespace mg
