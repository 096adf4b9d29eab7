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

#include "internal.hpp"

namespace mg {

namespace {

constexpr int TPB = 256;
constexpr int MAXLEN = 64;
constexpr int MAXDICT = 8192;  // largest dictionary; all LDS below is static

// ------------------------------------------------------------------ histogram
__global__ void __launch_bounds__(TPB) k_histogram(const uint16_t* __restrict__ sym, uint64_t n, int dict,
                                                   int chunk, uint64_t nch, unsigned long long* __restrict__ hist,
                                                   uint32_t* __restrict__ chunk_esc, uint32_t* __restrict__ status) {
  __shared__ uint32_t sh[MAXDICT];
  __shared__ uint32_t esc;
  for (int b = threadIdx.x; b < dict; b += TPB) sh[b] = 0;
  __syncthreads();
  for (uint64_t k = blockIdx.x; k < nch; k += gridDim.x) {
    if (threadIdx.x == 0) esc = 0;
    __syncthreads();
    const uint64_t beg = k * (uint64_t)chunk;
    const uint64_t end = min(beg + (uint64_t)chunk, n);
    uint32_t e = 0;
    for (uint64_t i = beg + threadIdx.x; i < end; i += TPB) {
      const uint32_t s = sym[i];
      if (s < (uint32_t)dict)
        atomicAdd(&sh[s], 1u);
      else
        atomicOr(status, 1u);  // symbol outside the dictionary
      e += (s == 0);
    }
    if (e) atomicAdd(&esc, e);
    __syncthreads();
    if (threadIdx.x == 0) chunk_esc[k] = esc;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < dict; b += TPB)
    if (sh[b]) atomicAdd(&hist[b], (unsigned long long)sh[b]);
}

// ------------------------------------------------------------------ codebook
// One workgroup; everything stays in LDS.  keys: (count << 16 | symbol),
// empty bins sort last.  The two-queue merge runs on one lane with the queue
// heads held in registers; internal-node depths come from pointer jumping,
// leaf lengths from the number of leaves per depth (deepest for the smallest
// weights), canonical codes from a second sort by (length, symbol).
__global__ void __launch_bounds__(1024) k_codebook(const uint64_t* __restrict__ hist, int dict,
                                                   uint8_t* __restrict__ len_out, uint64_t* __restrict__ codes) {
  __shared__ uint64_t keys[MAXDICT];
  __shared__ uint16_t syms[MAXDICT];
  __shared__ uint16_t par[MAXDICT];
  __shared__ uint8_t dep[MAXDICT];
  __shared__ uint8_t lens[MAXDICT];
  __shared__ int nleaf;
  __shared__ uint32_t icount[MAXLEN + 2];
  __shared__ uint32_t lstart[MAXLEN + 2];
  __shared__ uint64_t first[MAXLEN + 1];
  __shared__ uint32_t lcount[MAXLEN + 1], loff[MAXLEN + 1];
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  if (t == 0) nleaf = 0;
  for (int i = t; i <= MAXLEN + 1; i += nt) icount[i] = 0;
  __syncthreads();
  for (int s = t; s < dict; s += nt) {
    const uint64_t c = hist[s];
    keys[s] = c ? ((c << 16) | (uint64_t)s) : ~0ull;
    lens[s] = 0;
    if (c) atomicAdd(&nleaf, 1);
  }
  __syncthreads();
  auto bitonic = [&]() {
    for (int k = 2; k <= dict; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = t; i < dict; i += nt) {
          const int p = i ^ j;
          if (p > i) {
            const uint64_t a = keys[i], b = keys[p];
            if ((a > b) == ((i & k) == 0)) {
              keys[i] = b;
              keys[p] = a;
            }
          }
        }
        __syncthreads();
      }
    }
  };
  bitonic();
  const int n = nleaf;
  for (int i = t; i < n; i += nt) {
    syms[i] = (uint16_t)(keys[i] & 0xffff);
    keys[i] >>= 16;
  }
  __syncthreads();
  if (n == 1) {
    if (t == 0) lens[syms[0]] = 1;
  } else if (n > 1) {
    // merge (in place: a consumed internal node's slot takes its parent's index)
    if (t == 0) {
      uint64_t* A = keys;
      const uint64_t INF = ~0ull;
      // register windows over both queues: lq[i] = weight of leaf (leaf + i),
      // iq[i] = weight of internal node (root + i) (INF until it exists); the
      // loads that refill a window are issued several picks before they are used
      uint64_t lq0 = A[0], lq1 = n > 1 ? A[1] : INF, lq2 = n > 2 ? A[2] : INF, lq3 = n > 3 ? A[3] : INF;
      uint64_t iq0 = INF, iq1 = INF, iq2 = INF, iq3 = INF;
      int leaf = 0, root = 0;
      for (int next = 0; next < n - 1; ++next) {
        uint64_t w = 0;
#pragma unroll
        for (int pick = 0; pick < 2; ++pick) {
          // the internal queue holds the nodes [root, next); the leaf queue wins ties
          if (leaf < n && (root >= next || lq0 <= iq0)) {
            w += lq0;
            ++leaf;
            lq0 = lq1;
            lq1 = lq2;
            lq2 = lq3;
            lq3 = leaf + 3 < n ? A[leaf + 3] : INF;
          } else {
            w += iq0;
            A[root] = (uint64_t)next;
            ++root;
            iq0 = iq1;
            iq1 = iq2;
            iq2 = iq3;
            iq3 = root + 3 < next ? A[root + 3] : INF;
          }
        }
        A[next] = w;
        // the new node enters the internal window if it is among its first four
        const int pos = next - root;
        if (pos == 0)
          iq0 = w;
        else if (pos == 1)
          iq1 = w;
        else if (pos == 2)
          iq2 = w;
        else if (pos == 3)
          iq3 = w;
      }
    }
    __syncthreads();
    // internal node k < n-1: parent index in keys[k] (the root n-2 holds its weight)
    const int ni = n - 1;
    for (int k = t; k < ni; k += nt) {
      par[k] = (uint16_t)(k == ni - 1 ? k : (int)keys[k]);
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
      int d = MAXLEN;
      while (d > 1 && lstart[d - 1] <= (uint32_t)i) --d;
      lens[syms[i]] = (uint8_t)d;
    }
  }
  __syncthreads();
  // canonical codes: sort by (length, symbol), then consecutive codes per length
  for (int i = t; i <= MAXLEN; i += nt) lcount[i] = 0;
  __syncthreads();
  for (int s = t; s < dict; s += nt) {
    keys[s] = lens[s] ? (((uint64_t)lens[s] << 16) | (uint64_t)s) : ~0ull;
    if (lens[s]) atomicAdd(&lcount[lens[s]], 1u);
  }
  __syncthreads();
  bitonic();
  if (t == 0) {
    uint64_t code = 0;
    uint32_t off = 0;
    for (int b = 1; b <= MAXLEN; ++b) {
      code = (code + (b > 1 ? lcount[b - 1] : 0)) << 1;
      first[b] = code;
      loff[b] = off;
      off += lcount[b];
    }
  }
  __syncthreads();
  for (int i = t; i < dict; i += nt) {
    const uint64_t k = keys[i];
    if (k == ~0ull) continue;
    const int L = (int)(k >> 16), s = (int)(k & 0xffff);
    codes[s] = first[L] + (uint64_t)(i - (int)loff[L]);
  }
  for (int s = t; s < dict; s += nt) {
    len_out[s] = lens[s];
    if (!lens[s]) codes[s] = 0;
  }
}

// ------------------------------------------------------------------ chunk sizes
__global__ void __launch_bounds__(TPB) k_chunk_bits(const uint16_t* __restrict__ sym, uint64_t n, int chunk,
                                                    uint64_t nch, uint32_t mask, const uint8_t* __restrict__ len,
                                                    uint32_t* __restrict__ chunk_bits) {
  __shared__ uint32_t acc;
  for (uint64_t k = blockIdx.x; k < nch; k += gridDim.x) {
    if (threadIdx.x == 0) acc = 0;
    __syncthreads();
    const uint64_t beg = k * (uint64_t)chunk;
    const uint64_t end = min(beg + (uint64_t)chunk, n);
    uint32_t b = 0;
    for (uint64_t i = beg + threadIdx.x; i < end; i += TPB) b += len[sym[i] & mask];
    atomicAdd(&acc, b);
    __syncthreads();
    if (threadIdx.x == 0) chunk_bits[k] = acc;
    __syncthreads();
  }
}

// ------------------------------------------------------------------ scans
// Exclusive scan over n values (words of chunk bit counts when WORDS), one
// workgroup; off has n+1 entries, off[n] the total.
template <bool WORDS>
__global__ void __launch_bounds__(1024) k_scan(const uint32_t* __restrict__ v, uint64_t n,
                                               uint64_t* __restrict__ off) {
  __shared__ uint64_t part[1024];
  const int t = threadIdx.x;
  const uint64_t per = (n + 1023) / 1024;
  const uint64_t beg = min((uint64_t)t * per, n), end = min(beg + per, n);
  uint64_t s = 0;
  for (uint64_t i = beg; i < end; ++i) s += WORDS ? (uint64_t)((v[i] + 31u) >> 5) : (uint64_t)v[i];
  part[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    uint64_t add = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  uint64_t run = part[t] - s;
  for (uint64_t i = beg; i < end; ++i) {
    off[i] = run;
    run += WORDS ? (uint64_t)((v[i] + 31u) >> 5) : (uint64_t)v[i];
  }
  if (t == 1023) off[n] = part[1023];
}

// ------------------------------------------------------------------ encode
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
template <int MAXW>
__global__ void __launch_bounds__(TPB) k_encode(const uint16_t* __restrict__ sym, uint64_t n, int chunk,
                                                uint64_t nch, uint32_t mask, const uint8_t* __restrict__ len,
                                                const uint64_t* __restrict__ codes,
                                                const uint64_t* __restrict__ word_off,
                                                uint32_t* __restrict__ payload,
                                                const uint64_t* __restrict__ esc_off,
                                                const int64_t* __restrict__ qside, char* obase,
                                                const uint64_t* __restrict__ ooff) {
  __shared__ uint32_t words[MAXW];
  int64_t* outliers = obase ? reinterpret_cast<int64_t*>(obase + *ooff) : nullptr;  // chunk * MAXLEN / 32 words
  __shared__ uint64_t scan[TPB];
  __shared__ uint32_t escan[TPB];
  const int t = threadIdx.x;
  const int per = chunk / TPB;
  for (uint64_t k = blockIdx.x; k < nch; k += gridDim.x) {
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
        if (s == 0 && outliers) outliers[eo++] = qside[i];
      }
    }
    __syncthreads();
    for (uint64_t i = t; i < nw; i += TPB) payload[w0 + i] = words[i];
    __syncthreads();
  }
}

// ------------------------------------------------------------------ decode
// Canonical decoding tables: per length L, the first code, the count and the
// offset into the symbols sorted by (length, symbol); lim1[L] is the
// left-aligned (64-bit) end of the codes of length <= L, minus one, so the
// length of the next code is the smallest L with window <= lim1[L].
struct DecTables {
  uint64_t first[MAXLEN + 1];
  uint64_t lim1[MAXLEN + 1];
  uint32_t count[MAXLEN + 1];
  uint32_t offset[MAXLEN + 1];
  uint32_t minlen, maxlen, bad, pad;
};

__global__ void __launch_bounds__(1024) k_decode_tables(const uint8_t* __restrict__ len, int dict, DecTables* tab,
                                                        uint16_t* __restrict__ sorted) {
  __shared__ uint8_t lens[MAXDICT];
  __shared__ uint32_t cnt[MAXLEN + 1];
  __shared__ uint32_t fill[MAXLEN + 1];
  __shared__ uint32_t bad;
  const int t = threadIdx.x, nt = blockDim.x;
  if (t == 0) bad = 0;
  for (int b = t; b <= MAXLEN; b += nt) cnt[b] = 0;
  __syncthreads();
  for (int s = t; s < dict; s += nt) {
    const uint8_t L = len[s];
    lens[s] = L;
    if (L > MAXLEN)
      atomicOr(&bad, 1u);
    else if (L)
      atomicAdd(&cnt[L], 1u);
  }
  __syncthreads();
  if (t == 0) {
    uint64_t code = 0;
    uint32_t off = 0, minlen = 0, maxlen = 0;
    for (int b = 1; b <= MAXLEN; ++b) {
      code = (code + (b > 1 ? cnt[b - 1] : 0)) << 1;
      tab->first[b] = code;
      tab->count[b] = cnt[b];
      tab->offset[b] = off;
      fill[b] = off;
      off += cnt[b];
      if (cnt[b]) {
        if (!minlen) minlen = b;
        maxlen = b;
      }
    }
    // Kraft: the codes of the longest length must fit in that length
    if (maxlen && maxlen < 64 && tab->first[maxlen] + cnt[maxlen] > (1ull << maxlen)) bad = 1;
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
    tab->bad = bad;
    for (int s = 0; s < dict; ++s) {
      const int L = lens[s];
      if (L && L <= MAXLEN) sorted[fill[L]++] = (uint16_t)s;
    }
  }
}

// One thread per chunk.  status[0] is set to 1 on malformed input.
__global__ void __launch_bounds__(256) k_decode(const uint32_t* __restrict__ payload, uint64_t payload_words,
                                               const uint64_t* __restrict__ word_off,
                                               const uint32_t* __restrict__ chunk_bits, uint64_t n, int chunk,
                                               uint64_t nch, const DecTables* __restrict__ tab,
                                               const uint16_t* __restrict__ sorted_g, int dict,
                                               uint16_t* __restrict__ sym, const uint64_t* __restrict__ esc_off,
                                               uint64_t n_out, const int64_t* __restrict__ outliers,
                                               int64_t* __restrict__ qside, uint32_t* __restrict__ status) {
  __shared__ uint64_t first[MAXLEN + 1], lim1[MAXLEN + 1];
  __shared__ uint32_t offs[MAXLEN + 1];
  __shared__ uint16_t sorted[MAXDICT];
  for (int b = threadIdx.x; b <= MAXLEN; b += blockDim.x) {
    first[b] = tab->first[b];
    lim1[b] = tab->lim1[b];
    offs[b] = tab->offset[b];
  }
  {
    const int used = tab->maxlen ? (int)(tab->offset[tab->maxlen] + tab->count[tab->maxlen]) : 0;
    for (int s = threadIdx.x; s < used && s < dict; s += blockDim.x) sorted[s] = sorted_g[s];
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
  const int minlen = (int)tab->minlen, maxlen = (int)tab->maxlen;
  const uint32_t* src = payload + w0;
  const uint64_t nw = w1 - w0;
  uint64_t buf = 0;  // left-aligned bits
  int have = 0;
  uint64_t next_word = 0, consumed = 0;
  uint64_t eo = esc_off ? esc_off[k] : 0;  // escapes are resolved only when outliers are given
  uint64_t pack = 0;
  const bool fast = maxlen <= 32;
  for (uint64_t i = 0; i < cntk; ++i) {
    // keep at least 33 valid bits at the top of the buffer
    while (have <= 32) {
      const uint64_t w = next_word < nw ? (uint64_t)src[next_word] : 0ull;
      ++next_word;
      buf |= w << (32 - have);
      have += 32;
    }
    int s;
    if (fast) {
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
      if (buf > lim1[L] || v < first[L]) {
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
        if (L >= minlen && code >= first[L] && code - first[L] < tab->count[L]) {
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
    pack |= (uint64_t)(uint16_t)s << (16 * (i & 3));
    if ((i & 3) == 3) {
      *reinterpret_cast<uint64_t*>(sym + beg + i - 3) = pack;
      pack = 0;
    }
    if (s == 0 && qside) {
      if (eo >= n_out) {
        atomicOr(status, 1u);
        return;
      }
      qside[beg + i] = outliers[eo++];
    }
  }
  for (uint64_t i = cntk & ~3ull; i < cntk; ++i) sym[beg + i] = (uint16_t)(pack >> (16 * (i & 3)));
  if (consumed != nbits) atomicOr(status, 1u);
}

inline unsigned blocks_for(uint64_t nch, unsigned cap) {
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(nch, cap));
}

}  // namespace

void launch_histogram(const uint16_t* sym, uint64_t n, int dict, int chunk, uint64_t* hist,
                      uint32_t* chunk_esc, uint32_t* status, hipStream_t st) {
  const uint64_t nch = (n + chunk - 1) / chunk;
  MG_HIP(hipMemsetAsync(hist, 0, sizeof(uint64_t) * dict, st));
  if (nch == 0) return;
  KernelTimer kt("histogram", st);
  hipLaunchKernelGGL(k_histogram, dim3(blocks_for(nch, 2048)), dim3(TPB), 0, st, sym, n,
                     dict, chunk, nch, (unsigned long long*)hist, chunk_esc, status);
  MG_HIP(hipGetLastError());
}

void launch_codebook(const uint64_t* hist, int dict, uint8_t* len, uint64_t* codes, hipStream_t st) {
  KernelTimer kt("codebook", st);
  hipLaunchKernelGGL(k_codebook, dim3(1), dim3(1024), 0, st, hist, dict, len, codes);
  MG_HIP(hipGetLastError());
}

void launch_chunk_bits(const uint16_t* sym, uint64_t n, int dict, int chunk, const uint8_t* len,
                       uint32_t* chunk_bits, hipStream_t st) {
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (nch == 0) return;
  KernelTimer kt("chunk_bits", st);
  hipLaunchKernelGGL(k_chunk_bits, dim3(blocks_for(nch, 8192)), dim3(TPB), 0, st, sym, n, chunk, nch,
                     (uint32_t)(dict - 1), len, chunk_bits);
  MG_HIP(hipGetLastError());
}

void launch_scan_words(const uint32_t* chunk_bits, uint64_t nch, uint64_t* word_off, hipStream_t st) {
  hipLaunchKernelGGL(k_scan<true>, dim3(1), dim3(1024), 0, st, chunk_bits, nch, word_off);
  MG_HIP(hipGetLastError());
}

void launch_scan_u32(const uint32_t* v, uint64_t n, uint64_t* off, hipStream_t st) {
  hipLaunchKernelGGL(k_scan<false>, dim3(1), dim3(1024), 0, st, v, n, off);
  MG_HIP(hipGetLastError());
}

void launch_encode(const uint16_t* sym, uint64_t n, int dict, int chunk, const uint8_t* len,
                   const uint64_t* codes, const uint64_t* word_off, uint32_t* payload,
                   const uint64_t* esc_off, const int64_t* qside, char* obase,
                   const uint64_t* ooff, hipStream_t st) {
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (nch == 0) return;
  KernelTimer kt("encode", st);
  if (chunk <= 4096)
    hipLaunchKernelGGL(k_encode<4096 * MAXLEN / 32>, dim3(blocks_for(nch, 4096)), dim3(TPB), 0, st, sym, n, chunk,
                       nch, (uint32_t)(dict - 1), len, codes, word_off, payload, esc_off, qside, obase, ooff);
  else
    hipLaunchKernelGGL(k_encode<8192 * MAXLEN / 32>, dim3(blocks_for(nch, 4096)), dim3(TPB), 0, st, sym, n, chunk,
                       nch, (uint32_t)(dict - 1), len, codes, word_off, payload, esc_off, qside, obase, ooff);
  MG_HIP(hipGetLastError());
}

uint64_t decode_table_bytes(int dict) {
  return carve_size<DecTables>(1) + carve_size<uint16_t>((uint64_t)dict) + carve_size<uint32_t>(4);
}

// Full decode entry used by the API: builds the tables, then decodes.
void launch_decode_full(const uint32_t* payload, uint64_t payload_words, const uint64_t* word_off,
                        const uint32_t* chunk_bits, uint64_t n, int dict, int chunk,
                        const uint8_t* len, uint16_t* sym, const uint64_t* esc_off, uint64_t n_out,
                        const int64_t* outliers, int64_t* qside, void* table_scratch,
                        uint32_t* d_status, hipStream_t st) {
  Carver cv(table_scratch);
  DecTables* tab = cv.take<DecTables>(1);
  uint16_t* sorted = cv.take<uint16_t>((uint64_t)dict);
  hipLaunchKernelGGL(k_decode_tables, dim3(1), dim3(1024), 0, st, len, dict, tab, sorted);
  const uint64_t nch = (n + chunk - 1) / chunk;
  if (nch) {
    const unsigned blocks = (unsigned)((nch + 255) / 256);
    KernelTimer kt("decode", st);
    hipLaunchKernelGGL(k_decode, dim3(blocks), dim3(256), 0, st, payload, payload_words, word_off, chunk_bits, n,
                       chunk, nch, tab, sorted, dict, sym, esc_off, n_out, outliers, qside, d_status);
  }
  MG_HIP(hipGetLastError());
}

}  // namespace mg
