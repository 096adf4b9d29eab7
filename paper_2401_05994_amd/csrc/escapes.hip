// Escaped quantized values: per-level fixed-width packing (gfx950).
//
// A value q that does not fit the symbol dictionary (|q| >= R) is coded by the
// Huffman stage as the escape symbol, and its code v = 2 (|q| - R) + [q < 0]
// is stored separately (the lossless stage of Sec. 2; the layout is this
// library's).  Per level l, in stream order, the codes take w_l bits each, w_l
// the bit length of the level's largest code, concatenated most-significant
// bit first into 32-bit words; each level starts on a word boundary.
//
// Compression: the encoder writes the codes compactly (escape j at ecodes[j]);
// then
//   k_esc_starts  index of the first escape of every level (from the chunk
//                 escape offsets and a count inside the chunk that holds the
//                 level's first stream position),
//   k_esc_widths  the largest code per level (segmented maximum),
//   k_esc_layout  counts, widths and word offsets per level, into the header,
//   k_esc_pack    one thread per output word gathers the codes it holds.
// Decompression: k_esc_scatter reads escape j's code from its level's words
// and stores q at the stream position the decoder recorded for it.
#include "internal.hpp"

namespace mg {

namespace {
constexpr int TPB = 256;

inline unsigned grid_for(uint64_t n, unsigned cap) {
  uint64_t g = (n + TPB - 1) / TPB;
  if (g < 1) g = 1;
  return (unsigned)std::min<uint64_t>(g, cap);
}

__device__ inline uint32_t bit_length(uint64_t v) { return v ? 64u - (uint32_t)__clzll((long long)v) : 0u; }

// the level l (0 <= l < nlev) with start[l] <= j < start[l + 1]
__device__ inline int level_of_index(const uint64_t* start, int nlev, uint64_t j) {
  int lo = 0, hi = nlev - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= j)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// One wavefront per l <= nlev: ostart[l] = escapes before stream position
// lt.off[l] (lt.off[nlev] = n): the chunk escape offset of the chunk holding
// that position plus the escape symbols of the chunk before it.
__device__ __forceinline__ void k_esc_starts(G3 mg_bid, G3 mg_gdim, const uint16_t* __restrict__ sym, uint64_t n, int chunk,
                                                   const uint64_t* __restrict__ esc_off, const LevelTable& lt, int nlev,
                                                   uint64_t* __restrict__ ostart) {
  const int l = mg_bid.x;
  const uint64_t p = l == nlev ? n : lt.off[l];
  const uint64_t c = p / (uint64_t)chunk;
  uint32_t cnt = 0;
  for (uint64_t i = c * (uint64_t)chunk + threadIdx.x; i < p; i += 64) cnt += sym[i] == 0;
  for (int m = 32; m > 0; m >>= 1) cnt += (uint32_t)__shfl_xor((int)cnt, m, 64);
  if (threadIdx.x == 0) ostart[l] = esc_off[c] + cnt;
}

__global__ void __launch_bounds__(64) k_esc_starts_k(const uint16_t* __restrict__ sym, uint64_t n, int chunk,
                                                   const uint64_t* __restrict__ esc_off, LevelTable lt, int nlev,
                                                   uint64_t* __restrict__ ostart) {
  k_esc_starts(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, sym, n, chunk, esc_off, lt, nlev, ostart);
}


// wmax[l] = max code of level l (wmax cleared by the caller)
__device__ __forceinline__ void k_esc_widths(G3 mg_bid, G3 mg_gdim, const uint64_t* __restrict__ ecodes,
                                                    const uint64_t* __restrict__ ostart, int nlev,
                                                    unsigned long long* __restrict__ wmax) {
  __shared__ uint64_t st[MAXL + 2];
  __shared__ unsigned long long mx[MAXL + 1];
  for (int l = threadIdx.x; l <= nlev; l += TPB) st[l] = ostart[l];
  for (int l = threadIdx.x; l < nlev; l += TPB) mx[l] = 0;
  __syncthreads();
  const uint64_t total = st[nlev];
  int l = -1;
  unsigned long long m = 0;
  for (uint64_t j = (uint64_t)mg_bid.x * TPB + threadIdx.x; j < total; j += (uint64_t)mg_gdim.x * TPB) {
    if (l < 0 || j >= st[l + 1]) {
      if (l >= 0 && m) atomicMax(&mx[l], m);
      l = level_of_index(st, nlev, j);
      m = 0;
    }
    const unsigned long long v = ecodes[j];
    m = v > m ? v : m;
  }
  if (l >= 0 && m) atomicMax(&mx[l], m);
  __syncthreads();
  for (int k = threadIdx.x; k < nlev; k += TPB)
    if (mx[k]) atomicMax(&wmax[k], mx[k]);
}

__global__ void __launch_bounds__(TPB) k_esc_widths_k(const uint64_t* __restrict__ ecodes,
                                                    const uint64_t* __restrict__ ostart, int nlev,
                                                    unsigned long long* __restrict__ wmax) {
  k_esc_widths(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, ecodes, ostart, nlev, wmax);
}


// Per level: count and width into the header arrays, word offsets into woff
// (nlev + 1 entries, woff[nlev] = all words).
__device__ __forceinline__ void k_esc_layout(G3 mg_bid, G3 mg_gdim, const uint64_t* __restrict__ ostart, const unsigned long long* __restrict__ wmax,
                             int nlev, uint64_t* __restrict__ hdr_counts, uint32_t* __restrict__ hdr_bits,
                             uint64_t* __restrict__ woff) {
  if (threadIdx.x != 0) return;
  uint64_t w = 0;
  for (int l = 0; l < nlev; ++l) {
    const uint64_t cnt = ostart[l + 1] - ostart[l];
    const uint32_t b = cnt ? bit_length(wmax[l]) : 0u;
    hdr_counts[l] = cnt;
    hdr_bits[l] = b;
    woff[l] = w;
    w += (cnt * b + 31) / 32;
  }
  woff[nlev] = w;
}

__global__ void k_esc_layout_k(const uint64_t* __restrict__ ostart, const unsigned long long* __restrict__ wmax,
                             int nlev, uint64_t* __restrict__ hdr_counts, uint32_t* __restrict__ hdr_bits,
                             uint64_t* __restrict__ woff) {
  k_esc_layout(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, ostart, wmax, nlev, hdr_counts, hdr_bits, woff);
}


// Bits [b, b + w) (w <= 64) of a word array of nw words, most-significant bit
// first; words past the end read as 0.
__device__ inline uint64_t read_bits(const uint32_t* __restrict__ words, uint64_t nw, uint64_t b, uint32_t w) {
  if (w == 0) return 0;
  const uint64_t i = b >> 5;
  const uint32_t off = (uint32_t)(b & 31);
  const uint64_t w0 = i < nw ? words[i] : 0u;
  const uint64_t w1 = i + 1 < nw ? words[i + 1] : 0u;
  const uint64_t hi = (w0 << 32) | w1;
  uint64_t v = (hi << off) >> (64 - w);
  if (off + w > 64) {
    const uint64_t w2 = i + 2 < nw ? words[i + 2] : 0u;
    v |= w2 >> (96 - off - w);
  }
  return v;
}

// One thread per output word (grid-stride): word j of level l holds bits
// [32 (j - woff[l]), +32) of the level's concatenated codes.  The words go
// after the payload (d_out + payload_off + 4 word_off[nch]).
__device__ __forceinline__ void k_esc_pack(G3 mg_bid, G3 mg_gdim, const uint64_t* __restrict__ ecodes,
                                                  const uint64_t* __restrict__ ostart,
                                                  const uint64_t* __restrict__ woff_g,
                                                  const uint32_t* __restrict__ bits_g, int nlev, char* d_out,
                                                  uint64_t payload_off, const uint64_t* __restrict__ word_off,
                                                  uint64_t nch) {
  __shared__ uint64_t st[MAXL + 2], wo[MAXL + 2];
  __shared__ uint32_t wb[MAXL + 1];
  for (int l = threadIdx.x; l <= nlev; l += TPB) {
    st[l] = ostart[l];
    wo[l] = woff_g[l];
    if (l < nlev) wb[l] = bits_g[l];
  }
  __syncthreads();
  uint32_t* out = reinterpret_cast<uint32_t*>(d_out + payload_off + 4 * word_off[nch]);
  const uint64_t total = wo[nlev];
  for (uint64_t j = (uint64_t)mg_bid.x * TPB + threadIdx.x; j < total; j += (uint64_t)mg_gdim.x * TPB) {
    const int l = level_of_index(wo, nlev, j);
    const uint32_t w = wb[l];  // > 0: a level without bits has no words
    const uint64_t cnt = st[l + 1] - st[l];
    const uint64_t b0 = 32 * (j - wo[l]);
    const uint64_t b1 = min(b0 + 32, cnt * w);
    uint32_t word = 0;
    for (uint64_t k = b0 / w; k * w < b1; ++k) {
      const uint64_t s = k * w, e = s + w;
      const uint64_t lo = s > b0 ? s : b0, hi = e < b1 ? e : b1;
      const uint32_t nb = (uint32_t)(hi - lo);
      uint64_t part = ecodes[st[l] + k] >> (e - hi);
      part &= nb >= 64 ? ~0ull : ((1ull << nb) - 1ull);
      word |= (uint32_t)(part << (b0 + 32 - hi));
    }
    out[j] = word;
  }
}

__global__ void __launch_bounds__(TPB) k_esc_pack_k(const uint64_t* __restrict__ ecodes,
                                                  const uint64_t* __restrict__ ostart,
                                                  const uint64_t* __restrict__ woff_g,
                                                  const uint32_t* __restrict__ bits_g, int nlev, char* d_out,
                                                  uint64_t payload_off, const uint64_t* __restrict__ word_off,
                                                  uint64_t nch) {
  k_esc_pack(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, ecodes, ostart, woff_g, bits_g, nlev, d_out, payload_off, word_off, nch);
}


// qside[epos[j]] = q of escape j, once every chunk has decoded cleanly; an
// escape whose recorded position lies outside the level its index belongs to
// marks the buffer malformed.
__global__ void __launch_bounds__(TPB) k_esc_scatter(const uint64_t* __restrict__ epos,
                                                     const uint32_t* __restrict__ words, uint64_t nw, EscLevels t,
                                                     int R, uint64_t n, int64_t* __restrict__ qside,
                                                     uint32_t* __restrict__ status) {
  if (*status) return;
  const uint64_t total = t.ostart[t.nlev];
  for (uint64_t j = (uint64_t)blockIdx.x * TPB + threadIdx.x; j < total; j += (uint64_t)gridDim.x * TPB) {
    const int l = level_of_index(t.ostart, t.nlev, j);
    const uint64_t p = epos[j];
    if (p >= n || p < t.loff[l] || p >= t.loff[l + 1]) {
      atomicOr(status, 1u);
      return;
    }
    const uint32_t w = t.bits[l];
    const uint64_t v = read_bits(words, nw, 32 * t.woff[l] + (j - t.ostart[l]) * w, w);
    const int64_t mag = (int64_t)(v >> 1) + (int64_t)R;
    qside[p] = (v & 1) ? -mag : mag;
  }
}

}  // namespace

void launch_escape_pack(const uint16_t* sym, uint64_t n, int chunk, const uint64_t* esc_off, const uint64_t* word_off,
                        uint64_t nch, const uint64_t* ecodes, int nlev, const LevelTable& lt, char* d_out,
                        uint64_t payload_off, uint64_t* hdr_counts, uint32_t* hdr_bits, uint64_t* ostart,
                        unsigned long long* wmax, uint64_t* woff, hipStream_t st) {
  KernelTimer kt("escapes", st);
  launch_fill_u64(reinterpret_cast<uint64_t*>(wmax), (uint64_t)nlev, 0, st);
  MG_LAUNCH((&k_esc_starts), (k_esc_starts_k), (64), (0), (dim3(nlev + 1)), st, sym, n, chunk, esc_off, lt, nlev, ostart);
  // few escapes unless the tolerance is tight: blocks past the escapes return
  // at once, so the grids assume at least 32 (64) stream positions per thread
  MG_LAUNCH((&k_esc_widths), (k_esc_widths_k), (TPB), (0), (dim3(grid_for(n / 32, 1024))), st, ecodes, ostart, nlev, wmax);
  MG_LAUNCH((&k_esc_layout), (k_esc_layout_k), (64), (0), (dim3(1)), st, ostart, wmax, nlev, hdr_counts, hdr_bits, woff);
  MG_LAUNCH((&k_esc_pack), (k_esc_pack_k), (TPB), (0), (dim3(grid_for(n / 64, 2048))), st, ecodes, ostart, woff, static_cast<const uint32_t*>(hdr_bits), nlev, d_out, payload_off, word_off, nch);
  MG_HIP(hipGetLastError());
}

void launch_escape_scatter(const uint64_t* epos, const uint32_t* words, uint64_t nw, const EscLevels& t, int R,
                           uint64_t n, int64_t* qside, uint32_t* status, hipStream_t st) {
  const uint64_t total = t.ostart[t.nlev];
  if (!total) return;
  hipLaunchKernelGGL(k_esc_scatter, dim3(grid_for(total, 4096)), dim3(TPB), 0, st, epos, words, nw, t, R, n, qside,
                     status);
  MG_HIP(hipGetLastError());
}

}  // namespace mg
