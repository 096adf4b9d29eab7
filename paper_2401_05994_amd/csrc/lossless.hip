// Second-stage lossless coder: zero suppression by two-level bitmaps (gfx950).
//
// Paper Sec. 2: the entropy-coded output goes through a final lossless stage.
// What this pipeline leaves for that stage are zero bits -- the all-zero
// shortest code of a dominant Huffman symbol, the mostly-zero high bitplanes
// of the refactoring -- so the stage suppresses zero words, chunk by chunk,
// with no sequential parse:
//   words in chunks of 4096 (the last may be shorter, m words); level-1
//   bitmap: bit 31 - i%32 of word i/32 set when data word i is nonzero;
//   level-2 bitmap: the same over the level-1 words; a coded chunk is the
//   level-2 bitmap, the nonzero level-1 words, the nonzero data words; it is
//   stored raw when that is not shorter than m (a stored length of m means
//   raw).  Container: 'MGZS', u16 version 1, u16 0, u64 raw bytes, u64
//   chunks, u64 word offsets[chunks + 1], then the stored chunks.
//
// One 256-thread block per chunk.  Lane i of a wavefront holds word
// 256 r + 64 w + i in iteration r, so the ballot of "nonzero" gives level-1
// words 8r + 2w and 8r + 2w + 1 (bit-reversed: the container is most
// significant bit first).  Encoding sizes every chunk, scans the sizes into
// the offset table, then writes; decoding checks each chunk's bitmaps
// against its stored length before it reads a data word.
#include <cstring>

#include "internal.hpp"

namespace mg {

namespace {

constexpr int ZS_T = 256;
constexpr int ZS_CHUNK = 4096;
constexpr int ZS_PER = ZS_CHUNK / ZS_T;      // 16 words per thread
constexpr int ZS_L1 = ZS_CHUNK / 32;         // 128 level-1 words
constexpr uint64_t ZS_FIXED = 24;

// Word i of the input; the last word of an input whose length is not a
// multiple of 4 is read byte by byte (zero padded).
__device__ inline uint32_t zs_word(const uint32_t* __restrict__ in, uint64_t i, uint64_t nwords, uint32_t tail) {
  if (i + 1 < nwords || tail == 0) return in[i];
  const uint8_t* b = reinterpret_cast<const uint8_t*>(in + i);
  uint32_t v = 0;
  for (uint32_t k = 0; k < tail; ++k) v |= (uint32_t)b[k] << (8 * k);
  return v;
}

struct ZsChunk {
  uint32_t m, n1, n2, nz1, nnz;
};

// Loads the chunk's words (v), builds the level-1 bitmap in LDS (l1) and the
// counts; every thread returns the same counts.
__device__ inline ZsChunk zs_scan_chunk(const uint32_t* __restrict__ in, uint64_t nwords, uint32_t tail,
                                        uint64_t k, uint32_t (&v)[ZS_PER], uint32_t* l1, uint32_t* cnt) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  ZsChunk c;
  const uint64_t base = k * ZS_CHUNK;
  c.m = (uint32_t)min((uint64_t)ZS_CHUNK, nwords - base);
  c.n1 = (c.m + 31) / 32;
  c.n2 = (c.n1 + 31) / 32;
  if (t < 2) cnt[t] = 0;
#pragma unroll
  for (int r = 0; r < ZS_PER; ++r) {
    const uint32_t i = (uint32_t)(r * ZS_T + t);
    v[r] = i < c.m ? zs_word(in, base + i, nwords, tail) : 0u;
  }
  __syncthreads();
  uint32_t nnz = 0;
#pragma unroll
  for (int r = 0; r < ZS_PER; ++r) {
    const uint64_t bm = __ballot(v[r] != 0u);
    if (lane == 0) {
      l1[8 * r + 2 * wv] = __brev((uint32_t)bm);
      l1[8 * r + 2 * wv + 1] = __brev((uint32_t)(bm >> 32));
    }
    nnz += (uint32_t)__popcll(bm);
  }
  __syncthreads();
  if (lane == 0) atomicAdd(&cnt[0], nnz);
  if (t < ZS_L1 && l1[t] != 0u) atomicAdd(&cnt[1], 1u);
  __syncthreads();
  c.nnz = cnt[0];
  c.nz1 = cnt[1];
  return c;
}

__device__ inline uint32_t zs_stored(const ZsChunk& c) {
  const uint32_t coded = c.n2 + c.nz1 + c.nnz;
  return coded < c.m ? coded : c.m;
}

__global__ void __launch_bounds__(ZS_T) k_zs_sizes(const uint32_t* __restrict__ in, uint64_t nwords, uint32_t tail,
                                                   uint32_t* __restrict__ sizes) {
  __shared__ uint32_t l1[ZS_L1];
  __shared__ uint32_t cnt[2];
  uint32_t v[ZS_PER];
  const ZsChunk c = zs_scan_chunk(in, nwords, tail, blockIdx.x, v, l1, cnt);
  if (threadIdx.x == 0) sizes[blockIdx.x] = zs_stored(c);
}

// Exclusive prefix of x over the first 128 threads (x of the others
// ignored), through sh (128 entries); *total receives the sum.
__device__ inline uint32_t zs_prefix128(uint32_t x, uint32_t* sh, uint32_t* total) {
  const int t = threadIdx.x;
  if (t < ZS_L1) sh[t] = x;
  __syncthreads();
  for (int d = 1; d < ZS_L1; d <<= 1) {
    uint32_t y = 0;
    if (t < ZS_L1 && t >= d) y = sh[t - d];
    __syncthreads();
    if (t < ZS_L1) sh[t] += y;
    __syncthreads();
  }
  const uint32_t incl = t < ZS_L1 ? sh[t] : 0u;
  *total = sh[ZS_L1 - 1];
  __syncthreads();
  return incl - (t < ZS_L1 ? x : 0u);
}

__global__ void __launch_bounds__(ZS_T) k_zs_write(const uint32_t* __restrict__ in, uint64_t nwords, uint32_t tail,
                                                   const uint64_t* __restrict__ offs, uint32_t* __restrict__ data) {
  __shared__ uint32_t l1[ZS_L1];
  __shared__ uint32_t pre_bits[ZS_L1];
  __shared__ uint32_t cnt[2];
  __shared__ uint32_t sh[ZS_L1];
  const int t = threadIdx.x;
  uint32_t v[ZS_PER];
  const ZsChunk c = zs_scan_chunk(in, nwords, tail, blockIdx.x, v, l1, cnt);
  uint32_t* out = data + offs[blockIdx.x];
  if (zs_stored(c) == c.m) {
#pragma unroll
    for (int r = 0; r < ZS_PER; ++r) {
      const uint32_t i = (uint32_t)(r * ZS_T + t);
      if (i < c.m) out[i] = v[r];
    }
    return;
  }
  const uint32_t w1 = t < ZS_L1 ? l1[t] : 0u;
  uint32_t unused;
  const uint32_t pb = zs_prefix128((uint32_t)__popc(w1), sh, &unused);
  const uint32_t pn = zs_prefix128(w1 != 0u ? 1u : 0u, sh, &unused);
  if (t < ZS_L1) pre_bits[t] = pb;
  // level-2 bitmap: waves 0 and 1 cover level-1 words 0..127
  if (t < ZS_L1) {
    const uint64_t bm = __ballot(w1 != 0u);
    const int lane = t & 63, wv = t >> 6;
    if (lane == 0 && 2 * wv < (int)c.n2) out[2 * wv] = __brev((uint32_t)bm);
    if (lane == 0 && 2 * wv + 1 < (int)c.n2) out[2 * wv + 1] = __brev((uint32_t)(bm >> 32));
    if (w1 != 0u) out[c.n2 + pn] = w1;
  }
  __syncthreads();
  const uint32_t dbase = c.n2 + c.nz1;
#pragma unroll
  for (int r = 0; r < ZS_PER; ++r) {
    const uint32_t i = (uint32_t)(r * ZS_T + t);
    if (v[r] != 0u) {
      const uint32_t q = i >> 5, b = i & 31;
      const uint32_t before = b ? (uint32_t)__popc(l1[q] >> (32 - b)) : 0u;
      out[dbase + pre_bits[q] + before] = v[r];
    }
  }
}

__global__ void __launch_bounds__(ZS_T) k_zs_decode(const uint32_t* __restrict__ data, uint64_t data_words,
                                                    const uint64_t* __restrict__ offs, uint64_t nwords,
                                                    uint32_t* __restrict__ outw, uint32_t* __restrict__ status) {
  __shared__ uint32_t l1[ZS_L1];
  __shared__ uint32_t pre_bits[ZS_L1];
  __shared__ uint32_t sh[ZS_L1];
  __shared__ uint32_t bad;
  const int t = threadIdx.x;
  const uint64_t k = blockIdx.x;
  const uint64_t base = k * ZS_CHUNK;
  const uint32_t m = (uint32_t)min((uint64_t)ZS_CHUNK, nwords - base);
  const uint32_t n1 = (m + 31) / 32, n2 = (n1 + 31) / 32;
  const uint64_t o0 = offs[k], o1 = offs[k + 1];
  uint32_t* out = outw + base;
  if (o1 < o0 || o1 > data_words || o1 - o0 > m || o1 - o0 < n2) {
    if (t == 0) atomicOr(status, 1u);
    return;
  }
  const uint32_t len = (uint32_t)(o1 - o0);
  const uint32_t* in = data + o0;
  if (len == m) {
#pragma unroll
    for (int r = 0; r < ZS_PER; ++r) {
      const uint32_t i = (uint32_t)(r * ZS_T + t);
      if (i < m) out[i] = in[i];
    }
    return;
  }
  if (t == 0) bad = 0;
  __syncthreads();
  // level-1 flags from the level-2 bitmap (n2 <= len words); flags past the
  // chunk's level-1 words must be clear
  bool f1 = false;
  if (t < (int)(32 * n2)) {
    const bool set = (in[t >> 5] >> (31 - (t & 31))) & 1u;
    f1 = set && t < (int)n1;
    if (set && t >= (int)n1) bad = 1;  // any writer stores the same value
  }
  uint32_t nz1 = 0;
  const uint32_t pn = zs_prefix128(f1 ? 1u : 0u, sh, &nz1);
  // the level-1 words: each must lie inside the chunk and be nonzero
  uint32_t w1 = 0;
  if (f1) {
    const uint32_t at = n2 + pn;
    if (at < len) w1 = in[at];
    if (at >= len || w1 == 0u) bad = 1;
  }
  // level-1 bits past the chunk's last data word must be clear
  if (t == (int)n1 - 1 && (m & 31) && (w1 & ((1u << (32 - (m & 31))) - 1u))) bad = 1;
  if (t < ZS_L1) l1[t] = w1;
  uint32_t tot = 0;
  const uint32_t pb = zs_prefix128(t < ZS_L1 ? (uint32_t)__popc(w1) : 0u, sh, &tot);
  if (t < ZS_L1) pre_bits[t] = pb;
  __syncthreads();
  // every data word the bitmaps point to lies inside the stored chunk
  if (bad || n2 + nz1 + tot != len) {
    if (t == 0) atomicOr(status, 1u);
    return;
  }
  const uint32_t dbase = n2 + nz1;
#pragma unroll
  for (int r = 0; r < ZS_PER; ++r) {
    const uint32_t i = (uint32_t)(r * ZS_T + t);
    if (i < m) {
      const uint32_t q = i >> 5, b = i & 31;
      const uint32_t w = l1[q];
      uint32_t val = 0;
      if ((w >> (31 - b)) & 1u) val = in[dbase + pre_bits[q] + (b ? (uint32_t)__popc(w >> (32 - b)) : 0u)];
      out[i] = val;
    }
  }
}

}  // namespace

uint64_t zs_bound(uint64_t raw_bytes) {
  const uint64_t nw = (raw_bytes + 3) / 4;
  const uint64_t nch = (nw + ZS_CHUNK - 1) / ZS_CHUNK;
  return ZS_FIXED + 8 * (nch + 1) + 4 * nw;
}

// Encodes raw_bytes of d_in (4-byte aligned) into the container at d_out;
// returns the container's size (synchronises st).  scratch: nch + 1 words.
uint64_t zs_encode(const void* d_in, uint64_t raw_bytes, void* d_out, uint64_t capacity, uint32_t* d_sizes,
                   hipStream_t st) {
  const uint64_t nw = (raw_bytes + 3) / 4;
  const uint64_t nch = (nw + ZS_CHUNK - 1) / ZS_CHUNK;
  const uint32_t tail = (uint32_t)(raw_bytes & 3);
  if (capacity < ZS_FIXED + 8 * (nch + 1)) fail(MGARD_ERR_CAPACITY, "output capacity below mgard_lossless_bound");
  uint8_t head[ZS_FIXED] = {0};
  std::memcpy(head, "MGZS", 4);
  const uint16_t ver = 1;
  std::memcpy(head + 4, &ver, 2);
  std::memcpy(head + 8, &raw_bytes, 8);
  std::memcpy(head + 16, &nch, 8);
  char* out = static_cast<char*>(d_out);
  MG_HIP(hipMemcpyAsync(out, head, ZS_FIXED, hipMemcpyHostToDevice, st));
  uint64_t* offs = reinterpret_cast<uint64_t*>(out + ZS_FIXED);
  uint32_t* data = reinterpret_cast<uint32_t*>(out + ZS_FIXED + 8 * (nch + 1));
  const uint32_t* in = static_cast<const uint32_t*>(d_in);
  KernelTimer kt("lossless_encode", st);
  if (nch) hipLaunchKernelGGL(k_zs_sizes, dim3((unsigned)nch), dim3(ZS_T), 0, st, in, nw, tail, d_sizes);
  launch_scan_u32(d_sizes, nch, offs, st);
  uint64_t total = 0;
  MG_HIP(hipMemcpyAsync(&total, offs + nch, 8, hipMemcpyDeviceToHost, st));
  MG_HIP(hipStreamSynchronize(st));
  const uint64_t bytes = ZS_FIXED + 8 * (nch + 1) + 4 * total;
  if (bytes > capacity) fail(MGARD_ERR_CAPACITY, "output capacity below mgard_lossless_bound");
  if (nch) hipLaunchKernelGGL(k_zs_write, dim3((unsigned)nch), dim3(ZS_T), 0, st, in, nw, tail, offs, data);
  MG_HIP(hipGetLastError());
  MG_HIP(hipStreamSynchronize(st));
  return bytes;
}

// Parses the container's fixed part (host copy h, 24 bytes).
bool zs_parse(const uint8_t* h, uint64_t bytes, uint64_t* raw_bytes, uint64_t* nch) {
  if (bytes < ZS_FIXED || std::memcmp(h, "MGZS", 4) != 0) return false;
  uint16_t ver = 0;
  std::memcpy(&ver, h + 4, 2);
  if (ver != 1) return false;
  std::memcpy(raw_bytes, h + 8, 8);
  std::memcpy(nch, h + 16, 8);
  const uint64_t nw = (*raw_bytes + 3) / 4;
  return *nch == (nw + ZS_CHUNK - 1) / ZS_CHUNK && *nch < (1ull << 40) && bytes >= ZS_FIXED + 8 * (*nch + 1);
}

// Decodes the container (in_bytes at d_in) into d_out (capacity >= 4
// ceil(raw/4)); MGARD_ERR_FORMAT for malformed input.  status: one word.
void zs_decode(const void* d_in, uint64_t in_bytes, uint64_t raw_bytes, uint64_t nch, void* d_out, uint32_t* status,
               hipStream_t st) {
  const uint64_t nw = (raw_bytes + 3) / 4;
  const char* in = static_cast<const char*>(d_in);
  const uint64_t* offs = reinterpret_cast<const uint64_t*>(in + ZS_FIXED);
  const uint64_t dstart = ZS_FIXED + 8 * (nch + 1);
  const uint64_t data_words = (in_bytes - dstart) / 4;
  launch_fill_u64(reinterpret_cast<uint64_t*>(status), 1, 0, st);
  KernelTimer kt("lossless_decode", st);
  if (nch)
    hipLaunchKernelGGL(k_zs_decode, dim3((unsigned)nch), dim3(ZS_T), 0, st,
                       reinterpret_cast<const uint32_t*>(in + dstart), data_words, offs, nw,
                       static_cast<uint32_t*>(d_out), status);
  MG_HIP(hipGetLastError());
  uint32_t hs = 0;
  MG_HIP(hipMemcpyAsync(&hs, status, 4, hipMemcpyDeviceToHost, st));
  MG_HIP(hipStreamSynchronize(st));
  if (hs) fail(MGARD_ERR_FORMAT, "malformed zero-suppressed data");
}

}  // namespace mg
