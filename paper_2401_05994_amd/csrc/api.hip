// C interface: argument checks, scratch layout, pipelines and the wire format.
//
// Compression (paper Sec. 2 and the first listing of Sec. 3): max|u| ->
// bin widths on the device -> decomposition with fused quantization ->
// histogram -> codebook -> chunk sizes -> encode, every table written
// straight into the caller's output buffer; one readback returns the size.
// Decompression reads the self-describing header (Sec. 2.1) back to the host,
// validates it, then decodes and recomposes on the device.
//
// Wire format (little-endian, byte offsets), version 2:
//    0 'MGHP'  4 u16 version  6 u8 dtype  7 u8 ndim  8 u8 eb  9 u8 alloc
//   10 u8 coord_flags  11 u8 fallback  12 u32 L  16 u32 dict  20 u32 chunk
//   24 f64 tol  32 f64 tau_abs  40 f64 maxabs  48 u64 n_symbols
//   56 u64 n_chunks  64 u64 n_outliers  72 u64 payload_words
//   80 u8 norm (0 L-infinity, 1 s-norm)  81 u8[7] zero  88 f64 s
//   96 u64 shape[ndim], f64 coordinates of flagged dimensions, f64 bins[L+1],
//   u64 level_escapes[L+1], u32 level_escape_bits[L+1], u8 code_len[dict],
//   u32 chunk_bits[n_chunks], u32 chunk_esc[n_chunks], u32 payload[payload_words],
//   u32 escape words (per level, ceil(count * bits / 32), escapes.hip).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

// Scratch of mgard_huffman_encode_noalloc, for callers that cannot allocate:
// the chunk word offsets (MGARD_NOALLOC_MAX_CHUNKS + 1 of them) and the
// encoder's packed code table, in one fixed array that each device holds from
// the library's load to the end of the process.  In host code this name is
// not a device address: the address comes from hipGetSymbolAddress, per
// device (mg::noalloc_scratch).
constexpr unsigned long long kNoallocBytes =
    (((unsigned long long)MGARD_NOALLOC_MAX_CHUNKS + 1) * 8 + 255) / 256 * 256 + 8192 * 4 + 256 + 256;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

// Device-resident network parameters (MLP layout of internal.hpp).
struct mgard_model {
  float* d_params = nullptr;
  int device = -1;
};

// A captured batch: the graph, its executable form and the one device
// allocation holding every field's static header and scratch.
struct mgard_batch {
  int device = -1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* mem = nullptr;     // every field's static header and scratch
  void* tables = nullptr;  // the grouped launches' job tables
  uint32_t launches = 0;   // grouped launches per graph launch
};

namespace mg {

void fail(mgard_status code, const std::string& msg) { throw Failure{code, msg}; }

Recorder*& recorder() {
  thread_local Recorder* r = nullptr;
  return r;
}

namespace {
// device-to-device copy of whole 8-byte words, as a kernel a batch can regroup
__device__ __forceinline__ void k_copy_u64(G3 mg_bid, G3 mg_gdim, uint64_t* __restrict__ dst,
                                           const uint64_t* __restrict__ src, uint64_t n) {
  for (uint64_t i = (uint64_t)mg_bid.x * 256 + threadIdx.x; i < n; i += (uint64_t)mg_gdim.x * 256) dst[i] = src[i];
}
__global__ void __launch_bounds__(256) k_copy_u64_k(uint64_t* __restrict__ dst, const uint64_t* __restrict__ src,
                                                    uint64_t n) {
  k_copy_u64(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, dst, src, n);
}
}  // namespace

// A static header copied into a stream's output: a copy on the stream, or a
// recorded copy kernel while a batch records (its bytes are whole words).
void copy_d2d(void* dst, const void* src, uint64_t bytes, hipStream_t st) {
  if (!recorder()) {
    MG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
    return;
  }
  if (bytes % 8 || reinterpret_cast<uintptr_t>(dst) % 8 || reinterpret_cast<uintptr_t>(src) % 8)
    fail(MGARD_ERR_ARG, "recorded copies move whole aligned words");
  const uint64_t n = bytes / 8;
  MG_LAUNCH((&k_copy_u64), (k_copy_u64_k), (256), (0), (dim3((unsigned)std::max<uint64_t>(1, std::min<uint64_t>((n + 255) / 256, 1024)))), st, static_cast<uint64_t*>(dst), static_cast<const uint64_t*>(src), n);
}

static const float* model_params(const mgard_model* m) {
  int dev = 0;
  MG_HIP(hipGetDevice(&dev));
  if (!m->d_params || m->device != dev) fail(MGARD_ERR_ARG, "model lives on another device");
  return m->d_params;
}

namespace {

thread_local std::string g_err;

template <typename F>
mgard_status guard(F&& f) {
  try {
    f();
    g_err.clear();
    return MGARD_OK;
  } catch (const Failure& e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return MGARD_ERR_OOM;
  } catch (...) {
    g_err = "unexpected exception";
    return MGARD_ERR_ARG;
  }
}

constexpr uint16_t kVersion = 2;
constexpr uint64_t kFixed = 96;

struct Opts {
  int eb = MGARD_REL;
  int alloc = MGARD_ALLOC_PLAIN;
  int norm = MGARD_NORM_LINF;
  double s = 0.0;
  int dict = 8192;
  int chunk = 1024;
  int lossless = MGARD_LOSSLESS_NONE;
  hipStream_t st = nullptr;
  const mgard_model* model = nullptr;
  const float* model_params = nullptr;  // device parameters of the model
};

Opts read_opts(const mgard_opts* o) {
  Opts r;
  if (!o) return r;
  // the options before the norm fields were added are accepted as well (L-infinity)
  const bool with_norm = o->struct_size == sizeof(mgard_opts);
  if (!with_norm && o->struct_size != offsetof(mgard_opts, norm)) fail(MGARD_ERR_ARG, "opts->struct_size mismatch");
  if (o->eb > 1) fail(MGARD_ERR_ARG, "opts->eb");
  if (o->alloc > 2) fail(MGARD_ERR_ARG, "opts->alloc");
  r.eb = (int)o->eb;
  r.alloc = (int)o->alloc;
  if (with_norm) {
    if (o->norm > 1) fail(MGARD_ERR_ARG, "opts->norm");
    r.norm = (int)o->norm;
    if (r.norm == MGARD_NORM_S) {
      if (!std::isfinite(o->s) || std::fabs(o->s) > 64.0) fail(MGARD_ERR_ARG, "opts->s must be finite, |s| <= 64");
      if (r.alloc != MGARD_ALLOC_PLAIN) fail(MGARD_ERR_ARG, "the s-norm bound takes the plain allocation");
      if (r.eb == MGARD_REL && o->s != 0.0) fail(MGARD_ERR_ARG, "a relative s-norm bound needs s = 0");
      r.s = o->s;
    }
  }
  if (o->dict_size) {
    const uint32_t d = o->dict_size;
    if (d < 256 || d > 8192 || (d & (d - 1))) fail(MGARD_ERR_ARG, "dict_size must be a power of two in [256, 8192]");
    r.dict = (int)d;
  }
  if (o->chunk_symbols) {
    const uint32_t c = o->chunk_symbols;
    if (c < 256 || c > 8192 || (c % 256)) fail(MGARD_ERR_ARG, "chunk_symbols must be a multiple of 256 in [256, 8192]");
    r.chunk = (int)c;
  }
  if (o->lossless > MGARD_LOSSLESS_ZS) fail(MGARD_ERR_ARG, "opts->lossless");
  r.lossless = (int)o->lossless;
  r.st = static_cast<hipStream_t>(o->stream);
  r.model = o->model;
  return r;
}

int dtype_size(mgard_dtype t) {
  if (t == MGARD_F32) return 4;
  if (t == MGARD_F64) return 8;
  fail(MGARD_ERR_DTYPE, "dtype must be MGARD_F32 or MGARD_F64");
}

uint64_t align8(uint64_t v) { return (v + 7) & ~uint64_t(7); }

struct Layout {
  uint64_t bins, lesc, lbits, code_len, chunk_bits, chunk_esc, payload;  // byte offsets
  uint64_t nch;
};

Layout layout(const Hierarchy& h, const double* const* coords, int dict, int chunk, uint64_t n) {
  Layout y{};
  uint64_t p = kFixed + 8ull * h.D;
  for (int d = 0; d < h.D; ++d)
    if (coords && coords[d]) p += 8ull * h.shape[d + (MAXD - h.D)];
  y.bins = p;
  p += 8ull * (h.L + 1);
  y.lesc = p;
  p += 8ull * (h.L + 1);
  y.lbits = p;
  p += 4ull * (h.L + 1);
  y.code_len = p;
  p += (uint64_t)dict;
  y.nch = (n + chunk - 1) / chunk;
  y.chunk_bits = p;
  p += 4 * y.nch;
  y.chunk_esc = p;
  p += 4 * y.nch;
  y.payload = p;
  return y;
}

// worst case: log2(dict)+1 bits per symbol, and every symbol escapes with a
// 64-bit code (plus one padding word per level)
uint64_t bound_of(const Hierarchy& h, const double* const* coords, int dict, int chunk) {
  const uint64_t n = h.count(h.L);
  Layout y = layout(h, coords, dict, chunk, n);
  int lg = 0;
  while ((1 << lg) < dict) ++lg;
  const uint64_t words = (n * (uint64_t)(lg + 1) + 31) / 32 + y.nch;
  return align8(y.payload + 4 * words) + 8 * n + 4ull * (h.L + 1) + 64;
}

struct Finale {  // device results read back by the host at the end
  uint64_t total_bytes, n_outliers, payload_words, pad;
  double scalars[8];  // tau_abs, maxabs, nonfinite, tau_eff, measured Linf, fallback used
  double bins[MAXL + 1];
};

__device__ __forceinline__ void k_finalize(G3 mg_bid, G3 mg_gdim, char* out, const uint64_t* word_off, const uint64_t* esc_off, uint64_t nch,
                           uint64_t payload_off, const uint64_t* esc_words, const double* scalars,
                           const double* bins, int L, uint64_t bins_off, int learned, Finale* fin,
                           uint64_t* size_out) {
  const int fallback = learned && scalars[5] != 0.0 ? 1 : 0;
  // a field that cannot be compressed (NaN or infinity in the input, or a
  // tolerance outside the supported range) reports size 0
  const bool rejected = scalars[2] != 0.0 || scalars[6] != 0.0;
  if (threadIdx.x != 0) return;
  const uint64_t pw = word_off[nch], no = esc_off[nch];
  double* hd = reinterpret_cast<double*>(out);
  hd[4] = scalars[0];  // tau_abs at 32
  hd[5] = scalars[1];  // maxabs at 40
  uint64_t* hu = reinterpret_cast<uint64_t*>(out);
  hu[8] = no;  // 64
  hu[9] = pw;  // 72
  out[11] = (char)fallback;
  double* bo = reinterpret_cast<double*>(out + bins_off);
  for (int l = 0; l <= L; ++l) bo[l] = bins[l];
  fin->total_bytes = payload_off + 4 * pw + 4 * *esc_words;
  if (size_out) *size_out = rejected ? 0 : fin->total_bytes;
  fin->n_outliers = no;
  fin->payload_words = pw;
  for (int i = 0; i < 7; ++i) fin->scalars[i] = scalars[i];
  if (!learned) {
    fin->scalars[4] = -1.0;
    fin->scalars[5] = 0.0;
  }
  for (int l = 0; l <= L; ++l) fin->bins[l] = bins[l];
}

__global__ void k_finalize_k(char* out, const uint64_t* word_off, const uint64_t* esc_off, uint64_t nch,
                           uint64_t payload_off, const uint64_t* esc_words, const double* scalars,
                           const double* bins, int L, uint64_t bins_off, int learned, Finale* fin,
                           uint64_t* size_out) {
  k_finalize(G3{blockIdx.x, blockIdx.y, blockIdx.z}, G3{gridDim.x, gridDim.y, gridDim.z}, out, word_off, esc_off, nch, payload_off, esc_words, scalars, bins, L, bins_off, learned, fin, size_out);
}


std::vector<uint8_t> header_bytes(const Hierarchy& h, const double* const* coords, int dtype, int eb,
                                  int alloc, double tol, int dict, int chunk, uint64_t n,
                                  uint64_t nch, int norm = MGARD_NORM_LINF, double snorm = 0.0) {
  std::vector<uint8_t> b(kFixed, 0);
  auto w16 = [&](size_t o, uint16_t v) { std::memcpy(&b[o], &v, 2); };
  auto w32 = [&](size_t o, uint32_t v) { std::memcpy(&b[o], &v, 4); };
  auto w64 = [&](size_t o, uint64_t v) { std::memcpy(&b[o], &v, 8); };
  auto wd = [&](size_t o, double v) { std::memcpy(&b[o], &v, 8); };
  std::memcpy(&b[0], "MGHP", 4);
  w16(4, kVersion);
  b[6] = (uint8_t)dtype;
  b[7] = (uint8_t)h.D;
  b[8] = (uint8_t)eb;
  b[9] = (uint8_t)alloc;
  uint8_t flags = 0;
  for (int d = 0; d < h.D; ++d)
    if (coords && coords[d]) flags |= (uint8_t)(1u << d);
  b[10] = flags;
  b[11] = 0;
  w32(12, (uint32_t)h.L);
  w32(16, (uint32_t)dict);
  w32(20, (uint32_t)chunk);
  wd(24, tol);
  wd(32, 0.0);
  wd(40, 0.0);
  w64(48, n);
  w64(56, nch);
  w64(64, 0);
  w64(72, 0);
  b[80] = (uint8_t)norm;
  wd(88, norm == MGARD_NORM_S ? snorm : 0.0);
  const int pad = MAXD - h.D;
  for (int d = 0; d < h.D; ++d) {
    uint64_t s = (uint64_t)h.shape[d + pad];
    const uint8_t* p = reinterpret_cast<const uint8_t*>(&s);
    b.insert(b.end(), p, p + 8);
  }
  for (int d = 0; d < h.D; ++d)
    if (coords && coords[d]) {
      const uint8_t* p = reinterpret_cast<const uint8_t*>(coords[d]);
      b.insert(b.end(), p, p + 8 * h.shape[d + pad]);
    }
  return b;
}

// Parses a header held on the host; fills hdr and, optionally, coordinates.
struct Parsed {
  mgard_header hd{};
  std::vector<std::vector<double>> coords;
  uint64_t bins_off = 0, lesc = 0, lbits = 0, code_len = 0, chunk_bits = 0, chunk_esc = 0, payload = 0,
           escapes = 0;
  std::vector<uint64_t> esc_counts;
  std::vector<uint32_t> esc_bits;
  uint64_t esc_words = 0;
  uint64_t need = 0;  // bytes of header needed up to the end of the escape table
};

// returns false when more bytes are needed (need is set)
bool parse_header(const uint8_t* b, uint64_t bytes, Parsed& P) {
  if (bytes < kFixed) {
    P.need = kFixed;
    return false;
  }
  if (std::memcmp(b, "MGHP", 4) != 0) fail(MGARD_ERR_FORMAT, "bad magic");
  mgard_header& h = P.hd;
  uint16_t ver;
  std::memcpy(&ver, b + 4, 2);
  h.version = ver;
  if (ver != kVersion) fail(MGARD_ERR_FORMAT, "unsupported version");
  h.dtype = b[6];
  h.ndim = b[7];
  h.eb = b[8];
  h.alloc = b[9];
  h.coord_flags = b[10];
  h.fallback = b[11];
  if (h.dtype > 1 || h.ndim < 1 || h.ndim > 4 || h.eb > 1 || h.alloc > 2 || (h.coord_flags >> h.ndim))
    fail(MGARD_ERR_FORMAT, "bad header fields");
  std::memcpy(&h.levels, b + 12, 4);
  std::memcpy(&h.dict_size, b + 16, 4);
  std::memcpy(&h.chunk_symbols, b + 20, 4);
  std::memcpy(&h.tol, b + 24, 8);
  std::memcpy(&h.tau_abs, b + 32, 8);
  std::memcpy(&h.maxabs, b + 40, 8);
  std::memcpy(&h.n_symbols, b + 48, 8);
  std::memcpy(&h.n_chunks, b + 56, 8);
  std::memcpy(&h.n_outliers, b + 64, 8);
  std::memcpy(&h.payload_words, b + 72, 8);
  const uint32_t d = h.dict_size, c = h.chunk_symbols;
  if (d < 256 || d > 8192 || (d & (d - 1)) || c < 256 || c > 8192 || (c % 256))
    fail(MGARD_ERR_FORMAT, "bad dictionary or chunk size");
  if (h.levels > MAXL - 1) fail(MGARD_ERR_FORMAT, "bad level count");
  uint64_t p = kFixed + 8ull * h.ndim;
  if (bytes < p) {
    P.need = p;
    return false;
  }
  uint64_t n = 1;
  for (uint32_t i = 0; i < h.ndim; ++i) {
    std::memcpy(&h.shape[i], b + kFixed + 8 * i, 8);
    if (h.shape[i] == 0 || h.shape[i] > (1ull << 31)) fail(MGARD_ERR_FORMAT, "bad shape");
    n *= h.shape[i];
    if (n > (1ull << 40)) fail(MGARD_ERR_FORMAT, "bad shape");
  }
  if (n != h.n_symbols) fail(MGARD_ERR_FORMAT, "symbol count does not match shape");
  if (h.n_chunks != (n + c - 1) / c) fail(MGARD_ERR_FORMAT, "chunk count does not match");
  if (h.n_outliers > n) fail(MGARD_ERR_FORMAT, "outlier count");
  if (h.payload_words > (n * 64 + 31) / 32 + h.n_chunks) fail(MGARD_ERR_FORMAT, "payload size");
  if (b[80] > 1) fail(MGARD_ERR_FORMAT, "bad norm");
  h.norm = b[80];
  std::memcpy(&h.s, b + 88, 8);
  if (!std::isfinite(h.s)) fail(MGARD_ERR_FORMAT, "bad smoothness");
  for (uint32_t i = 0; i < h.ndim; ++i)
    if ((h.coord_flags >> i) & 1) p += 8 * h.shape[i];
  P.bins_off = p;
  p += 8ull * (h.levels + 1);
  P.lesc = p;
  p += 8ull * (h.levels + 1);
  P.lbits = p;
  p += 4ull * (h.levels + 1);
  P.need = p;
  if (bytes < p) return false;
  // escapes per level: counts that add up to n_outliers, widths of at most 64 bits
  P.esc_counts.assign(h.levels + 1, 0);
  P.esc_bits.assign(h.levels + 1, 0);
  uint64_t esc_total = 0;
  P.esc_words = 0;
  for (uint32_t l = 0; l <= h.levels; ++l) {
    std::memcpy(&P.esc_counts[l], b + P.lesc + 8 * l, 8);
    std::memcpy(&P.esc_bits[l], b + P.lbits + 4 * l, 4);
    if (P.esc_counts[l] > n || P.esc_bits[l] > 64) fail(MGARD_ERR_FORMAT, "escape table");
    esc_total += P.esc_counts[l];
    P.esc_words += (P.esc_counts[l] * P.esc_bits[l] + 31) / 32;
  }
  if (esc_total != h.n_outliers) fail(MGARD_ERR_FORMAT, "escape counts do not add up to the outlier count");
  P.coords.assign(h.ndim, {});
  uint64_t q = kFixed + 8ull * h.ndim;
  for (uint32_t i = 0; i < h.ndim; ++i)
    if ((h.coord_flags >> i) & 1) {
      P.coords[i].resize(h.shape[i]);
      std::memcpy(P.coords[i].data(), b + q, 8 * h.shape[i]);
      q += 8 * h.shape[i];
    }
  P.code_len = p;
  p += d;
  P.chunk_bits = p;
  p += 4 * h.n_chunks;
  P.chunk_esc = p;
  p += 4 * h.n_chunks;
  P.payload = p;
  p += 4 * h.payload_words;
  P.escapes = p;
  p += 4 * P.esc_words;
  h.total_bytes = p;
  return true;
}

void check_bins(const Parsed& P, const uint8_t* b) {
  for (uint32_t l = 0; l <= P.hd.levels; ++l) {
    double v;
    std::memcpy(&v, b + P.bins_off + 8 * l, 8);
    if (!(v > 0.0) || !std::isfinite(v)) fail(MGARD_ERR_FORMAT, "bad bin width");
  }
}

// Scratch bytes of one compression.
template <typename T>
uint64_t compress_scratch_bytes(const Hierarchy& h, const Opts& o, uint64_t nch) {
  const uint64_t n = h.count(h.L);
  const uint64_t dbytes = decompose_scratch_bytes<T>(h);
  uint64_t need = dbytes + carve_size<uint16_t>(n) + carve_size<int64_t>(n) +
                  carve_size<double>(MAXL + 1) + carve_size<double>(8) + carve_size<uint64_t>(4) +
                  2 * carve_size<uint64_t>((uint64_t)o.dict) + 2 * carve_size<uint64_t>(nch + 1) +
                  carve_size<Finale>(1) + encode_scratch_bytes(o.dict) + carve_size<uint64_t>(n) +
                  3 * carve_size<uint64_t>(MAXL + 2) + carve_size<char>(mass_norm_scratch_bytes()) +
                  carve_size<double>(1) + 4096;
  const int nl = h.L + 1;
  const uint64_t lbytes =
      o.alloc == MGARD_ALLOC_LEARNED
          ? 2 * carve_size<T>(n) + carve_size<uint64_t>(MAXL + 2) + carve_size<double>((uint64_t)2 * nl * STATS_BLOCKS) +
                carve_size<double>(3 * (MAXL + 1)) + carve_size<float>((uint64_t)MLP_IN * (MAXL + 1)) +
                carve_size<float>(MAXL + 1) + carve_size<float>((uint64_t)2 * MLP_HID * (MAXL + 1)) +
                carve_size<double>(MAXL + 1) + carve_size<unsigned long long>(1) + 1024
          : 0;
  return need + lbytes;
}

constexpr int kLearnedAttempts = 2;  // learned widths tried before the plain ones

// Every device step of one compression, enqueued on o.st with no host
// synchronisation, host-memory copy or memset, so that it can be captured in
// a graph (the learned allocation, which batches do not use, reads back the
// bound check's result between its attempts).  The static header is copied from `header` (device memory); the
// results land in *fin_out (device) and, when size_out is given, the total
// size in *size_out (device).
// The buffers of one compression inside its scratch (the same carving for
// every phase of compress_enqueue).
struct CompressBufs {
  void* dscratch;
  void* learned_scratch;
  uint16_t* sym;
  int64_t* qside;
  double* bins;
  double* scalars;
  uint64_t* misc;  // [0] max bits, [2] status
  uint64_t* hist;
  uint64_t* codes;
  uint64_t* word_off;
  uint64_t* esc_off;
  Finale* fin;
  void* enc_scratch;
  uint64_t* ecodes;                // escape codes, compact (n entries at most)
  uint64_t* esc_start;             // per level: first escape index (L + 2)
  unsigned long long* esc_wmax;    // per level: largest code (L + 1)
  uint64_t* esc_woff;              // per level: first escape word (L + 2)
  void* norm_scratch;              // the L2 norm's block partials (s-norm, relative)
  double* nrm2;                    // u^T M u
};

template <typename T>
CompressBufs carve_compress(const Hierarchy& h, const Layout& y, const Opts& o, void* scratch) {
  const uint64_t n = h.count(h.L);
  const uint64_t nch = y.nch;
  const uint64_t dbytes = decompose_scratch_bytes<T>(h);
  const int nl = h.L + 1;
  const uint64_t lbytes =
      o.alloc == MGARD_ALLOC_LEARNED
          ? 2 * carve_size<T>(n) + carve_size<uint64_t>(MAXL + 2) + carve_size<double>((uint64_t)2 * nl * STATS_BLOCKS) +
                carve_size<double>(3 * (MAXL + 1)) + carve_size<float>((uint64_t)MLP_IN * (MAXL + 1)) +
                carve_size<float>(MAXL + 1) + carve_size<float>((uint64_t)2 * MLP_HID * (MAXL + 1)) +
                carve_size<double>(MAXL + 1) + carve_size<unsigned long long>(1) + 1024
          : 0;
  Carver cv(scratch);
  CompressBufs b;
  b.dscratch = cv.take<char>(dbytes);
  b.learned_scratch = lbytes ? cv.take<char>(lbytes) : nullptr;
  b.sym = cv.take<uint16_t>(n);
  b.qside = cv.take<int64_t>(n);
  b.bins = cv.take<double>(MAXL + 1);
  b.scalars = cv.take<double>(8);
  b.misc = cv.take<uint64_t>(4);
  b.hist = cv.take<uint64_t>((uint64_t)o.dict);
  b.codes = cv.take<uint64_t>((uint64_t)o.dict);
  b.word_off = cv.take<uint64_t>(nch + 1);
  b.esc_off = cv.take<uint64_t>(nch + 1);
  b.fin = cv.take<Finale>(1);
  b.enc_scratch = cv.take<char>(encode_scratch_bytes(o.dict));
  b.ecodes = cv.take<uint64_t>(n);
  b.esc_start = cv.take<uint64_t>(MAXL + 2);
  b.esc_wmax = cv.take<unsigned long long>(MAXL + 2);
  b.esc_woff = cv.take<uint64_t>(MAXL + 2);
  b.norm_scratch = cv.take<char>(mass_norm_scratch_bytes());
  b.nrm2 = cv.take<double>(1);
  return b;
}

// Phases: CE_ALL runs the whole compression; CE_FRONT stops after the
// histogram and CE_BACK runs from the chunk bit counts on, so a batch can
// build the codebooks of all its fields in one launch in between.
enum { CE_ALL = 0, CE_FRONT = 1, CE_BACK = 2 };

template <typename T>
Finale* compress_enqueue(Hierarchy& h, const T* table, const Layout& y, double tol, const T* d_in, char* d_out,
                         const Opts& o, void* scratch, const uint8_t* header, uint64_t header_bytes,
                         uint64_t* size_out, int phase = CE_ALL) {
  const bool f64 = sizeof(T) == 8;
  hipStream_t st = o.st;
  const uint64_t n = h.count(h.L);
  const uint64_t nch = y.nch;
  const CompressBufs cb = carve_compress<T>(h, y, o, scratch);
  void* dscratch = cb.dscratch;
  void* learned_scratch = cb.learned_scratch;
  uint16_t* sym = cb.sym;
  int64_t* qside = cb.qside;
  double* bins = cb.bins;
  double* scalars = cb.scalars;
  uint64_t* misc = cb.misc;
  uint64_t* hist = cb.hist;
  uint64_t* codes = cb.codes;
  uint64_t* word_off = cb.word_off;
  uint64_t* esc_off = cb.esc_off;
  Finale* fin = cb.fin;
  void* enc_scratch = cb.enc_scratch;
  uint32_t* chunk_esc = reinterpret_cast<uint32_t*>(d_out + y.chunk_esc);
  uint32_t* chunk_bits = reinterpret_cast<uint32_t*>(d_out + y.chunk_bits);
  uint8_t* code_len = reinterpret_cast<uint8_t*>(d_out + y.code_len);
  if (phase != CE_BACK) {
  copy_d2d(d_out, header, header_bytes, st);
  launch_fill_u64(&misc[2], 1, 0, st);

  // tolerance and bin widths
  launch_maxabs<T>(d_in, n, &misc[0], st);
  BinArgs ba{};
  for (int l = 0; l <= h.L; ++l) {
    ba.K[l] = h.K[l];
    ba.counts[l] = (double)h.level_count[l];
  }
  const int alloc = o.alloc == MGARD_ALLOC_COUNT ? MGARD_ALLOC_COUNT : MGARD_ALLOC_PLAIN;
  if (o.norm == MGARD_NORM_S) {
    // the s-norm widths: ||u|| (relative bound) on the device, factors from the host
    if (o.eb == MGARD_REL)
      launch_mass_norm<T>(h, device_mass_table(h, st), d_in, cb.norm_scratch, cb.nrm2, st);
    launch_bins_snorm(f64 ? 1 : 0, &misc[0], cb.nrm2, tol, o.eb, h.L, snorm_args(h, o.s), bins, scalars, st);
  } else {
    launch_bins(f64 ? 1 : 0, &misc[0], tol, o.eb, h.S, h.L, alloc, ba, bins, scalars, st);
  }

  QuantOut q;
  q.sym = sym;
  q.qside = qside;
  q.bins = bins;
  q.R = o.dict / 2;
  const int nlev = h.L + 1;
  if (o.alloc == MGARD_ALLOC_LEARNED) {
    // float coefficients -> level statistics -> network -> bin widths; the
    // recomposed result is checked on the device and the plain widths are
    // kept when the L-infinity error exceeds tau
    Carver lv(learned_scratch);
    T* cstream = lv.take<T>(n);
    T* recon = lv.take<T>(n);
    uint64_t* d_off = lv.take<uint64_t>(MAXL + 2);
    double* part = lv.take<double>((uint64_t)2 * nlev * STATS_BLOCKS);
    double* stats = lv.take<double>(3 * (MAXL + 1));
    float* x = lv.take<float>((uint64_t)MLP_IN * (MAXL + 1));
    float* theta = lv.take<float>(MAXL + 1);
    float* tmp = lv.take<float>((uint64_t)2 * MLP_HID * (MAXL + 1));
    double* learned = lv.take<double>(MAXL + 1);
    unsigned long long* err = lv.take<unsigned long long>(1);
    MG_HIP(hipMemcpyAsync(d_off, h.level_off.data(), 8 * (h.L + 2), hipMemcpyHostToDevice, st));
    decompose<T>(h, table, d_in, cstream, nullptr, dscratch, st);
    launch_level_stats<T>(cstream, d_off, nlev, part, stats, st);
    launch_features(stats, scalars, nlev, o.model_params, x, st);
    mlp_forward(o.model_params, x, nlev, theta, nullptr, tmp, st);
    // the bound check: widths b * exp(s * theta) for s = 1, then 1/2; the first
    // whose recomposition meets tau is kept, else the plain widths
    for (int attempt = 0; attempt < kLearnedAttempts; ++attempt) {
      launch_apply_theta(bins, theta, nlev, std::ldexp(1.0, -attempt), learned, st);
      launch_quantize<T>(cstream, n, d_off, nlev, learned, q.R, sym, qside, st);
      QuantOut ql = q;
      ql.bins = learned;
      recompose<T>(h, table, nullptr, &ql, recon, dscratch, st);
      launch_linf<T>(recon, d_in, n, err, st);
      if (attempt + 1 < kLearnedAttempts) {
        double ht[2];
        unsigned long long he = 0;
        MG_HIP(hipMemcpyAsync(&he, err, 8, hipMemcpyDeviceToHost, st));
        MG_HIP(hipMemcpyAsync(ht, scalars, 16, hipMemcpyDeviceToHost, st));
        MG_HIP(hipStreamSynchronize(st));
        double e;
        std::memcpy(&e, &he, 8);
        if (e <= ht[0]) break;
      }
    }
    launch_select_bins(err, scalars, bins, learned, nlev, st);
    launch_quantize<T>(cstream, n, d_off, nlev, bins, q.R, sym, qside, st);
  } else if (phase == CE_ALL) {
    // decomposition with fused quantization; the chunks that lie wholly in
    // the finest level are counted on a side stream as soon as that level's
    // symbols are written, while the coarser levels decompose
    const uint64_t k1 = std::min<uint64_t>((h.level_off[h.L] + o.chunk - 1) / o.chunk, nch);
    launch_fill_u64(hist, (uint64_t)o.dict, 0, st);
    SideStream side;
    const std::function<void()> fine_written = [&] {
      side.fork(st);
      launch_histogram_chunks(sym, n, o.dict, o.chunk, k1, nch, hist, chunk_esc,
                              reinterpret_cast<uint32_t*>(&misc[2]), side.s);
      side.record_join();
    };
    decompose<T>(h, table, d_in, nullptr, &q, dscratch, st, &fine_written);
    launch_histogram_chunks(sym, n, o.dict, o.chunk, 0, k1, hist, chunk_esc, reinterpret_cast<uint32_t*>(&misc[2]),
                            st);
    side.join(st);
  } else {
    // a recording batch aligns the fields' decompositions (of different
    // lengths) separately from the stages before and after them
    if (Recorder* r = recorder()) r->phase = 1;
    decompose<T>(h, table, d_in, nullptr, &q, dscratch, st);
    if (Recorder* r = recorder()) r->phase = 2;
  }

  // lossless stage, tables written in place
  if (o.alloc == MGARD_ALLOC_LEARNED || phase != CE_ALL)
    launch_histogram(sym, n, o.dict, o.chunk, hist, chunk_esc, reinterpret_cast<uint32_t*>(&misc[2]), st);
  if (phase == CE_FRONT) return fin;
  launch_codebook(hist, o.dict, code_len, codes, enc_scratch, st);
  }
  launch_chunk_bits(sym, n, o.dict, o.chunk, code_len, chunk_bits, st);
  launch_scan_pair(chunk_bits, chunk_esc, nch, word_off, esc_off, st);
  launch_encode(sym, n, o.dict, o.chunk, code_len, codes, word_off, reinterpret_cast<uint32_t*>(d_out + y.payload),
                esc_off, qside, cb.ecodes, enc_scratch, true, st);
  LevelTable lt{};
  for (int l = 0; l <= h.L + 1; ++l) lt.off[l] = h.level_off[l];
  launch_escape_pack(sym, n, o.chunk, esc_off, word_off, nch, cb.ecodes, h.L + 1, lt, d_out, y.payload,
                     reinterpret_cast<uint64_t*>(d_out + y.lesc), reinterpret_cast<uint32_t*>(d_out + y.lbits),
                     cb.esc_start, cb.esc_wmax, cb.esc_woff, st);
  MG_LAUNCH((&k_finalize), (k_finalize_k), (1), (0), (dim3(1)), st, d_out, word_off, esc_off, nch, y.payload, cb.esc_woff + (h.L + 1), scalars, bins, h.L, y.bins, o.alloc == MGARD_ALLOC_LEARNED ? 1 : 0, fin, size_out);
  MG_HIP(hipGetLastError());
  return fin;
}

template <typename T>
void compress_impl(Hierarchy& h, const double* const* coords, double tol, const T* d_in, char* d_out,
                   uint64_t* out_bytes, const Opts& o, mgard_info* info) {
  const bool f64 = sizeof(T) == 8;
  hipStream_t st = o.st;
  const T* table = static_cast<const T*>(device_table(h, f64, st));
  const uint64_t n = h.count(h.L);
  const Layout y = layout(h, coords, o.dict, o.chunk, n);
  std::vector<uint8_t> hb =
      header_bytes(h, coords, f64 ? 1 : 0, o.eb, o.alloc, tol, o.dict, o.chunk, n, y.nch, o.norm, o.s);
  const uint64_t need = compress_scratch_bytes<T>(h, o, y.nch);
  Workspace& ws = workspace();
  ws.reserve(need + carve_size<uint8_t>(hb.size()));
  Carver cv(ws.base());
  void* scratch = cv.take<char>(need);
  uint8_t* d_hdr = cv.take<uint8_t>(hb.size());
  // pinned staging: the header goes up and the sizes come back without a
  // pageable bounce copy
  const size_t fin_at = (hb.size() + 255) & ~size_t(255);
  uint8_t* stage = pinned_staging(fin_at + sizeof(Finale));
  std::memcpy(stage, hb.data(), hb.size());
  MG_HIP(hipMemcpyAsync(d_hdr, stage, hb.size(), hipMemcpyHostToDevice, st));
  Finale* fin = compress_enqueue<T>(h, table, y, tol, d_in, d_out, o, scratch, d_hdr, hb.size(), nullptr);
  Finale hf;
  MG_HIP(hipMemcpyAsync(stage + fin_at, fin, sizeof(Finale), hipMemcpyDeviceToHost, st));
  MG_HIP(hipStreamSynchronize(st));
  std::memcpy(&hf, stage + fin_at, sizeof(Finale));
  if (hf.scalars[2] != 0.0) fail(MGARD_ERR_NONFINITE, "input holds NaN or infinity");
  if (hf.scalars[6] != 0.0) fail(MGARD_ERR_TOL, "tolerance below the rounding reserve or the quantizer's range");
  *out_bytes = hf.total_bytes;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->tol = tol;
    info->tau_abs = hf.scalars[0];
    info->maxabs = hf.scalars[1];
    for (int l = 0; l <= h.L; ++l) info->bin_width[l] = hf.bins[l];
    info->linf_err = hf.scalars[4];
    info->n_symbols = n;
    info->n_outliers = hf.n_outliers;
    info->payload_words = hf.payload_words;
    info->out_bytes = hf.total_bytes;
    info->levels = (uint32_t)h.L;
    info->fallback_used = hf.scalars[5] != 0.0 ? 1u : 0u;
  }
}

// ext_status (device, 4 words), when given, receives the decode status and
// the call returns without waiting; the caller reads it after its stream.
template <typename T>
void decompress_impl(Hierarchy& h, const Parsed& P, const char* d_in, T* d_out, const Opts& o,
                     uint32_t* ext_status = nullptr) {
  const bool f64 = sizeof(T) == 8;
  hipStream_t st = o.st;
  const T* table = static_cast<const T*>(device_table(h, f64, st));
  const uint64_t n = P.hd.n_symbols, nch = P.hd.n_chunks;
  const int dict = (int)P.hd.dict_size, chunk = (int)P.hd.chunk_symbols;
  const uint64_t rbytes = recompose_scratch_bytes<T>(h);
  const uint64_t n_out = P.hd.n_outliers;
  if ((int)P.esc_counts.size() != h.L + 1 || h.L + 1 > MAXL + 1) fail(MGARD_ERR_FORMAT, "level count");
  EscLevels et{};
  et.nlev = h.L + 1;
  for (int l = 0; l <= h.L; ++l) {
    et.ostart[l + 1] = et.ostart[l] + P.esc_counts[l];
    et.woff[l + 1] = et.woff[l] + (P.esc_counts[l] * P.esc_bits[l] + 31) / 32;
    et.bits[l] = P.esc_bits[l];
  }
  for (int l = 0; l <= h.L + 1; ++l) et.loff[l] = h.level_off[l];
  uint64_t need = rbytes + carve_size<uint16_t>(n) + carve_size<int64_t>(n) + 2 * carve_size<uint64_t>(nch + 1) +
                  carve_size<uint64_t>(n_out) + decode_table_bytes(dict) + carve_size<uint32_t>(4) + 4096;
  Workspace& ws = workspace();
  ws.reserve(need);
  Carver cv(ws.base());
  void* rscratch = cv.take<char>(rbytes);
  uint16_t* sym = cv.take<uint16_t>(n);
  int64_t* qside = cv.take<int64_t>(n);
  uint64_t* word_off = cv.take<uint64_t>(nch + 1);
  uint64_t* esc_off = cv.take<uint64_t>(nch + 1);
  uint64_t* epos = cv.take<uint64_t>(n_out);
  void* tabs = cv.take<char>(decode_table_bytes(dict));
  uint32_t* status = cv.take<uint32_t>(4);
  if (ext_status) status = ext_status;
  MG_HIP(hipMemsetAsync(status, 0, 16, st));
  const uint32_t* chunk_bits = reinterpret_cast<const uint32_t*>(d_in + P.chunk_bits);
  const uint32_t* chunk_esc = reinterpret_cast<const uint32_t*>(d_in + P.chunk_esc);
  launch_scan_pair(chunk_bits, chunk_esc, nch, word_off, esc_off, st);
  launch_decode_full(reinterpret_cast<const uint32_t*>(d_in + P.payload), P.hd.payload_words, word_off,
                     chunk_bits, n, dict, chunk, reinterpret_cast<const uint8_t*>(d_in + P.code_len), sym,
                     esc_off, n_out, epos, tabs, status, st);
  launch_escape_scatter(epos, reinterpret_cast<const uint32_t*>(d_in + P.escapes), P.esc_words, et, dict / 2, n,
                        qside, status, st);
  QuantOut q;
  q.sym = sym;
  q.qside = qside;
  q.bins = reinterpret_cast<const double*>(d_in + P.bins_off);
  q.R = dict / 2;
  recompose<T>(h, table, nullptr, &q, d_out, rscratch, st);
  if (ext_status) return;
  uint8_t* stage = pinned_staging(16);
  MG_HIP(hipMemcpyAsync(stage, status, 16, hipMemcpyDeviceToHost, st));
  MG_HIP(hipStreamSynchronize(st));
  uint32_t hs[4];
  std::memcpy(hs, stage, 16);
  if (hs[0]) fail(MGARD_ERR_FORMAT, "payload does not decode");
}

// Plain widths for tol 1e-3 (relative) of d_in and the quantized level
// buffers, then the timing of every fused 3D level's launch candidates.
template <typename T>
void autotune_impl(Hierarchy& h, const T* d_in, const Opts& o) {
  if (!fused3d_ok<T>(h) || h.L < 1) return;
  const bool f64 = sizeof(T) == 8;
  hipStream_t st = o.st;
  const T* table = static_cast<const T*>(device_table(h, f64, st));
  const uint64_t n = h.count(h.L);
  const uint64_t dbytes = decompose_scratch_bytes<T>(h);
  Workspace& ws = workspace();
  ws.reserve(dbytes + carve_size<uint16_t>(n) + carve_size<int64_t>(n) + carve_size<double>(MAXL + 1) +
             carve_size<double>(8) + carve_size<uint64_t>(4) + 1024);
  Carver cv(ws.base());
  void* dscratch = cv.take<char>(dbytes);
  uint16_t* sym = cv.take<uint16_t>(n);
  int64_t* qside = cv.take<int64_t>(n);
  double* bins = cv.take<double>(MAXL + 1);
  double* scalars = cv.take<double>(8);
  uint64_t* misc = cv.take<uint64_t>(4);
  launch_maxabs<T>(d_in, n, &misc[0], st);
  BinArgs ba{};
  for (int l = 0; l <= h.L; ++l) {
    ba.K[l] = h.K[l];
    ba.counts[l] = (double)h.level_count[l];
  }
  launch_bins(f64 ? 1 : 0, &misc[0], 1e-3, MGARD_REL, h.S, h.L, MGARD_ALLOC_PLAIN, ba, bins, scalars, st);
  QuantOut q;
  q.sym = sym;
  q.qside = qside;
  q.bins = bins;
  q.R = o.dict / 2;
  fused3d_tune<T>(h, table, d_in, &q, dscratch, st);
  MG_HIP(hipStreamSynchronize(st));
}

bool tuned_all_levels(const Hierarchy& h, bool f64) {
  for (int l = 1; l <= h.L; ++l) {
    const int n0 = (int)h.sizes[l][1], n1 = (int)h.sizes[l][2], n2 = (int)h.sizes[l][3];
    if (!tune_known(TUNE_COEFF_SEG, f64, n0, n1, n2) || !tune_known(TUNE_SCATTER_PLANES, f64, n0, n1, n2))
      return false;
  }
  return true;
}

uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

const double* const* field_coords(const mgard_field& f) {
  for (uint32_t d = 0; d < f.ndim && d < 4; ++d)
    if (f.coords[d]) return f.coords;
  return nullptr;
}

struct BatchJob {
  std::shared_ptr<Hierarchy> h;
  Layout y;
  std::vector<uint8_t> hb;
  const void* table = nullptr;
  bool f64 = false;
  uint64_t scratch = 0, hdr_off = 0, scr_off = 0, out_off = 0, bound = 0;
};

std::vector<BatchJob> plan_jobs(uint32_t nfields, const mgard_field* fields, double tol, const Opts& o,
                                bool with_tables, uint64_t* out_total, uint64_t* mem_total) {
  std::vector<BatchJob> jobs(nfields);
  uint64_t out_off = 0, mem = 0;
  for (uint32_t i = 0; i < nfields; ++i) {
    const mgard_field& f = fields[i];
    if (f.dtype != MGARD_F32 && f.dtype != MGARD_F64) fail(MGARD_ERR_DTYPE, "field dtype");
    BatchJob& J = jobs[i];
    const double* const* cc = field_coords(f);
    J.h = get_hierarchy(f.ndim, f.shape, cc);
    J.f64 = f.dtype == MGARD_F64;
    if (with_tables) J.table = device_table(*J.h, J.f64, o.st);
    const uint64_t n = J.h->count(J.h->L);
    J.y = layout(*J.h, cc, o.dict, o.chunk, n);
    J.hb = header_bytes(*J.h, cc, J.f64 ? 1 : 0, o.eb, o.alloc, tol, o.dict, o.chunk, n, J.y.nch);
    J.bound = bound_of(*J.h, cc, o.dict, o.chunk);
    J.out_off = out_off;
    out_off = align256(out_off + J.bound);
    J.scratch = J.f64 ? compress_scratch_bytes<double>(*J.h, o, J.y.nch) : compress_scratch_bytes<float>(*J.h, o, J.y.nch);
    J.hdr_off = mem;
    mem += align256(J.hb.size());
    J.scr_off = mem;
    mem += align256(J.scratch);
  }
  *out_total = out_off;
  *mem_total = mem;
  return jobs;
}

struct CoordPtrs {
  const double* p[MAXD] = {nullptr, nullptr, nullptr, nullptr};
};

// ------------------------------------------------------------------ out-of-core
// A host-resident array in slabs along dimension 0, each compressed as a field
// of its own at the absolute tolerance of the whole array, behind a container
// header (layout in include/mgard_hip.h).  Slab k + 1 is copied to the device
// while slab k is compressed and slab k - 1 copied back, on three streams:
// copies in (cs), compute (the caller's stream), copies out (ds).
constexpr uint32_t kChunkMagic = 0x4B43474Du;  // "MGCK"
constexpr uint64_t kChunkFixed = 88;

struct Slabs {
  std::vector<uint64_t> p0, p1;
  uint64_t size() const { return p0.size(); }
};

Slabs slab_plan(uint64_t n0, uint64_t slab) {
  if (slab < 3) fail(MGARD_ERR_ARG, "slab_planes must be at least 3");
  Slabs s;
  for (uint64_t p = 0; p < n0; p += slab) {
    s.p0.push_back(p);
    s.p1.push_back(std::min(p + slab, n0));
  }
  // a last slab of fewer than 3 planes joins the one before it
  if (s.size() > 1 && s.p1.back() - s.p0.back() < 3) {
    s.p1[s.size() - 2] = n0;
    s.p0.pop_back();
    s.p1.pop_back();
  }
  return s;
}

// The streams, events and double buffers of one chunked call; everything
// queued is finished before any of it is released.
struct Pipeline {
  hipStream_t cs = nullptr, ds = nullptr, ks = nullptr;
  hipEvent_t in_done[2] = {nullptr, nullptr}, out_done[2] = {nullptr, nullptr}, used[2] = {nullptr, nullptr};
  void* a[2] = {nullptr, nullptr};  // device copies of slabs (or of slab streams)
  void* b[2] = {nullptr, nullptr};  // device results
  uint64_t* bits = nullptr;
  std::vector<void*> keep;  // slabs kept on the device from the first pass to the second
  explicit Pipeline(hipStream_t st) : ks(st) {
    MG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    MG_HIP(hipStreamCreateWithFlags(&ds, hipStreamNonBlocking));
    for (int i = 0; i < 2; ++i) {
      MG_HIP(hipEventCreateWithFlags(&in_done[i], hipEventDisableTiming));
      MG_HIP(hipEventCreateWithFlags(&out_done[i], hipEventDisableTiming));
      MG_HIP(hipEventCreateWithFlags(&used[i], hipEventDisableTiming));
    }
  }
  void alloc(uint64_t a_bytes, uint64_t b_bytes, uint64_t nbits) {
    for (int i = 0; i < 2; ++i) {
      if (hipMalloc(&a[i], std::max<uint64_t>(a_bytes, 256)) != hipSuccess ||
          hipMalloc(&b[i], std::max<uint64_t>(b_bytes, 256)) != hipSuccess) {
        (void)hipGetLastError();
        fail(MGARD_ERR_OOM, "slab buffers");
      }
    }
    if (hipMalloc(&bits, 8 * std::max<uint64_t>(nbits, 1)) != hipSuccess) {
      (void)hipGetLastError();
      fail(MGARD_ERR_OOM, "slab maxima");
    }
  }
  ~Pipeline() {
    if (ks) (void)hipStreamSynchronize(ks);
    if (cs) (void)hipStreamSynchronize(cs);
    if (ds) (void)hipStreamSynchronize(ds);
    for (int i = 0; i < 2; ++i) {
      if (a[i]) (void)hipFree(a[i]);
      if (b[i]) (void)hipFree(b[i]);
      if (in_done[i]) (void)hipEventDestroy(in_done[i]);
      if (out_done[i]) (void)hipEventDestroy(out_done[i]);
      if (used[i]) (void)hipEventDestroy(used[i]);
    }
    if (bits) (void)hipFree(bits);
    for (void* p : keep) (void)hipFree(p);
    if (cs) (void)hipStreamDestroy(cs);
    if (ds) (void)hipStreamDestroy(ds);
  }
};

// Per-slab coordinates: dimension 0 starts at the slab's first plane.
CoordPtrs slab_coords(uint32_t ndim, const double* const* coords, uint64_t p0) {
  CoordPtrs c;
  if (coords)
    for (uint32_t d = 0; d < ndim; ++d) c.p[d] = coords[d] ? coords[d] + (d == 0 ? p0 : 0) : nullptr;
  return c;
}

uint64_t chunked_bound(uint32_t ndim, const uint64_t* shape, const double* const* coords, uint64_t slab,
                       const Opts& o) {
  const Slabs sp = slab_plan(shape[0], slab);
  uint64_t total = kChunkFixed + 8 * (sp.size() + 1);
  std::array<uint64_t, MAXD> cs{};
  for (uint32_t d = 0; d < ndim; ++d) cs[d] = shape[d];
  for (uint64_t k = 0; k < sp.size(); ++k) {
    cs[0] = sp.p1[k] - sp.p0[k];
    const CoordPtrs cc = slab_coords(ndim, coords, sp.p0[k]);
    total += bound_of(*get_hierarchy(ndim, cs.data(), coords ? cc.p : nullptr), coords ? cc.p : nullptr, o.dict,
                      o.chunk);
  }
  return total;
}

template <typename T>
void compress_chunked_impl(uint32_t ndim, const uint64_t* shape, const double* const* coords, double tol,
                           const T* h_in, uint64_t slab, char* h_out, uint64_t cap, uint64_t* out_bytes,
                           const Opts& o0) {
  const Slabs sp = slab_plan(shape[0], slab);
  const uint64_t ns = sp.size();
  uint64_t plane = 1;
  for (uint32_t d = 1; d < ndim; ++d) plane *= shape[d];
  const uint64_t head = kChunkFixed + 8 * (ns + 1);
  if (cap < head) fail(MGARD_ERR_CAPACITY, "output capacity below the container header");
  std::vector<std::shared_ptr<Hierarchy>> hs(ns);
  std::vector<CoordPtrs> cps(ns);
  std::array<uint64_t, MAXD> cshape{};
  for (uint32_t d = 0; d < ndim; ++d) cshape[d] = shape[d];
  uint64_t max_in = 0, max_bound = 0;
  for (uint64_t k = 0; k < ns; ++k) {
    cshape[0] = sp.p1[k] - sp.p0[k];
    cps[k] = slab_coords(ndim, coords, sp.p0[k]);
    hs[k] = get_hierarchy(ndim, cshape.data(), coords ? cps[k].p : nullptr);
    max_in = std::max(max_in, cshape[0] * plane * sizeof(T));
    max_bound = std::max(max_bound, bound_of(*hs[k], coords ? cps[k].p : nullptr, o0.dict, o0.chunk));
  }
  Pipeline pl(o0.st);
  pl.alloc(max_in, max_bound, ns);
  // With a relative tolerance every slab is read twice.  The first slabs stay
  // on the device between the passes, as many as half of the free device
  // memory holds after this call's other buffers and one slab's scratch, so
  // only the rest cross the host link a second time.
  uint64_t nkeep = 0;
  if (o0.eb == MGARD_REL) {
    size_t freeb = 0, totalb = 0;
    MG_HIP(hipMemGetInfo(&freeb, &totalb));
    const uint64_t other = 4 * max_in + 2 * max_bound;  // one slab's scratch is a few slabs
    const uint64_t budget = freeb / 2 > other ? freeb / 2 - other : 0;
    nkeep = std::min<uint64_t>(ns, max_in ? budget / max_in : 0);
    // MGARD_CHUNKED_KEEP caps the count (a test covers the mixed path with it)
    if (const char* e = std::getenv("MGARD_CHUNKED_KEEP")) nkeep = std::min<uint64_t>(nkeep, std::strtoull(e, nullptr, 10));
    for (uint64_t k = 0; k < nkeep; ++k) {
      void* p = nullptr;
      if (hipMalloc(&p, std::max<uint64_t>(max_in, 256)) != hipSuccess) {
        (void)hipGetLastError();
        nkeep = k;
        break;
      }
      pl.keep.push_back(p);
    }
  }
  auto slab_dev = [&](uint64_t k) -> void* { return k < nkeep ? pl.keep[k] : pl.a[k & 1]; };
  auto copy_in = [&](uint64_t k) {
    const int s = (int)(k & 1);
    MG_HIP(hipMemcpyAsync(slab_dev(k), h_in + sp.p0[k] * plane, (sp.p1[k] - sp.p0[k]) * plane * sizeof(T),
                          hipMemcpyHostToDevice, pl.cs));
    MG_HIP(hipEventRecord(pl.in_done[s], pl.cs));
  };
  // pass 1, relative tolerance only: max |u| of every slab
  double tau = tol;
  if (o0.eb == MGARD_REL) {
    for (uint64_t k = 0; k < ns; ++k) {
      const int s = (int)(k & 1);
      if (k >= 2) MG_HIP(hipStreamWaitEvent(pl.cs, pl.used[s], 0));  // slab k - 2 is read
      copy_in(k);
      MG_HIP(hipStreamWaitEvent(pl.ks, pl.in_done[s], 0));
      launch_maxabs<T>(static_cast<const T*>(slab_dev(k)), (sp.p1[k] - sp.p0[k]) * plane, pl.bits + k, pl.ks);
      MG_HIP(hipEventRecord(pl.used[s], pl.ks));
    }
    std::vector<uint64_t> hb(ns);
    MG_HIP(hipMemcpyAsync(hb.data(), pl.bits, 8 * ns, hipMemcpyDeviceToHost, pl.ks));
    MG_HIP(hipStreamSynchronize(pl.ks));
    MG_HIP(hipStreamSynchronize(pl.cs));
    uint64_t mb = 0;
    for (uint64_t v : hb) mb = std::max(mb, v);
    double maxabs;
    if (sizeof(T) == 8) {
      if (mb >= 0x7ff0000000000000ull) fail(MGARD_ERR_NONFINITE, "input holds NaN or infinity");
      std::memcpy(&maxabs, &mb, 8);
    } else {
      if (mb >= 0x7f800000ull) fail(MGARD_ERR_NONFINITE, "input holds NaN or infinity");
      const uint32_t b32 = (uint32_t)mb;
      float f;
      std::memcpy(&f, &b32, 4);
      maxabs = (double)f;
    }
    tau = tol * maxabs;
    if (!(tau > 0.0)) fail(MGARD_ERR_TOL, "relative tolerance of an all-zero array");
  }
  // pass 2: slab k + 1 in while slab k is compressed and slab k - 1 copied out
  Opts o = o0;
  o.eb = MGARD_ABS;
  o.st = pl.ks;
  std::vector<uint64_t> offs{head};
  if (nkeep == 0) copy_in(0);
  for (uint64_t k = 0; k < ns; ++k) {
    const int s = (int)(k & 1);
    // a[s ^ 1] was last read by an earlier slab, whose compression has returned
    if (k + 1 < ns && k + 1 >= nkeep) copy_in(k + 1);
    if (k >= nkeep) MG_HIP(hipStreamWaitEvent(pl.ks, pl.in_done[s], 0));
    if (k >= 2) MG_HIP(hipStreamWaitEvent(pl.ks, pl.out_done[s], 0));  // b[s] copied out
    uint64_t nb = 0;
    compress_impl<T>(*hs[k], coords ? cps[k].p : nullptr, tau, static_cast<const T*>(slab_dev(k)),
                     static_cast<char*>(pl.b[s]), &nb, o, nullptr);
    if (offs.back() + nb > cap) {
      *out_bytes = chunked_bound(ndim, shape, coords, slab, o0);
      fail(MGARD_ERR_CAPACITY, "output capacity below mgard_chunked_bound");
    }
    MG_HIP(hipMemcpyAsync(h_out + offs.back(), pl.b[s], nb, hipMemcpyDeviceToHost, pl.ds));
    MG_HIP(hipEventRecord(pl.out_done[s], pl.ds));
    offs.push_back(offs.back() + nb);
  }
  MG_HIP(hipStreamSynchronize(pl.ds));
  // the container header
  uint8_t hb[kChunkFixed];
  std::memset(hb, 0, sizeof(hb));
  auto put32 = [&](uint64_t at, uint32_t v) { std::memcpy(hb + at, &v, 4); };
  auto put64 = [&](uint64_t at, uint64_t v) { std::memcpy(hb + at, &v, 8); };
  put32(0, kChunkMagic);
  put32(4, 1);
  put32(8, ndim);
  put32(12, sizeof(T) == 8 ? 1 : 0);
  for (uint32_t d = 0; d < ndim; ++d) put64(16 + 8 * d, shape[d]);
  put64(48, slab);
  put64(56, ns);
  std::memcpy(hb + 64, &tol, 8);
  put32(72, (uint32_t)o0.eb);
  std::memcpy(hb + 80, &tau, 8);
  std::memcpy(h_out, hb, kChunkFixed);
  std::memcpy(h_out + kChunkFixed, offs.data(), 8 * (ns + 1));
  *out_bytes = offs.back();
}

struct ChunkHead {
  uint32_t ndim = 0, dtype = 0;
  uint64_t shape[MAXD] = {0, 0, 0, 0};
  uint64_t slab = 0, ns = 0;
  std::vector<uint64_t> offs;
};

ChunkHead parse_chunked(const uint8_t* b, uint64_t bytes) {
  ChunkHead c;
  if (bytes < kChunkFixed) fail(MGARD_ERR_FORMAT, "buffer shorter than a container header");
  uint32_t magic, ver;
  std::memcpy(&magic, b, 4);
  std::memcpy(&ver, b + 4, 4);
  if (magic != kChunkMagic || ver != 1) fail(MGARD_ERR_FORMAT, "not a chunked container");
  std::memcpy(&c.ndim, b + 8, 4);
  std::memcpy(&c.dtype, b + 12, 4);
  if (c.ndim < 1 || c.ndim > MAXD || c.dtype > 1) fail(MGARD_ERR_FORMAT, "container shape or dtype");
  std::memcpy(c.shape, b + 16, 32);
  std::memcpy(&c.slab, b + 48, 8);
  std::memcpy(&c.ns, b + 56, 8);
  const Slabs sp = slab_plan(c.shape[0], c.slab);
  if (sp.size() != c.ns || bytes < kChunkFixed + 8 * (c.ns + 1)) fail(MGARD_ERR_FORMAT, "container slab table");
  c.offs.resize(c.ns + 1);
  std::memcpy(c.offs.data(), b + kChunkFixed, 8 * (c.ns + 1));
  if (c.offs[0] != kChunkFixed + 8 * (c.ns + 1) || c.offs.back() > bytes) fail(MGARD_ERR_FORMAT, "container offsets");
  for (uint64_t k = 0; k < c.ns; ++k)
    if (c.offs[k + 1] < c.offs[k]) fail(MGARD_ERR_FORMAT, "container offsets");
  return c;
}

template <typename T>
void decompress_chunked_impl(const ChunkHead& c, const uint8_t* h_in, T* h_out, const Opts& o0) {
  const Slabs sp = slab_plan(c.shape[0], c.slab);
  const uint64_t ns = sp.size();
  uint64_t plane = 1;
  for (uint32_t d = 1; d < c.ndim; ++d) plane *= c.shape[d];
  // every slab's header, read from the host copy
  std::vector<Parsed> ps(ns);
  std::vector<std::shared_ptr<Hierarchy>> hs(ns);
  uint64_t max_in = 0, max_out = 0;
  for (uint64_t k = 0; k < ns; ++k) {
    const uint8_t* b = h_in + c.offs[k];
    const uint64_t len = c.offs[k + 1] - c.offs[k];
    Parsed& P = ps[k];
    if (!parse_header(b, len, P)) fail(MGARD_ERR_FORMAT, "truncated slab header");
    check_bins(P, b);
    if (P.hd.total_bytes > len || P.hd.ndim != c.ndim || P.hd.dtype != c.dtype ||
        P.hd.shape[0] != sp.p1[k] - sp.p0[k])
      fail(MGARD_ERR_FORMAT, "slab header does not match the container");
    for (uint32_t d = 1; d < c.ndim; ++d)
      if (P.hd.shape[d] != c.shape[d]) fail(MGARD_ERR_FORMAT, "slab header does not match the container");
    CoordPtrs cp;
    for (uint32_t d = 0; d < P.hd.ndim; ++d) cp.p[d] = P.coords[d].empty() ? nullptr : P.coords[d].data();
    hs[k] = get_hierarchy(P.hd.ndim, P.hd.shape, cp.p);
    if ((uint32_t)hs[k]->L != P.hd.levels) fail(MGARD_ERR_FORMAT, "level count does not match shape");
    max_in = std::max(max_in, len);
    max_out = std::max(max_out, (sp.p1[k] - sp.p0[k]) * plane * sizeof(T));
  }
  // Nothing waits on the host between slabs: each slab's decode status goes to
  // its own 4 words (read once at the end), and events order the buffers:
  // slab k's copy in waits for the kernels of slab k - 2 (same input buffer),
  // its kernels for its copy in and for the copy out of slab k - 2 (same
  // output buffer), its copy out for its kernels.
  Pipeline pl(o0.st);
  pl.alloc(max_in, max_out, 2 * ns);
  uint32_t* st_all = reinterpret_cast<uint32_t*>(pl.bits);
  Opts o = o0;
  o.st = pl.ks;
  auto copy_in = [&](uint64_t k) {
    const int s = (int)(k & 1);
    if (k >= 2) MG_HIP(hipStreamWaitEvent(pl.cs, pl.used[s], 0));
    MG_HIP(hipMemcpyAsync(pl.a[s], h_in + c.offs[k], c.offs[k + 1] - c.offs[k], hipMemcpyHostToDevice, pl.cs));
    MG_HIP(hipEventRecord(pl.in_done[s], pl.cs));
  };
  // Copy engines.  The HIP runtime (ROCm 7) keeps each stream on the DMA
  // engine of its previous copy and moves a copy that finds that engine busy
  // to another one; measured on MI355X, the engine a first copy takes on an
  // idle device moves 542 MB to pinned host memory in 9.5 ms and the other
  // one in 18.2 ms (30 GB/s either way).  The copies out are the large ones
  // here (a slab's values against its compressed bytes), so the copy-out
  // stream takes the fast engine: a short copy on it (into the first slab's
  // host range, which that slab's own copy out overwrites after it, in
  // stream order) is in flight when the first copy in is queued, so the
  // copy-in stream lands on the other engine and both stay there.  The
  // engine choice changes only the speed, never the result (1025^3 float32,
  // slabs of 129 planes: 158 -> 96 ms).
  {
    const uint64_t b0 = (sp.p1[0] - sp.p0[0]) * plane * sizeof(T);
    MG_HIP(hipMemcpyAsync(h_out, pl.b[0], std::min<uint64_t>(b0, 32ull << 20), hipMemcpyDeviceToHost, pl.ds));
  }
  copy_in(0);
  for (uint64_t k = 0; k < ns; ++k) {
    const int s = (int)(k & 1);
    if (k + 1 < ns) copy_in(k + 1);
    MG_HIP(hipStreamWaitEvent(pl.ks, pl.in_done[s], 0));
    if (k >= 2) MG_HIP(hipStreamWaitEvent(pl.ks, pl.out_done[s], 0));
    decompress_impl<T>(*hs[k], ps[k], static_cast<const char*>(pl.a[s]), static_cast<T*>(pl.b[s]), o, st_all + 4 * k);
    MG_HIP(hipEventRecord(pl.used[s], pl.ks));
    MG_HIP(hipStreamWaitEvent(pl.ds, pl.used[s], 0));
    MG_HIP(hipMemcpyAsync(h_out + sp.p0[k] * plane, pl.b[s], (sp.p1[k] - sp.p0[k]) * plane * sizeof(T),
                          hipMemcpyDeviceToHost, pl.ds));
    MG_HIP(hipEventRecord(pl.out_done[s], pl.ds));
  }
  MG_HIP(hipStreamSynchronize(pl.ds));
  uint8_t* stage = pinned_staging(16 * ns);
  MG_HIP(hipMemcpyAsync(stage, st_all, 16 * ns, hipMemcpyDeviceToHost, pl.ks));
  MG_HIP(hipStreamSynchronize(pl.ks));
  for (uint64_t k = 0; k < ns; ++k) {
    uint32_t w;
    std::memcpy(&w, stage + 16 * k, 4);
    if (w) fail(MGARD_ERR_FORMAT, "payload does not decode");
  }
}

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[256] = {};

// Device address of `scratch` on the current device, looked up once per device.
void* noalloc_scratch() {
  int dev = 0;
  MG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 256) fail(MGARD_ERR_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    MG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(MGARD_ERR_DEVICE, "no device address for the fixed scratch array");
    g_noalloc_ptr[dev] = p;
  }
  return g_noalloc_ptr[dev];
}

void check_encode_args(const uint16_t* d_symbols, uint32_t dict_size, uint32_t chunk, const uint8_t* d_code_len,
                       const uint64_t* d_codes, const uint32_t* d_chunk_bits, const uint32_t* d_payload,
                       const uint64_t* payload_words) {
  if (!d_symbols || !d_code_len || !d_codes || !d_chunk_bits || !d_payload || !payload_words)
    fail(MGARD_ERR_ARG, "null buffer");
  if (dict_size < 256 || dict_size > 8192 || (dict_size & (dict_size - 1))) fail(MGARD_ERR_ARG, "dict_size");
  if (chunk < 256 || chunk > 8192 || chunk % 256) fail(MGARD_ERR_ARG, "chunk");
  if (reinterpret_cast<uintptr_t>(d_symbols) % 16) fail(MGARD_ERR_ARG, "d_symbols must be 16-byte aligned");
}

// The encoding stage on caller buffers with its scratch given: word_off
// (nch + 1 entries) and enc_scratch (encode_scratch_bytes(dict)).  Every
// scratch entry read is written first by this call.
void encode_stage(const uint16_t* d_symbols, uint64_t n, uint32_t dict_size, uint32_t chunk,
                  const uint8_t* d_code_len, const uint64_t* d_codes, uint32_t* d_chunk_bits, uint32_t* d_payload,
                  uint64_t payload_capacity, uint64_t* payload_words, uint64_t* word_off, void* enc_scratch,
                  hipStream_t st) {
  const uint64_t nch = (n + chunk - 1) / chunk;
  launch_chunk_bits(d_symbols, n, (int)dict_size, (int)chunk, d_code_len, d_chunk_bits, st);
  launch_scan_words(d_chunk_bits, nch, word_off, st);
  uint64_t total = 0;
  MG_HIP(hipMemcpyAsync(&total, word_off + nch, 8, hipMemcpyDeviceToHost, st));
  MG_HIP(hipStreamSynchronize(st));
  *payload_words = total;
  if (total > payload_capacity) fail(MGARD_ERR_CAPACITY, "payload capacity");
  launch_encode(d_symbols, n, (int)dict_size, (int)chunk, d_code_len, d_codes, word_off, d_payload, nullptr, nullptr,
                nullptr, enc_scratch, false, st);
  MG_HIP(hipStreamSynchronize(st));
}

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" {

void mgard_default_opts(mgard_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(mgard_opts);
  o->eb = MGARD_REL;
  o->alloc = MGARD_ALLOC_PLAIN;
  o->dict_size = 8192;
  o->chunk_symbols = 1024;
}

const char* mgard_last_error(void) { return g_err.c_str(); }

const char* mgard_version(void) { return "mgard-hip 1 (gfx950)"; }

mgard_status mgard_release_workspace(void) {
  return guard([&] {
    workspace().release();
    aux_workspace().release();
  });
}

uint64_t mgard_compress_bound(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                              mgard_dtype dtype, const mgard_opts* opts) {
  uint64_t r = 0;
  mgard_status s = guard([&] {
    Opts o = read_opts(opts);
    (void)dtype_size(dtype);
    auto h = get_hierarchy(ndim, shape, coords);
    r = bound_of(*h, coords, o.dict, o.chunk);
  });
  return s == MGARD_OK ? r : 0;
}

mgard_status mgard_compress(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                            mgard_dtype dtype, double tol, const void* d_in, void* d_out,
                            uint64_t out_capacity, uint64_t* out_bytes, const mgard_opts* opts,
                            mgard_info* info) {
  return guard([&] {
    Opts o = read_opts(opts);
    const int ts = dtype_size(dtype);
    (void)ts;
    if (!d_in || !d_out || !out_bytes) fail(MGARD_ERR_ARG, "null buffer");
    if (!(tol > 0.0) || !std::isfinite(tol)) fail(MGARD_ERR_TOL, "tolerance must be positive and finite");
    if (o.alloc == MGARD_ALLOC_LEARNED) {
      if (!o.model) fail(MGARD_ERR_ARG, "learned allocation needs opts->model");
      o.model_params = model_params(o.model);
    }
    auto h = get_hierarchy(ndim, shape, coords);
    const uint64_t bound = bound_of(*h, coords, o.dict, o.chunk);
    if (out_capacity < bound) {
      *out_bytes = bound;
      fail(MGARD_ERR_CAPACITY, "output capacity below mgard_compress_bound");
    }
    if (dtype == MGARD_F32)
      compress_impl<float>(*h, coords, tol, static_cast<const float*>(d_in), static_cast<char*>(d_out), out_bytes,
                           o, info);
    else
      compress_impl<double>(*h, coords, tol, static_cast<const double*>(d_in), static_cast<char*>(d_out),
                            out_bytes, o, info);
    if (o.lossless == MGARD_LOSSLESS_ZS) {
      // the stream's container, staged aside; kept when it is the smaller
      const uint64_t nb = *out_bytes;
      const uint64_t nch = (nb + 16383) / 16384;
      Workspace& aux = aux_workspace();
      aux.reserve(carve_size<char>(zs_bound(nb)) + carve_size<uint32_t>(nch + 1) + 1024);
      Carver cv(aux.base());
      char* stage = cv.take<char>(zs_bound(nb));
      uint32_t* sizes = cv.take<uint32_t>(nch + 1);
      const uint64_t cb = zs_encode(d_out, nb, stage, zs_bound(nb), sizes, o.st);
      if (cb < nb) {
        MG_HIP(hipMemcpyAsync(d_out, stage, cb, hipMemcpyDeviceToDevice, o.st));
        MG_HIP(hipStreamSynchronize(o.st));
        *out_bytes = cb;
        if (info) info->out_bytes = cb;
      }
    }
  });
}

mgard_status mgard_autotune(uint32_t ndim, const uint64_t* shape, const double* const* coords, mgard_dtype dtype,
                            const void* d_in, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    (void)dtype_size(dtype);
    if (!d_in) fail(MGARD_ERR_ARG, "null buffer");
    auto h = get_hierarchy(ndim, shape, coords);
    if (dtype == MGARD_F32)
      autotune_impl<float>(*h, static_cast<const float*>(d_in), o);
    else
      autotune_impl<double>(*h, static_cast<const double*>(d_in), o);
  });
}

uint64_t mgard_batch_bound(uint32_t nfields, const mgard_field* fields, const mgard_opts* opts) {
  uint64_t total = 0;
  mgard_status s = guard([&] {
    Opts o = read_opts(opts);
    if (!fields && nfields) fail(MGARD_ERR_ARG, "null fields");
    uint64_t mem = 0;
    (void)plan_jobs(nfields, fields, 1.0, o, false, &total, &mem);
  });
  return s == MGARD_OK ? total : 0;
}

mgard_status mgard_batch_create(uint32_t nfields, const mgard_field* fields, double tol, void* d_out,
                                uint64_t out_capacity, uint64_t* h_offsets, uint64_t* d_sizes,
                                const mgard_opts* opts, mgard_batch** plan) {
  return guard([&] {
    if (!plan) fail(MGARD_ERR_ARG, "null plan");
    *plan = nullptr;
    Opts o = read_opts(opts);
    if (o.alloc == MGARD_ALLOC_LEARNED) fail(MGARD_ERR_ARG, "batches use the plain or count allocation");
    if (o.norm == MGARD_NORM_S) fail(MGARD_ERR_ARG, "batches bound the L-infinity norm");
    if (!nfields || !fields || !d_out || !h_offsets || !d_sizes) fail(MGARD_ERR_ARG, "null buffer or no fields");
    if (!(tol > 0.0) || !std::isfinite(tol)) fail(MGARD_ERR_TOL, "tolerance must be positive and finite");
    for (uint32_t i = 0; i < nfields; ++i)
      if (!fields[i].d_in) fail(MGARD_ERR_ARG, "null field input");
    std::unique_ptr<mgard_batch, void (*)(mgard_batch*)> B(new mgard_batch, mgard_batch_free);
    MG_HIP(hipGetDevice(&B->device));
    uint64_t out_total = 0, mem_total = 0;
    std::vector<BatchJob> jobs = plan_jobs(nfields, fields, tol, o, true, &out_total, &mem_total);
    if (out_capacity < out_total) fail(MGARD_ERR_CAPACITY, "output capacity below mgard_batch_bound");
    if (hipMalloc(&B->mem, std::max<uint64_t>(mem_total, 256)) != hipSuccess) {
      (void)hipGetLastError();
      B->mem = nullptr;
      fail(MGARD_ERR_OOM, "batch scratch");
    }
    char* mem = static_cast<char*>(B->mem);
    for (uint32_t i = 0; i < nfields; ++i) {
      MG_HIP(hipMemcpy(mem + jobs[i].hdr_off, jobs[i].hb.data(), jobs[i].hb.size(), hipMemcpyHostToDevice));
      h_offsets[i] = jobs[i].out_off;
    }
    // launch shapes for every level shape not tuned yet
    for (uint32_t i = 0; i < nfields; ++i) {
      Hierarchy& h = *jobs[i].h;
      if (tuned_all_levels(h, jobs[i].f64)) continue;
      if (jobs[i].f64)
        autotune_impl<double>(h, static_cast<const double*>(fields[i].d_in), o);
      else
        autotune_impl<float>(h, static_cast<const float*>(fields[i].d_in), o);
    }
    MG_HIP(hipDeviceSynchronize());

    // Every field's launches, recorded in order: up to the histogram, the
    // codebook, then the rest (the order of a single compression, with no
    // side stream).
    std::vector<Recorder> recs(nfields);
    {
      struct Restore {
        ~Restore() {
          recorder() = nullptr;
          timing_pause(false);
        }
      } restore;
      timing_pause(true);
      for (uint32_t i = 0; i < nfields; ++i) {
        const BatchJob& J = jobs[i];
        char* out = static_cast<char*>(d_out) + J.out_off;
        const uint8_t* hdr = reinterpret_cast<const uint8_t*>(mem + J.hdr_off);
        recorder() = &recs[i];
        auto record = [&](auto tag) {
          using T = decltype(tag);
          const T* in = static_cast<const T*>(fields[i].d_in);
          const T* table = static_cast<const T*>(J.table);
          compress_enqueue<T>(*J.h, table, J.y, tol, in, out, o, mem + J.scr_off, hdr, J.hb.size(), d_sizes + i,
                              CE_FRONT);
          const CompressBufs cb = carve_compress<T>(*J.h, J.y, o, mem + J.scr_off);
          launch_codebook(cb.hist, o.dict, reinterpret_cast<uint8_t*>(out + J.y.code_len), cb.codes, cb.enc_scratch,
                          o.st);
          compress_enqueue<T>(*J.h, table, J.y, tol, in, out, o, mem + J.scr_off, hdr, J.hb.size(), d_sizes + i,
                              CE_BACK);
        };
        if (J.f64)
          record(double{});
        else
          record(float{});
        recorder() = nullptr;
      }
    }

    // Grouping.  Fields are split into classes by their first decomposition
    // body (the fused 3D path, the generic path, the one-block small levels,
    // per precision); each class becomes its own chain of grouped launches,
    // and the chains run on parallel branches of the graph, so the
    // latency-bound line solves of one class overlap the bandwidth-bound
    // kernels of another.  Within a class, each field's records fall in three
    // phases: the stages before the decomposition, the decomposition (whose
    // length depends on the shape), the stages after it.  Every record gets a
    // slot: its index in the first and third phases (those after the longest
    // first phase), and in the decomposition its index counted back from the
    // phase's end, so that every field finishes its decomposition in the same
    // slot.  The records of one slot and body form one grouped launch; slots
    // run in order, so each field's records keep their order, and fields share
    // no memory.
    struct Group {
      const GroupOps* ops;
      std::vector<const LaunchRecord*> members;
    };
    for (uint32_t i = 0; i < nfields; ++i) {
      int last = 0;
      for (const LaunchRecord& r : recs[i].recs) {
        if (r.phase < last || r.phase > 2) fail(MGARD_ERR_ARG, "recorded phases out of order");
        last = r.phase;
      }
    }
    std::vector<const GroupOps*> class_key;
    std::vector<std::vector<uint32_t>> class_fields;
    for (uint32_t i = 0; i < nfields; ++i) {
      const GroupOps* key = nullptr;
      for (const LaunchRecord& r : recs[i].recs)
        if (r.phase == 1) {
          key = r.ops;
          break;
        }
      size_t c = 0;
      while (c < class_key.size() && class_key[c] != key) ++c;
      if (c == class_key.size()) {
        class_key.push_back(key);
        class_fields.emplace_back();
      }
      class_fields[c].push_back(i);
    }
    auto group_class = [&](const std::vector<uint32_t>& members) {
      std::vector<size_t> len[3];
      size_t maxlen[3] = {0, 0, 0};
      for (uint32_t i : members) {
        size_t c[3] = {0, 0, 0};
        for (const LaunchRecord& r : recs[i].recs) ++c[r.phase];
        for (int ph = 0; ph < 3; ++ph) {
          len[ph].push_back(c[ph]);
          maxlen[ph] = std::max(maxlen[ph], c[ph]);
        }
      }
      const size_t nslots = maxlen[0] + maxlen[1] + maxlen[2];
      std::vector<std::vector<Group>> slots(nslots);
      for (size_t m = 0; m < members.size(); ++m) {
        size_t k[3] = {0, 0, 0};
        for (const LaunchRecord& r : recs[members[m]].recs) {
          const int ph = r.phase;
          size_t slot = k[ph]++;
          if (ph == 1) slot += maxlen[0] + (maxlen[1] - len[1][m]);
          if (ph == 2) slot += maxlen[0] + maxlen[1];
          std::vector<Group>& gs = slots[slot];
          Group* g = nullptr;
          for (Group& x : gs)
            if (x.ops == r.ops) g = &x;
          if (!g) {
            gs.push_back(Group{r.ops, {}});
            g = &gs.back();
          }
          g->members.push_back(&r);
        }
      }
      std::vector<Group> out;
      for (auto& gs : slots)
        for (auto& g : gs) out.push_back(std::move(g));
      return out;
    };
    std::vector<Group> groups;
    std::vector<size_t> class_begin;  // groups of class c: [class_begin[c], class_begin[c + 1])
    for (const auto& members : class_fields) {
      class_begin.push_back(groups.size());
      for (Group& g : group_class(members)) groups.push_back(std::move(g));
    }
    class_begin.push_back(groups.size());

    // job tables: per group, (first block, grid, arguments) of every member
    std::vector<uint64_t> toff(groups.size());
    std::vector<uint32_t> tblocks(groups.size());
    uint64_t tbytes = 0;
    for (size_t k = 0; k < groups.size(); ++k) {
      toff[k] = tbytes;
      tbytes = align256(tbytes + groups[k].members.size() * groups[k].ops->job_bytes);
    }
    std::vector<uint8_t> htab(std::max<uint64_t>(tbytes, 256), 0);
    for (size_t k = 0; k < groups.size(); ++k) {
      uint64_t begin = 0;
      for (size_t m = 0; m < groups[k].members.size(); ++m) {
        const LaunchRecord* r = groups[k].members[m];
        groups[k].ops->write_job(htab.data() + toff[k] + m * groups[k].ops->job_bytes, (uint32_t)begin, r->grid,
                                 r->pack.data());
        begin += (uint64_t)r->grid.x * r->grid.y * r->grid.z;
      }
      if (begin > 0x7fffffffull) fail(MGARD_ERR_SHAPE, "a grouped launch needs more than 2^31 blocks");
      tblocks[k] = (uint32_t)begin;
    }
    if (hipMalloc(&B->tables, htab.size()) != hipSuccess) {
      (void)hipGetLastError();
      B->tables = nullptr;
      fail(MGARD_ERR_OOM, "batch job tables");
    }
    MG_HIP(hipMemcpy(B->tables, htab.data(), htab.size(), hipMemcpyHostToDevice));

    // one graph: class 0's chain on the capturing stream, every other class's
    // chain on a stream of its own forked from it and joined back at the end
    const size_t ncls = class_fields.size();
    std::vector<hipStream_t> cs(ncls, nullptr);
    std::vector<hipEvent_t> ev(ncls, nullptr);
    struct Release {
      std::vector<hipStream_t>& s;
      std::vector<hipEvent_t>& e;
      ~Release() {
        for (hipStream_t x : s)
          if (x) (void)hipStreamDestroy(x);
        for (hipEvent_t x : e)
          if (x) (void)hipEventDestroy(x);
      }
    } release{cs, ev};
    for (size_t c = 0; c < ncls; ++c) {
      MG_HIP(hipStreamCreateWithFlags(&cs[c], hipStreamNonBlocking));
      MG_HIP(hipEventCreateWithFlags(&ev[c], hipEventDisableTiming));
    }
    MG_HIP(hipStreamBeginCapture(cs[0], hipStreamCaptureModeThreadLocal));
    try {
      MG_HIP(hipEventRecord(ev[0], cs[0]));
      for (size_t c = 1; c < ncls; ++c) MG_HIP(hipStreamWaitEvent(cs[c], ev[0], 0));
      uint32_t n = 0;
      for (size_t c = 0; c < ncls; ++c)
        for (size_t k = class_begin[c]; k < class_begin[c + 1]; ++k) {
          if (!tblocks[k]) continue;
          groups[k].ops->launch(static_cast<char*>(B->tables) + toff[k], (uint32_t)groups[k].members.size(),
                                tblocks[k], cs[c]);
          ++n;
        }
      for (size_t c = 1; c < ncls; ++c) {
        MG_HIP(hipEventRecord(ev[c], cs[c]));
        MG_HIP(hipStreamWaitEvent(cs[0], ev[c], 0));
      }
      MG_HIP(hipGetLastError());
      MG_HIP(hipStreamEndCapture(cs[0], &B->graph));
      B->launches = n;
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(cs[0], &g);
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      throw;
    }
    MG_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    *plan = B.release();
  });
}

uint32_t mgard_batch_launches(const mgard_batch* plan) { return plan ? plan->launches : 0; }

mgard_status mgard_batch_launch(mgard_batch* plan, void* stream) {
  return guard([&] {
    if (!plan || !plan->exec) fail(MGARD_ERR_ARG, "null plan");
    int dev = -1;
    MG_HIP(hipGetDevice(&dev));
    if (dev != plan->device) fail(MGARD_ERR_ARG, "plan lives on another device");
    MG_HIP(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
  });
}

void mgard_batch_free(mgard_batch* plan) {
  if (!plan) return;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->mem || plan->tables) (void)hipDeviceSynchronize();
  if (plan->mem) (void)hipFree(plan->mem);
  if (plan->tables) (void)hipFree(plan->tables);
  delete plan;
}

mgard_status mgard_inspect(const void* h_buf, uint64_t bytes, mgard_header* hdr) {
  return guard([&] {
    if (!h_buf || !hdr) fail(MGARD_ERR_ARG, "null pointer");
    Parsed P;
    if (!parse_header(static_cast<const uint8_t*>(h_buf), bytes, P)) {
      *hdr = P.hd;
      hdr->total_bytes = P.need;
      fail(MGARD_ERR_CAPACITY, "more header bytes needed");
    }
    check_bins(P, static_cast<const uint8_t*>(h_buf));
    *hdr = P.hd;
  });
}

mgard_status mgard_decompress(const void* d_in, uint64_t in_bytes, void* d_out, uint64_t out_capacity,
                              const mgard_opts* opts, mgard_header* hdr) {
  return guard([&] {
    Opts o = read_opts(opts);
    if (!d_in || !d_out) fail(MGARD_ERR_ARG, "null buffer");
    // One read of the buffer's first kPrefix bytes serves the container
    // check and, almost always, the whole header.
    constexpr uint64_t kPrefix = 4096;
    std::vector<uint8_t> hb;
    {
      const uint64_t got = std::min<uint64_t>(in_bytes, kPrefix);
      uint8_t* stage = pinned_staging(kPrefix);
      MG_HIP(hipMemcpyAsync(stage, d_in, got, hipMemcpyDeviceToHost, o.st));
      MG_HIP(hipStreamSynchronize(o.st));
      hb.assign(stage, stage + got);
    }
    {
      // a stream in the lossless stage's container: decoded aside first
      uint8_t zh[24] = {0};
      const uint64_t got = std::min<uint64_t>(in_bytes, 24);
      std::memcpy(zh, hb.data(), got);
      uint64_t raw = 0, nch = 0;
      if (got >= 4 && std::memcmp(zh, "MGZS", 4) == 0) {
        if (!zs_parse(zh, in_bytes, &raw, &nch)) fail(MGARD_ERR_FORMAT, "malformed lossless container");
        Workspace& aux = aux_workspace();
        aux.reserve(carve_size<uint32_t>((raw + 3) / 4) + carve_size<uint64_t>(1) + 1024);
        Carver cv(aux.base());
        uint32_t* plain = cv.take<uint32_t>((raw + 3) / 4);
        uint32_t* status = reinterpret_cast<uint32_t*>(cv.take<uint64_t>(1));
        zs_decode(d_in, in_bytes, raw, nch, plain, status, o.st);
        d_in = plain;
        in_bytes = raw;
        const uint64_t got2 = std::min<uint64_t>(in_bytes, kPrefix);
        uint8_t* stage = pinned_staging(kPrefix);
        MG_HIP(hipMemcpyAsync(stage, d_in, got2, hipMemcpyDeviceToHost, o.st));
        MG_HIP(hipStreamSynchronize(o.st));
        hb.assign(stage, stage + got2);
      }
    }
    if (in_bytes < kFixed) fail(MGARD_ERR_FORMAT, "buffer shorter than a header");
    Parsed P;
    // the header grows in three parts (fixed, shape, coordinates + bins): read each as it is known
    for (int part = 0; !parse_header(hb.data(), hb.size(), P); ++part) {
      if (part == 3 || P.need <= hb.size() || P.need > in_bytes) fail(MGARD_ERR_FORMAT, "truncated header");
      hb.resize(P.need);
      MG_HIP(hipMemcpyAsync(hb.data(), d_in, P.need, hipMemcpyDeviceToHost, o.st));
      MG_HIP(hipStreamSynchronize(o.st));
      P = Parsed();
    }
    check_bins(P, hb.data());
    if (P.hd.total_bytes > in_bytes) fail(MGARD_ERR_FORMAT, "buffer shorter than its header says");
    const int ts = P.hd.dtype ? 8 : 4;
    if (out_capacity < P.hd.n_symbols * (uint64_t)ts) fail(MGARD_ERR_CAPACITY, "output buffer too small");
    CoordPtrs cp;
    for (uint32_t d = 0; d < P.hd.ndim; ++d) cp.p[d] = P.coords[d].empty() ? nullptr : P.coords[d].data();
    auto h = get_hierarchy(P.hd.ndim, P.hd.shape, cp.p);
    if ((uint32_t)h->L != P.hd.levels) fail(MGARD_ERR_FORMAT, "level count does not match shape");
    if (P.hd.dtype)
      decompress_impl<double>(*h, P, static_cast<const char*>(d_in), static_cast<double*>(d_out), o);
    else
      decompress_impl<float>(*h, P, static_cast<const char*>(d_in), static_cast<float*>(d_out), o);
    if (hdr) *hdr = P.hd;
  });
}

mgard_status mgard_stream_layout(uint32_t ndim, const uint64_t* shape, uint32_t* levels,
                                 uint64_t* level_offsets, uint32_t max_offsets) {
  return guard([&] {
    if (!levels) fail(MGARD_ERR_ARG, "null pointer");
    auto h = get_hierarchy(ndim, shape, nullptr);
    *levels = (uint32_t)h->L;
    if (level_offsets) {
      if (max_offsets < (uint32_t)h->L + 2) fail(MGARD_ERR_CAPACITY, "level_offsets too short");
      for (int l = 0; l <= h->L + 1; ++l) level_offsets[l] = h->level_off[l];
    }
  });
}

mgard_status mgard_decompose(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                             mgard_dtype dtype, const void* d_in, void* d_coeff, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    (void)dtype_size(dtype);
    if (!d_in || !d_coeff) fail(MGARD_ERR_ARG, "null buffer");
    auto h = get_hierarchy(ndim, shape, coords);
    const bool f64 = dtype == MGARD_F64;
    const void* table = device_table(*h, f64, o.st);
    Workspace& ws = workspace();
    if (f64) {
      ws.reserve(decompose_scratch_bytes<double>(*h));
      decompose<double>(*h, static_cast<const double*>(table), static_cast<const double*>(d_in),
                        static_cast<double*>(d_coeff), nullptr, ws.base(), o.st);
    } else {
      ws.reserve(decompose_scratch_bytes<float>(*h));
      decompose<float>(*h, static_cast<const float*>(table), static_cast<const float*>(d_in),
                       static_cast<float*>(d_coeff), nullptr, ws.base(), o.st);
    }
    MG_HIP(hipStreamSynchronize(o.st));
  });
}

mgard_status mgard_recompose(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                             mgard_dtype dtype, const void* d_coeff, void* d_out, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    (void)dtype_size(dtype);
    if (!d_coeff || !d_out) fail(MGARD_ERR_ARG, "null buffer");
    auto h = get_hierarchy(ndim, shape, coords);
    const bool f64 = dtype == MGARD_F64;
    const void* table = device_table(*h, f64, o.st);
    Workspace& ws = workspace();
    if (f64) {
      ws.reserve(recompose_scratch_bytes<double>(*h));
      recompose<double>(*h, static_cast<const double*>(table), static_cast<const double*>(d_coeff), nullptr,
                        static_cast<double*>(d_out), ws.base(), o.st);
    } else {
      ws.reserve(recompose_scratch_bytes<float>(*h));
      recompose<float>(*h, static_cast<const float*>(table), static_cast<const float*>(d_coeff), nullptr,
                       static_cast<float*>(d_out), ws.base(), o.st);
    }
    MG_HIP(hipStreamSynchronize(o.st));
  });
}

// small device copies of level offsets and bin widths for the stage calls
static void stage_tables(const Hierarchy& h, const double* h_bins, hipStream_t st, uint64_t** d_off,
                         double** d_bins) {
  Workspace& ws = workspace();
  ws.reserve(carve_size<uint64_t>(MAXL + 2) + carve_size<double>(MAXL + 1) + 1024);
  Carver cv(ws.base());
  *d_off = cv.take<uint64_t>(MAXL + 2);
  *d_bins = cv.take<double>(MAXL + 1);
  MG_HIP(hipMemcpyAsync(*d_off, h.level_off.data(), 8 * (h.L + 2), hipMemcpyHostToDevice, st));
  MG_HIP(hipMemcpyAsync(*d_bins, h_bins, 8 * (h.L + 1), hipMemcpyHostToDevice, st));
}

mgard_status mgard_quantize(uint32_t ndim, const uint64_t* shape, mgard_dtype dtype, const void* d_coeff,
                            const double* h_bins, uint32_t dict_size, uint16_t* d_symbols, int64_t* d_qside,
                            const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    (void)dtype_size(dtype);
    if (!d_coeff || !h_bins || !d_symbols || !d_qside) fail(MGARD_ERR_ARG, "null buffer");
    if (dict_size < 256 || dict_size > 8192 || (dict_size & (dict_size - 1))) fail(MGARD_ERR_ARG, "dict_size");
    auto h = get_hierarchy(ndim, shape, nullptr);
    for (int l = 0; l <= h->L; ++l)
      if (!(h_bins[l] > 0.0) || !std::isfinite(h_bins[l])) fail(MGARD_ERR_ARG, "bin widths must be positive");
    uint64_t* off;
    double* bins;
    stage_tables(*h, h_bins, o.st, &off, &bins);
    const uint64_t n = h->count(h->L);
    if (dtype == MGARD_F64)
      launch_quantize<double>(static_cast<const double*>(d_coeff), n, off, h->L + 1, bins, (int)dict_size / 2,
                              d_symbols, d_qside, o.st);
    else
      launch_quantize<float>(static_cast<const float*>(d_coeff), n, off, h->L + 1, bins, (int)dict_size / 2,
                             d_symbols, d_qside, o.st);
    MG_HIP(hipStreamSynchronize(o.st));
  });
}

mgard_status mgard_dequantize(uint32_t ndim, const uint64_t* shape, mgard_dtype dtype,
                              const uint16_t* d_symbols, const int64_t* d_qside, const double* h_bins,
                              uint32_t dict_size, void* d_coeff, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    (void)dtype_size(dtype);
    if (!d_coeff || !h_bins || !d_symbols || !d_qside) fail(MGARD_ERR_ARG, "null buffer");
    if (dict_size < 256 || dict_size > 8192 || (dict_size & (dict_size - 1))) fail(MGARD_ERR_ARG, "dict_size");
    auto h = get_hierarchy(ndim, shape, nullptr);
    uint64_t* off;
    double* bins;
    stage_tables(*h, h_bins, o.st, &off, &bins);
    const uint64_t n = h->count(h->L);
    if (dtype == MGARD_F64)
      launch_dequantize<double>(d_symbols, d_qside, n, off, h->L + 1, bins, (int)dict_size / 2,
                                static_cast<double*>(d_coeff), o.st);
    else
      launch_dequantize<float>(d_symbols, d_qside, n, off, h->L + 1, bins, (int)dict_size / 2,
                               static_cast<float*>(d_coeff), o.st);
    MG_HIP(hipStreamSynchronize(o.st));
  });
}

mgard_status mgard_histogram(const uint16_t* d_symbols, uint64_t n, uint32_t dict_size, uint32_t chunk,
                             uint64_t* d_hist, uint32_t* d_chunk_esc, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    if (!d_symbols || !d_hist || !d_chunk_esc) fail(MGARD_ERR_ARG, "null buffer");
    if (dict_size < 256 || dict_size > 8192 || (dict_size & (dict_size - 1))) fail(MGARD_ERR_ARG, "dict_size");
    if (chunk < 256 || chunk > 8192 || chunk % 256) fail(MGARD_ERR_ARG, "chunk");
    if (reinterpret_cast<uintptr_t>(d_symbols) % 16) fail(MGARD_ERR_ARG, "d_symbols must be 16-byte aligned");
    Workspace& ws = workspace();
    ws.reserve(1024);
    uint32_t* status = static_cast<uint32_t*>(ws.base());
    MG_HIP(hipMemsetAsync(status, 0, 4, o.st));
    launch_histogram(d_symbols, n, (int)dict_size, (int)chunk, d_hist, d_chunk_esc, status, o.st);
    uint32_t hs = 0;
    MG_HIP(hipMemcpyAsync(&hs, status, 4, hipMemcpyDeviceToHost, o.st));
    MG_HIP(hipStreamSynchronize(o.st));
    if (hs) fail(MGARD_ERR_ARG, "a symbol lies outside the dictionary");
  });
}

mgard_status mgard_huffman_codebook(const uint64_t* d_hist, uint32_t dict_size, uint8_t* d_code_len,
                                    uint64_t* d_codes, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    if (!d_hist || !d_code_len || !d_codes) fail(MGARD_ERR_ARG, "null buffer");
    if (dict_size < 256 || dict_size > 8192 || (dict_size & (dict_size - 1))) fail(MGARD_ERR_ARG, "dict_size");
    launch_codebook(d_hist, (int)dict_size, d_code_len, d_codes, nullptr, o.st);
    MG_HIP(hipStreamSynchronize(o.st));
  });
}

mgard_status mgard_huffman_encode(const uint16_t* d_symbols, uint64_t n, uint32_t dict_size, uint32_t chunk,
                                  const uint8_t* d_code_len, const uint64_t* d_codes, uint32_t* d_chunk_bits,
                                  uint32_t* d_payload, uint64_t payload_capacity, uint64_t* payload_words,
                                  const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    check_encode_args(d_symbols, dict_size, chunk, d_code_len, d_codes, d_chunk_bits, d_payload, payload_words);
    const uint64_t nch = (n + chunk - 1) / chunk;
    Workspace& ws = workspace();
    ws.reserve(carve_size<uint64_t>(nch + 1) + encode_scratch_bytes((int)dict_size) + 1024);
    Carver cv(ws.base());
    uint64_t* word_off = cv.take<uint64_t>(nch + 1);
    void* enc_scratch = cv.take<char>(encode_scratch_bytes((int)dict_size));
    encode_stage(d_symbols, n, dict_size, chunk, d_code_len, d_codes, d_chunk_bits, d_payload, payload_capacity,
                 payload_words, word_off, enc_scratch, o.st);
  });
}

mgard_status mgard_huffman_encode_noalloc(const uint16_t* d_symbols, uint64_t n, uint32_t dict_size, uint32_t chunk,
                                          const uint8_t* d_code_len, const uint64_t* d_codes, uint32_t* d_chunk_bits,
                                          uint32_t* d_payload, uint64_t payload_capacity, uint64_t* payload_words,
                                          const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    check_encode_args(d_symbols, dict_size, chunk, d_code_len, d_codes, d_chunk_bits, d_payload, payload_words);
    const uint64_t nch = (n + chunk - 1) / chunk;
    if (nch > (uint64_t)MGARD_NOALLOC_MAX_CHUNKS)
      fail(MGARD_ERR_CAPACITY, "more chunks than MGARD_NOALLOC_MAX_CHUNKS");
    Carver cv(noalloc_scratch());
    uint64_t* word_off = cv.take<uint64_t>(nch + 1);
    void* enc_scratch = cv.take<char>(encode_scratch_bytes((int)dict_size));
    if (cv.used > kNoallocBytes) fail(MGARD_ERR_CAPACITY, "fixed scratch too small");
    encode_stage(d_symbols, n, dict_size, chunk, d_code_len, d_codes, d_chunk_bits, d_payload, payload_capacity,
                 payload_words, word_off, enc_scratch, o.st);
  });
}

mgard_status mgard_huffman_decode(const uint32_t* d_payload, uint64_t payload_words, const uint32_t* d_chunk_bits,
                                  uint64_t n, uint32_t dict_size, uint32_t chunk, const uint8_t* d_code_len,
                                  uint16_t* d_symbols, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    if (!d_payload || !d_chunk_bits || !d_code_len || !d_symbols) fail(MGARD_ERR_ARG, "null buffer");
    if (dict_size < 256 || dict_size > 8192 || (dict_size & (dict_size - 1))) fail(MGARD_ERR_ARG, "dict_size");
    if (chunk < 256 || chunk > 8192 || chunk % 256) fail(MGARD_ERR_ARG, "chunk");
    if (reinterpret_cast<uintptr_t>(d_symbols) % 16) fail(MGARD_ERR_ARG, "d_symbols must be 16-byte aligned");
    const uint64_t nch = (n + chunk - 1) / chunk;
    Workspace& ws = workspace();
    ws.reserve(carve_size<uint64_t>(nch + 1) + decode_table_bytes((int)dict_size) + carve_size<uint32_t>(4) +
               1024);
    Carver cv(ws.base());
    uint64_t* word_off = cv.take<uint64_t>(nch + 1);
    void* tabs = cv.take<char>(decode_table_bytes((int)dict_size));
    uint32_t* status = cv.take<uint32_t>(4);
    MG_HIP(hipMemsetAsync(status, 0, 16, o.st));
    launch_scan_words(d_chunk_bits, nch, word_off, o.st);
    launch_decode_full(d_payload, payload_words, word_off, d_chunk_bits, n, (int)dict_size, (int)chunk,
                       d_code_len, d_symbols, nullptr, 0, nullptr, tabs, status, o.st);
    uint32_t hs[4];
    MG_HIP(hipMemcpyAsync(hs, status, 16, hipMemcpyDeviceToHost, o.st));
    MG_HIP(hipStreamSynchronize(o.st));
    if (hs[0]) fail(MGARD_ERR_FORMAT, "payload does not decode");
  });
}

mgard_status mgard_maxabs(mgard_dtype dtype, const void* d_in, uint64_t n, double* h_maxabs,
                          const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    (void)dtype_size(dtype);
    if (!d_in || !h_maxabs) fail(MGARD_ERR_ARG, "null pointer");
    Workspace& ws = workspace();
    ws.reserve(1024);
    uint64_t* bits = static_cast<uint64_t*>(ws.base());
    if (dtype == MGARD_F64)
      launch_maxabs<double>(static_cast<const double*>(d_in), n, bits, o.st);
    else
      launch_maxabs<float>(static_cast<const float*>(d_in), n, bits, o.st);
    uint64_t hb = 0;
    MG_HIP(hipMemcpyAsync(&hb, bits, 8, hipMemcpyDeviceToHost, o.st));
    MG_HIP(hipStreamSynchronize(o.st));
    double m;
    if (dtype == MGARD_F64) {
      if (hb >= 0x7ff0000000000000ull) fail(MGARD_ERR_NONFINITE, "NaN or infinity");
      std::memcpy(&m, &hb, 8);
    } else {
      if (hb >= 0x7f800000ull) fail(MGARD_ERR_NONFINITE, "NaN or infinity");
      uint32_t b32 = (uint32_t)hb;
      float f;
      std::memcpy(&f, &b32, 4);
      m = f;
    }
    *h_maxabs = m;
  });
}

mgard_status mgard_timing(int enable) {
  return guard([&] { timing_set(enable); });
}

mgard_status mgard_timing_report(char* h_buf, uint64_t capacity, uint64_t* needed) {
  return guard([&] {
    std::string r = timing_report();
    if (needed) *needed = r.size() + 1;
    if (!h_buf || capacity < r.size() + 1) fail(MGARD_ERR_CAPACITY, "report buffer too small");
    std::memcpy(h_buf, r.c_str(), r.size() + 1);
  });
}

mgard_status mgard_plain_constant(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                                  double* h_S, double* h_K, uint32_t max_levels) {
  return guard([&] {
    if (!h_S) fail(MGARD_ERR_ARG, "null pointer");
    auto h = get_hierarchy(ndim, shape, coords);
    *h_S = h->S;
    if (h_K) {
      if (max_levels < (uint32_t)h->L + 1) fail(MGARD_ERR_CAPACITY, "h_K too short");
      for (int l = 0; l <= h->L; ++l) h_K[l] = h->K[l];
    }
  });
}

// ------------------------------------------------------------ learned allocation
mgard_status mgard_model_create(const float* h_params, uint64_t n_params, mgard_model** out) {
  return guard([&] {
    if (!h_params || !out) fail(MGARD_ERR_ARG, "null pointer");
    if (n_params != (uint64_t)MLP_NPARAM) fail(MGARD_ERR_ARG, "parameter count must be MGARD_MLP_NPARAM");
    for (uint64_t i = 0; i < n_params; ++i)
      if (!std::isfinite(h_params[i])) fail(MGARD_ERR_ARG, "non-finite parameter");
    for (int i = 0; i < MLP_IN; ++i)
      if (!(h_params[MLP_IN + i] > 0.0f)) fail(MGARD_ERR_ARG, "feature scales must be positive");
    auto* m = new mgard_model();
    MG_HIP(hipGetDevice(&m->device));
    if (hipMalloc(&m->d_params, n_params * sizeof(float)) != hipSuccess) {
      delete m;
      fail(MGARD_ERR_OOM, "model parameters");
    }
    MG_HIP(hipMemcpy(m->d_params, h_params, n_params * sizeof(float), hipMemcpyHostToDevice));
    *out = m;
  });
}

void mgard_model_free(mgard_model* model) {
  if (!model) return;
  if (model->d_params) (void)hipFree(model->d_params);
  delete model;
}

mgard_status mgard_level_stats(uint32_t ndim, const uint64_t* shape, mgard_dtype dtype, const void* d_coeff,
                               double* h_stats, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    (void)dtype_size(dtype);
    if (!d_coeff || !h_stats) fail(MGARD_ERR_ARG, "null pointer");
    auto h = get_hierarchy(ndim, shape, nullptr);
    const int nl = h->L + 1;
    Workspace& ws = workspace();
    ws.reserve(carve_size<uint64_t>(MAXL + 2) + carve_size<double>((uint64_t)2 * nl * STATS_BLOCKS) +
               carve_size<double>(3 * (MAXL + 1)) + 1024);
    Carver cv(ws.base());
    uint64_t* d_off = cv.take<uint64_t>(MAXL + 2);
    double* part = cv.take<double>((uint64_t)2 * nl * STATS_BLOCKS);
    double* stats = cv.take<double>(3 * (MAXL + 1));
    MG_HIP(hipMemcpyAsync(d_off, h->level_off.data(), 8 * (h->L + 2), hipMemcpyHostToDevice, o.st));
    if (dtype == MGARD_F64)
      launch_level_stats<double>(static_cast<const double*>(d_coeff), d_off, nl, part, stats, o.st);
    else
      launch_level_stats<float>(static_cast<const float*>(d_coeff), d_off, nl, part, stats, o.st);
    MG_HIP(hipMemcpyAsync(h_stats, stats, 8 * 3 * nl, hipMemcpyDeviceToHost, o.st));
    MG_HIP(hipStreamSynchronize(o.st));
  });
}

mgard_status mgard_level_features(uint32_t ndim, const uint64_t* shape, mgard_dtype dtype, const void* d_coeff,
                                  double tau_abs, float* h_x, uint32_t max_rows, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    (void)dtype_size(dtype);
    if (!d_coeff || !h_x) fail(MGARD_ERR_ARG, "null pointer");
    if (!(tau_abs > 0.0) || !std::isfinite(tau_abs)) fail(MGARD_ERR_TOL, "tau_abs must be positive and finite");
    auto h = get_hierarchy(ndim, shape, nullptr);
    const int nl = h->L + 1;
    if ((uint32_t)nl > max_rows) fail(MGARD_ERR_CAPACITY, "h_x holds fewer rows than levels + 1");
    Workspace& ws = workspace();
    ws.reserve(carve_size<uint64_t>(MAXL + 2) + carve_size<double>((uint64_t)2 * nl * STATS_BLOCKS) +
               carve_size<double>(3 * (MAXL + 1)) + carve_size<double>(8) +
               carve_size<float>((uint64_t)MLP_IN * (MAXL + 1)) + 1024);
    Carver cv(ws.base());
    uint64_t* d_off = cv.take<uint64_t>(MAXL + 2);
    double* part = cv.take<double>((uint64_t)2 * nl * STATS_BLOCKS);
    double* stats = cv.take<double>(3 * (MAXL + 1));
    double* scalars = cv.take<double>(8);
    float* x = cv.take<float>((uint64_t)MLP_IN * (MAXL + 1));
    MG_HIP(hipMemcpyAsync(d_off, h->level_off.data(), 8 * (h->L + 2), hipMemcpyHostToDevice, o.st));
    MG_HIP(hipMemcpyAsync(scalars, &tau_abs, 8, hipMemcpyHostToDevice, o.st));
    if (dtype == MGARD_F64)
      launch_level_stats<double>(static_cast<const double*>(d_coeff), d_off, nl, part, stats, o.st);
    else
      launch_level_stats<float>(static_cast<const float*>(d_coeff), d_off, nl, part, stats, o.st);
    launch_features(stats, scalars, nl, nullptr, x, o.st);
    MG_HIP(hipMemcpyAsync(h_x, x, 4 * MLP_IN * nl, hipMemcpyDeviceToHost, o.st));
    MG_HIP(hipStreamSynchronize(o.st));
  });
}

mgard_status mgard_bin_widths(uint32_t ndim, const uint64_t* shape, const double* const* coords, mgard_dtype dtype,
                              double tol, const void* d_in, double* h_bins, uint32_t max_bins, double* h_tau_abs,
                              const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    const int es = dtype_size(dtype);
    (void)es;
    if (!d_in || !h_bins) fail(MGARD_ERR_ARG, "null pointer");
    if (!(tol > 0.0) || !std::isfinite(tol)) fail(MGARD_ERR_TOL, "tolerance must be positive and finite");
    if (o.alloc == MGARD_ALLOC_LEARNED) fail(MGARD_ERR_ARG, "the a-priori widths are PLAIN or COUNT");
    auto h = get_hierarchy(ndim, shape, coords);
    if ((uint32_t)h->L + 1 > max_bins) fail(MGARD_ERR_CAPACITY, "h_bins holds fewer entries than levels + 1");
    const uint64_t n = h->count(h->L);
    Workspace& ws = workspace();
    ws.reserve(carve_size<uint64_t>(4) + carve_size<double>(MAXL + 1) + carve_size<double>(8) +
               carve_size<char>(mass_norm_scratch_bytes()) + carve_size<double>(1) + 1024);
    Carver cv(ws.base());
    uint64_t* misc = cv.take<uint64_t>(4);
    double* bins = cv.take<double>(MAXL + 1);
    double* scalars = cv.take<double>(8);
    void* nscr = cv.take<char>(mass_norm_scratch_bytes());
    double* nrm2 = cv.take<double>(1);
    if (dtype == MGARD_F64)
      launch_maxabs<double>(static_cast<const double*>(d_in), n, misc, o.st);
    else
      launch_maxabs<float>(static_cast<const float*>(d_in), n, misc, o.st);
    if (o.norm == MGARD_NORM_S) {
      if (o.eb == MGARD_REL) {
        const double* bands = device_mass_table(*h, o.st);
        if (dtype == MGARD_F64)
          launch_mass_norm<double>(*h, bands, static_cast<const double*>(d_in), nscr, nrm2, o.st);
        else
          launch_mass_norm<float>(*h, bands, static_cast<const float*>(d_in), nscr, nrm2, o.st);
      }
      launch_bins_snorm(dtype == MGARD_F64 ? 1 : 0, misc, nrm2, tol, o.eb, h->L, snorm_args(*h, o.s), bins, scalars,
                        o.st);
    } else {
      BinArgs ba{};
      for (int l = 0; l <= h->L; ++l) {
        ba.K[l] = h->K[l];
        ba.counts[l] = (double)h->level_count[l];
      }
      launch_bins(dtype == MGARD_F64 ? 1 : 0, misc, tol, o.eb, h->S, h->L, o.alloc, ba, bins, scalars, o.st);
    }
    double hs[8];
    MG_HIP(hipMemcpyAsync(h_bins, bins, 8 * (h->L + 1), hipMemcpyDeviceToHost, o.st));
    MG_HIP(hipMemcpyAsync(hs, scalars, sizeof(hs), hipMemcpyDeviceToHost, o.st));
    MG_HIP(hipStreamSynchronize(o.st));
    if (hs[2] != 0.0) fail(MGARD_ERR_NONFINITE, "input holds NaN or infinity");
    if (hs[6] != 0.0) fail(MGARD_ERR_TOL, "tolerance below the rounding reserve or the quantizer's range");
    if (h_tau_abs) *h_tau_abs = hs[0];
  });
}

mgard_status mgard_l2_norm(uint32_t ndim, const uint64_t* shape, const double* const* coords, mgard_dtype dtype,
                           const void* d_in, double* h_norm, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    (void)dtype_size(dtype);
    if (!d_in || !h_norm) fail(MGARD_ERR_ARG, "null pointer");
    auto h = get_hierarchy(ndim, shape, coords);
    Workspace& ws = workspace();
    ws.reserve(carve_size<char>(mass_norm_scratch_bytes()) + carve_size<double>(1) + 1024);
    Carver cv(ws.base());
    void* nscr = cv.take<char>(mass_norm_scratch_bytes());
    double* nrm2 = cv.take<double>(1);
    const double* bands = device_mass_table(*h, o.st);
    if (dtype == MGARD_F64)
      launch_mass_norm<double>(*h, bands, static_cast<const double*>(d_in), nscr, nrm2, o.st);
    else
      launch_mass_norm<float>(*h, bands, static_cast<const float*>(d_in), nscr, nrm2, o.st);
    double v = 0.0;
    MG_HIP(hipMemcpyAsync(&v, nrm2, 8, hipMemcpyDeviceToHost, o.st));
    MG_HIP(hipStreamSynchronize(o.st));
    *h_norm = std::sqrt(v);
  });
}

mgard_status mgard_linf_error(mgard_dtype dtype, const void* d_a, const void* d_b, uint64_t n, double* h_err,
                              const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    (void)dtype_size(dtype);
    if (!d_a || !d_b || !h_err) fail(MGARD_ERR_ARG, "null pointer");
    Workspace& ws = workspace();
    ws.reserve(1024);
    auto* e = static_cast<unsigned long long*>(ws.base());
    if (dtype == MGARD_F64)
      launch_linf<double>(static_cast<const double*>(d_a), static_cast<const double*>(d_b), n, e, o.st);
    else
      launch_linf<float>(static_cast<const float*>(d_a), static_cast<const float*>(d_b), n, e, o.st);
    unsigned long long bits = 0;
    MG_HIP(hipMemcpyAsync(&bits, e, 8, hipMemcpyDeviceToHost, o.st));
    MG_HIP(hipStreamSynchronize(o.st));
    std::memcpy(h_err, &bits, 8);
  });
}

mgard_status mgard_mlp_forward(const float* d_params, const float* d_x, uint32_t batch, float* d_out,
                               float* d_cache, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    if (!d_params || !d_x || !d_out) fail(MGARD_ERR_ARG, "null pointer");
    if (batch == 0 || batch > (1u << 24)) fail(MGARD_ERR_ARG, "batch");
    const uint64_t B = batch;
    float* xn = d_cache;
    float* acts = d_cache ? d_cache + B * MLP_IN : nullptr;
    Workspace& ws = workspace();
    ws.reserve(carve_size<float>(B * MLP_IN) + carve_size<float>(2 * B * MLP_HID) + 1024);
    Carver cv(ws.base());
    if (!xn) xn = cv.take<float>(B * MLP_IN);
    float* tmp = cv.take<float>(2 * B * MLP_HID);
    mlp_normalize(d_x, d_params, (int)B, xn, o.st);
    mlp_forward(d_params, xn, (int)B, d_out, acts, tmp, o.st);
    MG_HIP(hipStreamSynchronize(o.st));
  });
}

mgard_status mgard_mlp_backward(const float* d_params, const float* d_cache, const float* d_dout, uint32_t batch,
                                float* d_grads, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    if (!d_params || !d_cache || !d_dout || !d_grads) fail(MGARD_ERR_ARG, "null pointer");
    if (batch == 0 || batch > (1u << 24)) fail(MGARD_ERR_ARG, "batch");
    const uint64_t B = batch;
    Workspace& ws = workspace();
    ws.reserve(carve_size<float>(2 * B * MLP_HID) + 1024);
    float* tmp = static_cast<float*>(ws.base());
    MG_HIP(hipMemsetAsync(d_grads, 0, 2 * MLP_IN * sizeof(float), o.st));
    mlp_backward(d_params, d_cache, d_cache + B * MLP_IN, d_dout, (int)B, d_grads, tmp, o.st);
    MG_HIP(hipStreamSynchronize(o.st));
  });
}

mgard_status mgard_mlp_mse(const float* d_pred, const float* d_target, uint32_t batch, float* d_dout,
                           double* h_loss, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    if (!d_pred || !d_target || !d_dout || !h_loss) fail(MGARD_ERR_ARG, "null pointer");
    if (batch == 0) fail(MGARD_ERR_ARG, "batch");
    Workspace& ws = workspace();
    ws.reserve(1024);
    double* dl = static_cast<double*>(ws.base());
    mlp_mse(d_pred, d_target, (int)batch, d_dout, dl, o.st);
    MG_HIP(hipMemcpyAsync(h_loss, dl, 8, hipMemcpyDeviceToHost, o.st));
    MG_HIP(hipStreamSynchronize(o.st));
  });
}

mgard_status mgard_mlp_adam(float* d_params, const float* d_grads, float* d_m, float* d_v, uint32_t step, float lr,
                            float beta1, float beta2, float eps, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    if (!d_params || !d_grads || !d_m || !d_v) fail(MGARD_ERR_ARG, "null pointer");
    if (step == 0) fail(MGARD_ERR_ARG, "Adam steps count from 1");
    const int off = 2 * MLP_IN;  // feature normalisation is not trained
    mlp_adam(d_params + off, d_grads + off, d_m + off, d_v + off, MLP_NPARAM - off, lr, beta1, beta2, eps,
             (int)step, o.st);
    MG_HIP(hipStreamSynchronize(o.st));
  });
}

uint64_t mgard_chunked_bound(uint32_t ndim, const uint64_t* shape, const double* const* coords, mgard_dtype dtype,
                             uint64_t slab_planes, const mgard_opts* opts) {
  uint64_t r = 0;
  mgard_status st = guard([&] {
    Opts o = read_opts(opts);
    (void)dtype_size(dtype);
    if (!shape || ndim < 1 || ndim > MAXD) fail(MGARD_ERR_SHAPE, "shape");
    r = chunked_bound(ndim, shape, coords, slab_planes, o);
  });
  return st == MGARD_OK ? r : 0;
}

mgard_status mgard_compress_chunked(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                                    mgard_dtype dtype, double tol, const void* h_in, uint64_t slab_planes,
                                    void* h_out, uint64_t out_capacity, uint64_t* out_bytes,
                                    const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    (void)dtype_size(dtype);
    if (!h_in || !h_out || !out_bytes || !shape) fail(MGARD_ERR_ARG, "null buffer");
    if (ndim < 1 || ndim > MAXD) fail(MGARD_ERR_SHAPE, "shape");
    if (!(tol > 0.0) || !std::isfinite(tol)) fail(MGARD_ERR_TOL, "tolerance must be positive and finite");
    if (o.alloc == MGARD_ALLOC_LEARNED) fail(MGARD_ERR_ARG, "chunked compression takes the plain or count allocation");
    if (o.norm == MGARD_NORM_S) fail(MGARD_ERR_ARG, "chunked compression bounds the L-infinity norm");
    if (dtype == MGARD_F32)
      compress_chunked_impl<float>(ndim, shape, coords, tol, static_cast<const float*>(h_in), slab_planes,
                                   static_cast<char*>(h_out), out_capacity, out_bytes, o);
    else
      compress_chunked_impl<double>(ndim, shape, coords, tol, static_cast<const double*>(h_in), slab_planes,
                                    static_cast<char*>(h_out), out_capacity, out_bytes, o);
  });
}

mgard_status mgard_decompress_chunked(const void* h_in, uint64_t in_bytes, void* h_out, uint64_t out_capacity,
                                      const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    if (!h_in || !h_out) fail(MGARD_ERR_ARG, "null buffer");
    const ChunkHead c = parse_chunked(static_cast<const uint8_t*>(h_in), in_bytes);
    uint64_t n = 1;
    for (uint32_t d = 0; d < c.ndim; ++d) n *= c.shape[d];
    if (out_capacity < n * (c.dtype ? 8 : 4)) fail(MGARD_ERR_CAPACITY, "output buffer too small");
    if (c.dtype)
      decompress_chunked_impl<double>(c, static_cast<const uint8_t*>(h_in), static_cast<double*>(h_out), o);
    else
      decompress_chunked_impl<float>(c, static_cast<const uint8_t*>(h_in), static_cast<float*>(h_out), o);
  });
}


// ------------------------------------------------------------------ lossless stage
uint64_t mgard_lossless_bound(uint64_t raw_bytes) { return zs_bound(raw_bytes); }

mgard_status mgard_lossless_encode(const void* d_in, uint64_t raw_bytes, void* d_out, uint64_t out_capacity,
                                   uint64_t* out_bytes, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    if ((!d_in && raw_bytes) || !d_out || !out_bytes) fail(MGARD_ERR_ARG, "null buffer");
    if (reinterpret_cast<uintptr_t>(d_in) % 4) fail(MGARD_ERR_ARG, "d_in must be 4-byte aligned");
    if (reinterpret_cast<uintptr_t>(d_out) % 8) fail(MGARD_ERR_ARG, "d_out must be 8-byte aligned");
    const uint64_t nch = (raw_bytes + 16383) / 16384;
    Workspace& aux = aux_workspace();
    aux.reserve(carve_size<uint32_t>(nch + 1) + 1024);
    Carver cv(aux.base());
    uint32_t* sizes = cv.take<uint32_t>(nch + 1);
    *out_bytes = zs_encode(d_in, raw_bytes, d_out, out_capacity, sizes, o.st);
  });
}

mgard_status mgard_lossless_decode(const void* d_in, uint64_t in_bytes, void* d_out, uint64_t out_capacity,
                                   uint64_t* raw_bytes, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    if (!d_in || !d_out || !raw_bytes) fail(MGARD_ERR_ARG, "null buffer");
    if (reinterpret_cast<uintptr_t>(d_in) % 8 || reinterpret_cast<uintptr_t>(d_out) % 4)
      fail(MGARD_ERR_ARG, "d_in must be 8-byte and d_out 4-byte aligned");
    uint8_t zh[24] = {0};
    const uint64_t got = std::min<uint64_t>(in_bytes, 24);
    MG_HIP(hipMemcpyAsync(zh, d_in, got, hipMemcpyDeviceToHost, o.st));
    MG_HIP(hipStreamSynchronize(o.st));
    uint64_t raw = 0, nch = 0;
    if (!zs_parse(zh, in_bytes, &raw, &nch)) fail(MGARD_ERR_FORMAT, "not a lossless container");
    *raw_bytes = raw;
    if (out_capacity < 4 * ((raw + 3) / 4)) fail(MGARD_ERR_CAPACITY, "output buffer too small");
    Workspace& aux = aux_workspace();
    aux.reserve(1024);
    uint32_t* status = static_cast<uint32_t*>(aux.base());
    zs_decode(d_in, in_bytes, raw, nch, d_out, status, o.st);
  });
}

// ------------------------------------------------------------------ refactoring
uint64_t mgard_refactor_bound(uint32_t ndim, const uint64_t* shape, const double* const* coords, mgard_dtype dtype,
                              uint32_t planes) {
  try {
    if (planes < 1 || planes > 32) return 0;
    (void)dtype_size(dtype);
    auto h = get_hierarchy(ndim, shape, coords);
    bool hc[MAXD] = {false, false, false, false};
    for (uint32_t d = 0; d < ndim; ++d) hc[d] = coords && coords[d];
    const RfLevels lv = rf_levels(*h, planes);
    return rf_meta_layout(*h, hc, planes, lv).total;
  } catch (...) {
    return 0;
  }
}

mgard_status mgard_refactor(uint32_t ndim, const uint64_t* shape, const double* const* coords, mgard_dtype dtype,
                            uint32_t planes, const void* d_in, void* d_out, uint64_t out_capacity, uint64_t* out_bytes,
                            const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    const int s = dtype_size(dtype);
    if (!d_in || !d_out || !out_bytes) fail(MGARD_ERR_ARG, "null buffer");
    if (planes < 1 || planes > 32) fail(MGARD_ERR_ARG, "planes must be 1..32");
    auto h = get_hierarchy(ndim, shape, coords);
    bool hc[MAXD] = {false, false, false, false};
    for (uint32_t d = 0; d < ndim; ++d) hc[d] = coords && coords[d];
    const RfLevels lv = rf_levels(*h, planes);
    const RfMetaLayout ml = rf_meta_layout(*h, hc, planes, lv);
    *out_bytes = ml.total;
    if (out_capacity < ml.total) fail(MGARD_ERR_CAPACITY, "output capacity below mgard_refactor_bound");
    const bool f64 = dtype == MGARD_F64;
    const uint64_t n = h->count(h->L);
    const void* table = device_table(*h, f64, o.st);
    const double* bands = device_mass_table(*h, o.st);
    const uint64_t dbytes = f64 ? decompose_scratch_bytes<double>(*h) : decompose_scratch_bytes<float>(*h);
    Workspace& ws = workspace();
    ws.reserve(carve_size<char>(n * s) + carve_size<char>(dbytes) + carve_size<uint64_t>(MAXL + 2) +
               carve_size<uint64_t>(1) + carve_size<double>(1) + carve_size<char>(mass_norm_scratch_bytes()) +
               carve_size<int>(MAXL + 2) + 4096);
    Carver cv(ws.base());
    char* cstream = cv.take<char>(n * s);
    void* dscratch = cv.take<char>(dbytes);
    uint64_t* lbits = cv.take<uint64_t>(MAXL + 2);
    uint64_t* ubits = cv.take<uint64_t>(1);
    double* nrm2 = cv.take<double>(1);
    void* nscr = cv.take<char>(mass_norm_scratch_bytes());
    int* exps = cv.take<int>(MAXL + 2);
    const std::vector<uint8_t> hb = rf_header(*h, coords, f64 ? 1 : 0, planes, lv, ml);
    char* out = static_cast<char*>(d_out);
    MG_HIP(hipMemcpyAsync(out, hb.data(), hb.size(), hipMemcpyHostToDevice, o.st));
    uint64_t hbits = 0;
    if (f64)
      launch_maxabs<double>(static_cast<const double*>(d_in), n, ubits, o.st);
    else
      launch_maxabs<float>(static_cast<const float*>(d_in), n, ubits, o.st);
    MG_HIP(hipMemcpyAsync(&hbits, ubits, 8, hipMemcpyDeviceToHost, o.st));
    MG_HIP(hipStreamSynchronize(o.st));
    if (hbits >= (f64 ? 0x7ff0000000000000ull : 0x7f800000ull)) fail(MGARD_ERR_NONFINITE, "NaN or infinity");
    uint32_t* seg = reinterpret_cast<uint32_t*>(out + ml.meta_bytes);
    uint32_t* R = reinterpret_cast<uint32_t*>(out + ml.R_off);
    if (f64) {
      launch_mass_norm<double>(*h, bands, static_cast<const double*>(d_in), nscr, nrm2, o.st);
      decompose<double>(*h, static_cast<const double*>(table), static_cast<const double*>(d_in),
                        reinterpret_cast<double*>(cstream), nullptr, dscratch, o.st);
      for (int l = 0; l <= h->L; ++l)
        launch_maxabs<double>(reinterpret_cast<const double*>(cstream) + h->level_off[l], h->level_count[l],
                              lbits + l, o.st);
    } else {
      launch_mass_norm<float>(*h, bands, static_cast<const float*>(d_in), nscr, nrm2, o.st);
      decompose<float>(*h, static_cast<const float*>(table), static_cast<const float*>(d_in),
                       reinterpret_cast<float*>(cstream), nullptr, dscratch, o.st);
      for (int l = 0; l <= h->L; ++l)
        launch_maxabs<float>(reinterpret_cast<const float*>(cstream) + h->level_off[l], h->level_count[l],
                             lbits + l, o.st);
    }
    launch_rf_meta(lbits, ubits, nrm2, f64 ? 1 : 0, h->L + 1, exps, out, ml.exp_off, o.st);
    if (f64)
      launch_rf_planes<double>(reinterpret_cast<const double*>(cstream), lv, (int)planes, exps, seg, R, o.st);
    else
      launch_rf_planes<float>(reinterpret_cast<const float*>(cstream), lv, (int)planes, exps, seg, R, o.st);
    MG_HIP(hipStreamSynchronize(o.st));
  });
}

mgard_status mgard_refactor_inspect(const void* h_meta, uint64_t bytes, uint64_t* meta_bytes, uint32_t* levels,
                                    uint32_t* planes, uint64_t* total_bytes) {
  return guard([&] {
    if (!h_meta || !meta_bytes) fail(MGARD_ERR_ARG, "null pointer");
    RfParsed P;
    if (!rf_parse(static_cast<const uint8_t*>(h_meta), bytes, P)) {
      *meta_bytes = P.need;
      fail(MGARD_ERR_CAPACITY, "more metadata bytes needed");
    }
    *meta_bytes = P.meta_bytes;
    if (levels) *levels = (uint32_t)P.L;
    if (planes) *planes = (uint32_t)P.B;
    if (total_bytes) *total_bytes = P.meta_bytes + P.loff[P.L + 1];
  });
}

mgard_status mgard_refactor_request(const void* h_meta, uint64_t bytes, double tol, const uint32_t* h_have,
                                    uint32_t* h_want, uint32_t max_levels, double* h_estimate,
                                    const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    if (!h_meta || !h_want) fail(MGARD_ERR_ARG, "null pointer");
    if (!(tol > 0.0) || !std::isfinite(tol)) fail(MGARD_ERR_TOL, "tolerance must be positive and finite");
    RfParsed P;
    if (!rf_parse(static_cast<const uint8_t*>(h_meta), bytes, P)) fail(MGARD_ERR_CAPACITY, "truncated metadata");
    if (max_levels < (uint32_t)P.L + 1) fail(MGARD_ERR_CAPACITY, "h_want shorter than levels + 1");
    const double* cp[MAXD];
    auto h = get_hierarchy((uint32_t)P.ndim, P.shape, P.coord_ptrs(cp));
    rf_check_layout(P, *h, nullptr);
    const std::vector<uint32_t> k = rf_request(P, *h, tol, o.eb, o.norm, o.s, h_have, h_estimate);
    for (int l = 0; l <= P.L; ++l) h_want[l] = k[l];
  });
}

mgard_status mgard_refactor_ranges(const void* h_meta, uint64_t bytes, const uint32_t* h_have,
                                   const uint32_t* h_want, uint32_t n_levels, uint64_t* h_offsets,
                                   uint64_t* h_lengths, uint32_t* count) {
  return guard([&] {
    if (!h_meta || !h_want || !h_offsets || !h_lengths || !count) fail(MGARD_ERR_ARG, "null pointer");
    RfParsed P;
    if (!rf_parse(static_cast<const uint8_t*>(h_meta), bytes, P)) fail(MGARD_ERR_CAPACITY, "truncated metadata");
    if (n_levels != (uint32_t)P.L + 1) fail(MGARD_ERR_ARG, "plane arrays must hold levels + 1 entries");
    uint32_t c = 0;
    for (int l = 0; l <= P.L; ++l) {
      const uint32_t hv = h_have ? h_have[l] : 0u, wt = h_want[l];
      if (hv > (uint32_t)P.B || wt > (uint32_t)P.B) fail(MGARD_ERR_ARG, "more planes than stored");
      if (wt <= hv) continue;
      const uint64_t pb = (P.loff[l + 1] - P.loff[l]) / (uint64_t)(P.B + 1);
      const uint64_t first = hv == 0 ? 0 : hv + 1, last = (uint64_t)wt + 1;  // slot 0: the sign plane
      h_offsets[c] = P.meta_bytes + P.loff[l] + first * pb;
      h_lengths[c] = (last - first) * pb;
      ++c;
    }
    *count = c;
  });
}

mgard_status mgard_reconstruct(const void* d_in, uint64_t in_bytes, const uint32_t* h_planes, uint32_t n_levels,
                               void* d_out, uint64_t out_capacity, const mgard_opts* opts) {
  return guard([&] {
    Opts o = read_opts(opts);
    if (!d_in || !h_planes || !d_out) fail(MGARD_ERR_ARG, "null buffer");
    std::vector<uint8_t> hb(256);
    RfParsed P;
    for (;;) {
      const uint64_t got = std::min<uint64_t>(hb.size(), in_bytes);
      MG_HIP(hipMemcpyAsync(hb.data(), d_in, got, hipMemcpyDeviceToHost, o.st));
      MG_HIP(hipStreamSynchronize(o.st));
      if (rf_parse(hb.data(), got, P)) break;
      if (P.need > in_bytes) fail(MGARD_ERR_FORMAT, "truncated refactored buffer");
      hb.resize(P.need);
    }
    if (n_levels != (uint32_t)P.L + 1) fail(MGARD_ERR_ARG, "h_planes must hold levels + 1 entries");
    const double* cp[MAXD];
    auto h = get_hierarchy((uint32_t)P.ndim, P.shape, P.coord_ptrs(cp));
    RfLevels lv;
    rf_check_layout(P, *h, &lv);
    if (in_bytes < P.meta_bytes + P.loff[P.L + 1]) fail(MGARD_ERR_FORMAT, "truncated refactored buffer");
    const uint64_t n = h->count(h->L);
    const int s = P.dtype ? 8 : 4;
    if (out_capacity < n * s) fail(MGARD_ERR_CAPACITY, "output buffer too small");
    for (int l = 0; l <= P.L; ++l) {
      if (h_planes[l] > (uint32_t)P.B) fail(MGARD_ERR_ARG, "more planes requested than stored");
      lv.planes[l] = (int)h_planes[l];
      lv.exp[l] = P.exps[l];
    }
    const bool f64 = P.dtype == 1;
    const void* table = device_table(*h, f64, o.st);
    const uint64_t rbytes = f64 ? recompose_scratch_bytes<double>(*h) : recompose_scratch_bytes<float>(*h);
    Workspace& ws = workspace();
    ws.reserve(carve_size<char>(n * s) + carve_size<char>(rbytes) + 1024);
    Carver cv(ws.base());
    char* cstream = cv.take<char>(n * s);
    void* rscratch = cv.take<char>(rbytes);
    const uint32_t* seg = reinterpret_cast<const uint32_t*>(static_cast<const char*>(d_in) + P.meta_bytes);
    if (f64) {
      launch_rf_decode<double>(seg, lv, P.B, reinterpret_cast<double*>(cstream), o.st);
      recompose<double>(*h, static_cast<const double*>(table), reinterpret_cast<const double*>(cstream), nullptr,
                        static_cast<double*>(d_out), rscratch, o.st);
    } else {
      launch_rf_decode<float>(seg, lv, P.B, reinterpret_cast<float*>(cstream), o.st);
      recompose<float>(*h, static_cast<const float*>(table), reinterpret_cast<const float*>(cstream), nullptr,
                       static_cast<float*>(d_out), rscratch, o.st);
    }
    MG_HIP(hipStreamSynchronize(o.st));
  });
}

}  // extern "C"
