// Refactoring into bitplane precision segments (gfx950).
//
// Paper Sec. 2: the refactoring module encodes the multilevel coefficients
// into precision segments of different significance per level by bitplane
// encoding, accumulates the error each segment removes, and recomposition
// fetches segments greedily by those error estimators (Sec. 3, second
// listing: request a tolerance, fetch the needed components, reconstruct).
//
// Per level l (stream range [off_l, off_l + n_l)) with exponent e_l
// (max|c| = f 2^e_l, 1/2 <= f < 1) and B planes:
//   m = floor(|c| 2^(B - e_l)) < 2^B, sign = c < 0;
//   segments: the sign plane, then planes k = 0..B-1 holding bit B-1-k of m,
//   coefficient i of the level at bit 31 - i%32 of word i/32, W_l words each;
//   R_l[k] = max (m mod 2^(B-k)), k = 0..B (the residual table);
//   reconstruction from k planes: c^ = T(+-(m with its low B-k bits cleared)
//   2^(e_l - B)).
//
// Kernels, one wavefront per 2048 consecutive coefficients of a level:
//   k_rf_planes  lane L ends up holding word L of each of the wavefront's 64
//                plane words: iteration j turns the bits of coefficients
//                64j .. 64j+63 into one ballot per plane, whose two halves
//                lanes 2j and 2j+1 keep (bit-reversed); the words are then stored
//                coalesced; the residual maxima reduce across the wavefront
//                and go to R with one atomic max per plane;
//   k_rf_decode  the inverse: lane L loads word L of every plane it needs,
//                iteration j reads the two words of coefficients
//                64j .. 64j+63 from lanes 2j and 2j+1 as scalars.
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace mg {

namespace {

constexpr int RF_T = 256;               // threads per block: four wavefronts
constexpr int RF_COEF = 2048;           // coefficients per wavefront
constexpr int RF_NOEXP = -2147483647 - 1;

__device__ inline int rf_level_of(const RfLevels& lv, uint64_t gw) {
  int l = -1;
  for (int k = 0; k < lv.nlev; ++k)
    if (gw >= lv.wave0[k]) l = k;
  return l;
}

template <typename T>
__global__ void __launch_bounds__(RF_T) k_rf_planes(const T* __restrict__ cs, RfLevels lv, int B,
                                                    const int* __restrict__ exps, uint32_t* __restrict__ seg,
                                                    uint32_t* __restrict__ R) {
  const uint64_t gw = (uint64_t)blockIdx.x * (RF_T / 64) + (threadIdx.x >> 6);
  if (gw >= lv.wave0[lv.nlev]) return;
  const int l = rf_level_of(lv, gw);
  const uint64_t w = gw - lv.wave0[l];
  const uint64_t n = lv.n[l];
  const int lane = threadIdx.x & 63;
  const int e = exps[l];
  const T* c = cs + lv.off[l];
  // every load of the wavefront's 2048 coefficients before any is used
  T v[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) v[j] = c[min(w * RF_COEF + 64 * j + lane, n - 1)];
  uint32_t pw[32], sw = 0, r[33];
#pragma unroll
  for (int k = 0; k < 32; ++k) pw[k] = 0;
#pragma unroll
  for (int k = 0; k < 33; ++k) r[k] = 0;
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const uint64_t i = w * RF_COEF + 64 * j + lane;
    const bool valid = i < n;
    const double a = fabs((double)v[j]);
    const uint32_t m = (valid && e != RF_NOEXP) ? (uint32_t)floor(ldexp(a, B - e)) : 0u;
    const bool neg = valid && v[j] < T(0);
    const bool lo_lane = lane == 2 * j, hi_lane = lane == 2 * j + 1;
    // a ballot has lane i at bit i; a plane word has coefficient i at bit
    // 31 - i, hence the bit reversal
    {
      const uint64_t bm = __ballot(neg);
      sw = lo_lane ? __brev((uint32_t)bm) : hi_lane ? __brev((uint32_t)(bm >> 32)) : sw;
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      if (k >= B) break;
      const uint64_t bm = __ballot(((m >> (B - 1 - k)) & 1u) != 0u);
      pw[k] = lo_lane ? __brev((uint32_t)bm) : hi_lane ? __brev((uint32_t)(bm >> 32)) : pw[k];
    }
#pragma unroll
    for (int k = 0; k <= 32; ++k) {
      if (k > B) break;
      const uint32_t mask = B - k >= 32 ? 0xffffffffu : ((1u << (B - k)) - 1u);
      const uint32_t x = m & mask;
      r[k] = x > r[k] ? x : r[k];
    }
  }
  // words 64w + lane of the level's planes (the last wavefront of a level may
  // hold fewer than 64)
  const uint64_t W = lv.words[l];
  const uint64_t wi = w * 64 + lane;
  uint32_t* base = seg + lv.word_off[l];
  if (wi < W) {
    base[wi] = sw;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      if (k >= B) break;
      base[(uint64_t)(1 + k) * W + wi] = pw[k];
    }
  }
#pragma unroll
  for (int k = 0; k <= 32; ++k) {
    if (k > B) break;
    uint32_t x = r[k];
#pragma unroll
    for (int s = 32; s; s >>= 1) {
      const uint32_t o = __shfl_xor(x, s);
      x = o > x ? o : x;
    }
    if (lane == 0 && x) atomicMax(&R[l * (B + 1) + k], x);
  }
}

// e_l from the per-level max |c| bit patterns, and the header's dynamic
// fields: max|u|, ||u||, exponents (int32 at hdr_exp).
__global__ void k_rf_meta(const uint64_t* __restrict__ lbits, const uint64_t* __restrict__ ubits,
                          const double* __restrict__ nrm2, int f64, int nlev, int* __restrict__ exps,
                          unsigned char* __restrict__ hdr, uint64_t hdr_exp) {
  const int l = threadIdx.x;
  auto value = [&](uint64_t b) -> double {
    if (f64) return __longlong_as_double((long long)b);
    return (double)__uint_as_float((uint32_t)b);
  };
  if (l < nlev) {
    const double mx = value(lbits[l]);
    int e = RF_NOEXP;
    if (mx > 0.0) frexp(mx, &e);
    exps[l] = e;
    int32_t* he = reinterpret_cast<int32_t*>(hdr + hdr_exp);
    he[l] = e;
  }
  if (l == 0) {
    double* hd = reinterpret_cast<double*>(hdr + 16);
    hd[0] = value(ubits[0]);
    hd[1] = sqrt(nrm2[0]);
  }
}

template <typename T>
__global__ void __launch_bounds__(RF_T) k_rf_decode(const uint32_t* __restrict__ seg, RfLevels lv, int B,
                                                    T* __restrict__ cs) {
  const uint64_t gw = (uint64_t)blockIdx.x * (RF_T / 64) + (threadIdx.x >> 6);
  if (gw >= lv.wave0[lv.nlev]) return;
  const int l = rf_level_of(lv, gw);
  const uint64_t w = gw - lv.wave0[l];
  const uint64_t n = lv.n[l];
  const int lane = threadIdx.x & 63;
  const int e = lv.exp[l];
  const int kl = (e == RF_NOEXP) ? 0 : lv.planes[l];
  T* out = cs + lv.off[l];
  if (kl == 0) {
#pragma unroll 4
    for (int j = 0; j < 32; ++j) {
      const uint64_t i = w * RF_COEF + 64 * j + lane;
      if (i < n) out[i] = T(0);
    }
    return;
  }
  const uint64_t W = lv.words[l];
  const uint64_t wi = min(w * 64 + lane, W - 1);
  const uint32_t* base = seg + lv.word_off[l];
  const uint32_t sw = base[wi];
  uint32_t pw[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) pw[k] = k < kl ? base[(uint64_t)(1 + k) * W + wi] : 0u;
  const int sh = 31 - (lane & 31);
  const bool upper = lane >= 32;
#pragma unroll 2
  for (int j = 0; j < 32; ++j) {
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      if (k >= kl) break;
      const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)pw[k], 2 * j);
      const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)pw[k], 2 * j + 1);
      m |= (((upper ? hi : lo) >> sh) & 1u) << (B - 1 - k);
    }
    const uint32_t slo = (uint32_t)__builtin_amdgcn_readlane((int)sw, 2 * j);
    const uint32_t shi = (uint32_t)__builtin_amdgcn_readlane((int)sw, 2 * j + 1);
    const bool neg = (((upper ? shi : slo) >> sh) & 1u) != 0u;
    const double mag = ldexp((double)m, e - B);
    const T val = static_cast<T>(neg ? -mag : mag);
    const uint64_t i = w * RF_COEF + 64 * j + lane;
    if (i < n) out[i] = val;
  }
}

}  // namespace

RfLevels rf_levels(const Hierarchy& h, uint32_t B) {
  RfLevels lv{};
  lv.nlev = h.L + 1;
  uint64_t wave = 0, words = 0;
  for (int l = 0; l <= h.L; ++l) {
    lv.off[l] = h.level_off[l];
    lv.n[l] = h.level_count[l];
    lv.words[l] = (h.level_count[l] + 31) / 32;
    lv.word_off[l] = words;
    words += (uint64_t)(B + 1) * lv.words[l];
    lv.wave0[l] = wave;
    wave += (h.level_count[l] + RF_COEF - 1) / RF_COEF;
  }
  lv.wave0[h.L + 1] = wave;
  lv.word_off[h.L + 1] = words;
  return lv;
}


// ------------------------------------------------------------------ host side
// Metadata layout (little-endian): 'MGRF', u16 version 1, u8 dtype, u8 ndim,
// u8 planes, u8 coordinate flags, u16 0, u32 L, f64 max|u|, f64 ||u||,
// u64 shape[ndim], f64 coordinates of each flagged dimension, i32
// exponent[L+1] (-2^31: an all-zero level), u32 R[(L+1)(B+1)], u64 level
// byte offsets in the segment area [L+2], zero padding to 8 bytes; then the
// segment area.
constexpr uint16_t kRfVersion = 1;
constexpr uint64_t kRfFixed = 32;

RfMetaLayout rf_meta_layout(const Hierarchy& h, const bool* has_coords, uint32_t B, const RfLevels& lv) {
  RfMetaLayout m{};
  const int pad = MAXD - h.D;
  uint64_t pos = kRfFixed + 8 * (uint64_t)h.D;
  for (int d = 0; d < h.D; ++d)
    if (has_coords[d]) pos += 8 * (uint64_t)h.shape[d + pad];
  m.exp_off = pos;
  pos += 4 * (uint64_t)(h.L + 1);
  m.R_off = pos;
  pos += 4 * (uint64_t)(h.L + 1) * (B + 1);
  m.loff_off = pos;
  pos += 8 * (uint64_t)(h.L + 2);
  m.meta_bytes = (pos + 7) & ~uint64_t(7);
  m.total = m.meta_bytes + 4 * lv.word_off[h.L + 1];
  return m;
}

std::vector<uint8_t> rf_header(const Hierarchy& h, const double* const* coords, int dtype, uint32_t B,
                               const RfLevels& lv, const RfMetaLayout& m) {
  std::vector<uint8_t> b(m.meta_bytes, 0);
  std::memcpy(&b[0], "MGRF", 4);
  std::memcpy(&b[4], &kRfVersion, 2);
  b[6] = (uint8_t)dtype;
  b[7] = (uint8_t)h.D;
  b[8] = (uint8_t)B;
  uint8_t flags = 0;
  for (int d = 0; d < h.D; ++d)
    if (coords && coords[d]) flags |= (uint8_t)(1u << d);
  b[9] = flags;
  const uint32_t L = (uint32_t)h.L;
  std::memcpy(&b[12], &L, 4);
  const int pad = MAXD - h.D;
  uint64_t pos = kRfFixed;
  for (int d = 0; d < h.D; ++d) {
    const uint64_t v = (uint64_t)h.shape[d + pad];
    std::memcpy(&b[pos], &v, 8);
    pos += 8;
  }
  for (int d = 0; d < h.D; ++d)
    if (coords && coords[d]) {
      std::memcpy(&b[pos], coords[d], 8 * (uint64_t)h.shape[d + pad]);
      pos += 8 * (uint64_t)h.shape[d + pad];
    }
  for (int l = 0; l <= h.L + 1; ++l) {
    const uint64_t v = 4 * lv.word_off[l];
    std::memcpy(&b[m.loff_off + 8 * (uint64_t)l], &v, 8);
  }
  return b;
}

bool rf_parse(const uint8_t* b, uint64_t bytes, RfParsed& P) {
  P = RfParsed{};
  if (bytes < kRfFixed) {
    P.need = kRfFixed;
    return false;
  }
  if (std::memcmp(b, "MGRF", 4) != 0) fail(MGARD_ERR_FORMAT, "not a refactored buffer");
  uint16_t ver = 0;
  std::memcpy(&ver, b + 4, 2);
  if (ver != kRfVersion) fail(MGARD_ERR_FORMAT, "unsupported refactoring version");
  P.dtype = b[6];
  P.ndim = b[7];
  P.B = b[8];
  const uint8_t flags = b[9];
  uint32_t L = 0;
  std::memcpy(&L, b + 12, 4);
  if (P.dtype > 1 || P.ndim < 1 || P.ndim > MAXD || P.B < 1 || P.B > 32 || L > MAXL || (flags >> P.ndim))
    fail(MGARD_ERR_FORMAT, "malformed refactoring metadata");
  P.L = (int)L;
  std::memcpy(&P.maxabs, b + 16, 8);
  std::memcpy(&P.l2norm, b + 24, 8);
  uint64_t pos = kRfFixed;
  if (bytes < pos + 8 * (uint64_t)P.ndim) {
    P.need = pos + 8 * (uint64_t)P.ndim;
    return false;
  }
  for (int d = 0; d < P.ndim; ++d) {
    std::memcpy(&P.shape[d], b + pos, 8);
    pos += 8;
    if (P.shape[d] == 0 || P.shape[d] > (1ull << 40)) fail(MGARD_ERR_FORMAT, "malformed shape");
    P.has_coords[d] = (flags >> d) & 1;
  }
  uint64_t need = pos;
  for (int d = 0; d < P.ndim; ++d)
    if (P.has_coords[d]) need += 8 * P.shape[d];
  need += 4 * (uint64_t)(P.L + 1) * (P.B + 2) + 8 * (uint64_t)(P.L + 2);
  need = (need + 7) & ~uint64_t(7);
  if (bytes < need) {
    P.need = need;
    return false;
  }
  P.coords.assign(P.ndim, {});
  for (int d = 0; d < P.ndim; ++d)
    if (P.has_coords[d]) {
      P.coords[d].resize(P.shape[d]);
      std::memcpy(P.coords[d].data(), b + pos, 8 * P.shape[d]);
      pos += 8 * P.shape[d];
    }
  P.exps.resize(P.L + 1);
  std::memcpy(P.exps.data(), b + pos, 4 * (uint64_t)(P.L + 1));
  pos += 4 * (uint64_t)(P.L + 1);
  P.R.resize((uint64_t)(P.L + 1) * (P.B + 1));
  std::memcpy(P.R.data(), b + pos, 4 * P.R.size());
  pos += 4 * P.R.size();
  P.loff.resize(P.L + 2);
  std::memcpy(P.loff.data(), b + pos, 8 * (uint64_t)(P.L + 2));
  P.meta_bytes = need;
  for (int l = 0; l <= P.L; ++l)
    if (P.exps[l] != RF_NOEXP && (P.exps[l] < -1100 || P.exps[l] > 1100))
      fail(MGARD_ERR_FORMAT, "malformed level exponent");
  return true;
}

const double* const* RfParsed::coord_ptrs(const double** buf) const {
  bool any = false;
  for (int d = 0; d < ndim; ++d) {
    buf[d] = has_coords[d] ? coords[d].data() : nullptr;
    any = any || has_coords[d];
  }
  return any ? buf : nullptr;
}

void rf_check_layout(const RfParsed& P, const Hierarchy& h, RfLevels* lv_out) {
  if (h.L != P.L) fail(MGARD_ERR_FORMAT, "level count does not match the shape");
  const RfLevels lv = rf_levels(h, (uint32_t)P.B);
  for (int l = 0; l <= P.L + 1; ++l)
    if (P.loff[l] != 4 * lv.word_off[l]) fail(MGARD_ERR_FORMAT, "segment offsets do not match the shape");
  if (lv_out) *lv_out = lv;
}

// The greedy retrieval of the oracle, in the same float64 expressions and order.
std::vector<uint32_t> rf_request(const RfParsed& P, const Hierarchy& h, double tol, int eb, int norm, double s,
                                 const uint32_t* have, double* estimate) {
  const int L = P.L, B = P.B;
  const double eps = P.dtype ? 2.220446049250313e-16 : 1.1920928955078125e-07;
  std::vector<std::vector<double>> E(L + 1, std::vector<double>(B + 1, 0.0));
  for (int l = 0; l <= L; ++l) {
    const int e = P.exps[l];
    if (e == RF_NOEXP) continue;
    for (int k = 0; k <= B; ++k) {
      double v = std::ldexp((double)P.R[(uint64_t)l * (B + 1) + k] + 1.0, e - B);
      if (k > 0) v += std::ldexp(eps, e);
      E[l][k] = v;
    }
  }
  std::vector<double> w(L + 1);
  const double rho = 4.0 * (L + 1) * eps * P.maxabs;
  double reserve = rho;
  if (norm == MGARD_NORM_LINF) {
    w[0] = 1.0;
    for (int l = 1; l <= L; ++l) w[l] = 1.0 + h.K[l];
  } else {
    for (int l = 0; l <= L; ++l) w[l] = std::pow(2.0, 2.0 * s * l) * h.W[l];
    reserve = rho * snorm_args(h, s).reserve;
  }
  std::vector<double> pb(L + 1);
  for (int l = 0; l <= L; ++l) pb[l] = (double)(4 * ((h.level_count[l] + 31) / 32));
  auto term = [&](int l, int k) {
    const double e = E[l][k];
    return norm == MGARD_NORM_LINF ? w[l] * e : w[l] * e * e;
  };
  std::vector<uint32_t> k(L + 1, 0);
  if (have)
    for (int l = 0; l <= L; ++l) {
      if (have[l] > (uint32_t)B) fail(MGARD_ERR_ARG, "held planes above the plane count");
      k[l] = have[l];
    }
  auto est = [&]() {
    double tot = 0.0;
    for (int l = 0; l <= L; ++l) tot += term(l, (int)k[l]);
    return reserve + (norm == MGARD_NORM_LINF ? tot : std::sqrt(tot));
  };
  double tau = tol;
  if (eb == MGARD_REL) {
    if (norm == MGARD_NORM_LINF)
      tau = tol * P.maxabs;
    else {
      if (s != 0.0) fail(MGARD_ERR_ARG, "a relative s-norm bound needs s = 0");
      tau = tol * P.l2norm;
    }
  }
  while (est() > tau) {
    int best = -1;
    double best_ratio = 0.0;
    for (int l = 0; l <= L; ++l) {
      if ((int)k[l] >= B || P.exps[l] == RF_NOEXP) continue;
      const double gain = term(l, (int)k[l]) - term(l, (int)k[l] + 1);
      const double ratio = gain / (pb[l] * (k[l] == 0 ? 2.0 : 1.0));
      if (best < 0 || ratio > best_ratio) {
        best = l;
        best_ratio = ratio;
      }
    }
    if (best < 0) break;
    ++k[best];
  }
  if (estimate) *estimate = est();
  return k;
}

template <typename T>
void launch_rf_planes(const T* cs, const RfLevels& lv, int B, const int* exps, uint32_t* seg, uint32_t* R,
                      hipStream_t st) {
  const uint64_t waves = lv.wave0[lv.nlev];
  if (!waves) return;
  KernelTimer kt("rf_planes", st);
  hipLaunchKernelGGL(k_rf_planes<T>, dim3((unsigned)((waves + 3) / 4)), dim3(RF_T), 0, st, cs, lv, B, exps, seg, R);
  MG_HIP(hipGetLastError());
}

void launch_rf_meta(const uint64_t* lbits, const uint64_t* ubits, const double* nrm2, int f64, int nlev, int* exps,
                    void* hdr, uint64_t hdr_exp, hipStream_t st) {
  hipLaunchKernelGGL(k_rf_meta, dim3(1), dim3(64), 0, st, lbits, ubits, nrm2, f64, nlev, exps,
                     static_cast<unsigned char*>(hdr), hdr_exp);
  MG_HIP(hipGetLastError());
}

template <typename T>
void launch_rf_decode(const uint32_t* seg, const RfLevels& lv, int B, T* cs, hipStream_t st) {
  const uint64_t waves = lv.wave0[lv.nlev];
  if (!waves) return;
  KernelTimer kt("rf_decode", st);
  hipLaunchKernelGGL(k_rf_decode<T>, dim3((unsigned)((waves + 3) / 4)), dim3(RF_T), 0, st, seg, lv, B, cs);
  MG_HIP(hipGetLastError());
}

template void launch_rf_planes<float>(const float*, const RfLevels&, int, const int*, uint32_t*, uint32_t*,
                                      hipStream_t);
template void launch_rf_planes<double>(const double*, const RfLevels&, int, const int*, uint32_t*, uint32_t*,
                                       hipStream_t);
template void launch_rf_decode<float>(const uint32_t*, const RfLevels&, int, float*, hipStream_t);
template void launch_rf_decode<double>(const uint32_t*, const RfLevels&, int, double*, hipStream_t);

}  // namespace mg
