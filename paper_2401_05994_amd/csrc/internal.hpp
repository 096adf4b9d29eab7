// Internal declarations shared by the host orchestration and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mgard_hip.h"
#include "launch.hpp"

namespace mg {

constexpr int MAXD = 4;    // dimensions handled by the kernels (leading slots padded)
constexpr int MAXL = 39;   // levels that fit in mgard_info::bin_width

struct Failure {
  mgard_status code;
  std::string msg;
};
[[noreturn]] void fail(mgard_status code, const std::string& msg);

#define MG_HIP(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) ::mg::fail(MGARD_ERR_DEVICE, std::string(#call) + ": " +        \
                                                        hipGetErrorString(e_));           \
  } while (0)

// ----------------------------------------------------------------- timing
// Scoped HIP-event timer around one launch (active only after mgard_timing(1)).
class KernelTimer {
 public:
  KernelTimer(const char* name, hipStream_t st);
  ~KernelTimer();
  KernelTimer(const KernelTimer&) = delete;
  KernelTimer& operator=(const KernelTimer&) = delete;

 private:
  hipStream_t st_;
  int idx_;
};
bool timing_enabled();
void timing_set(int on);
void timing_pause(bool paused);  // this thread only: no records while set (graph capture)
std::string timing_report();

// ----------------------------------------------------------------- hierarchy
// Per level l (1..L) and decomposed dimension d, the FP64 operator constants
// that take grid l to grid l-1 along d (see hierarchy.cpp for the formulas).
struct DimOps {
  int nf = 0, nc = 0;
  std::vector<double> wl, wr;      // interpolation weights, indexed by fine index (0 at coarse)
  std::vector<double> ma, mb, mc;  // fine mass matrix bands
  std::vector<double> rl, rr;      // restriction weights per coarse node
  std::vector<double> ta, tr, tcp; // Thomas factors of the coarse mass matrix
  double norm_inf = 0.0;           // || T^-1 P^T M ||_inf
};

// Offsets (in elements) of one (level, dim)'s arrays inside the device table.
struct DevDim {
  uint64_t wl, wr, ma, mb, mc, rl, rr, ta, tr, tcp;
};

struct Hierarchy {
  int D = 0;                          // user dimensions
  std::array<int64_t, MAXD> shape{};  // slot layout: user dim d sits in slot d + (MAXD - D)
  std::array<bool, MAXD> active{};    // decomposed slots
  int L = 0;
  std::vector<std::array<int64_t, MAXD>> sizes;     // sizes[l][slot], l = 0..L
  std::vector<std::array<DimOps, MAXD>> ops;        // ops[l][slot], l = 1..L
  std::vector<std::array<DevDim, MAXD>> devoff;     // device-table offsets
  std::vector<double> K;                            // K[l], K[0] = 0
  double S = 1.0;                                   // 1 + sum_l (1 + K_l)
  std::vector<uint64_t> level_count;                // stream entries per level
  std::vector<uint64_t> level_off;                  // L + 2 entries
  std::vector<double> table;                        // concatenated FP64 constants
  void* dev_table[2] = {nullptr, nullptr};          // table cast to float / double
  int dev_id[2] = {-1, -1};
  // per level l, 80 entries at l*80: sub-grid offsets [16], then C-order strides [16][4]
  std::vector<uint64_t> itab;
  void* dev_itab = nullptr;
  int dev_itab_id = -1;
  // s-norm bound: W[l], the hat-function integrals of level l's new nodes (all
  // nodes at l = 0); the finest grid's mass bands per decomposed slot (a, b, c,
  // shape[s] each, at mass_off[s] of mass_table), uploaded in float64
  std::vector<double> W;
  std::vector<double> mass_table;
  std::array<uint64_t, MAXD> mass_off{};
  void* dev_mass = nullptr;
  int dev_mass_id = -1;
  uint64_t count(int l) const {
    uint64_t n = 1;
    for (int s = 0; s < MAXD; ++s) n *= (uint64_t)sizes[l][s];
    return n;
  }
  ~Hierarchy();
};

// Builds (or returns a cached) hierarchy.  Throws Failure on bad arguments.
std::shared_ptr<Hierarchy> get_hierarchy(uint32_t ndim, const uint64_t* shape,
                                         const double* const* coords);
// Device copy of the constants in precision T (uploaded on first use).
const void* device_table(Hierarchy& h, bool f64, hipStream_t stream);
// Device copy (float64) of the finest grid's mass bands (uploaded on first use).
const double* device_mass_table(Hierarchy& h, hipStream_t stream);

// ----------------------------------------------------------------- workspace
// One growable device allocation per device, carved into aligned pieces.
class Workspace {
 public:
  void reserve(uint64_t bytes);
  void* base() const { return base_; }
  uint64_t size() const { return size_; }
  void release();

 private:
  void* base_ = nullptr;
  uint64_t size_ = 0;
};
Workspace& workspace();
// A second one, for staging that outlives calls which use the first (the
// lossless stage's input or output around compression and decompression).
Workspace& aux_workspace();
// Pinned host memory of at least `bytes` for the small synchronous copies of
// a call (headers, sizes, status words), per host thread, kept for the
// process's life; its contents do not survive the next call on the thread.
uint8_t* pinned_staging(size_t bytes);

struct Carver {
  char* p;
  uint64_t used = 0;
  explicit Carver(void* base) : p(static_cast<char*>(base)) {}
  template <typename X>
  X* take(uint64_t n) {
    uint64_t off = (used + 255) & ~uint64_t(255);
    used = off + n * sizeof(X);
    return reinterpret_cast<X*>(p + off);
  }
};
template <typename X>
inline uint64_t carve_size(uint64_t n) {
  return ((n * sizeof(X)) + 255) & ~uint64_t(255);
}

// --------------------------------------------------------- kernel launchers
// Geometry of one level as the kernels see it (slot layout, 4 slots).
template <typename T>
struct LevelGeom {
  int32_t nf[MAXD], nc[MAXD], act[MAXD];
  int32_t pad_slots;                 // MAXD - D
  const T* wl[MAXD];
  const T* wr[MAXD];
  uint64_t level_off;                // stream offset of this level
  const uint64_t* sub;               // device: sub-grid offsets [16] then strides [16][4] of this level
};

template <typename T>
struct DimConsts {
  const T *wl, *wr, *ma, *mb, *mc, *rl, *rr, *ta, *tr, *tcp;
};

template <typename T>
LevelGeom<T> level_geom(const Hierarchy& h, int l, const T* table);
template <typename T>
DimConsts<T> dim_consts(const Hierarchy& h, int l, int slot, const T* table);

// Decomposition / recomposition of a whole hierarchy (transform.hip).
// mode 0: float coefficient stream; mode 1: quantized symbols + qside.
struct QuantOut {
  uint16_t* sym = nullptr;
  int64_t* qside = nullptr;
  const double* bins = nullptr;  // device, L+1 entries
  int R = 0;
};
template <typename T>
uint64_t decompose_scratch_bytes(const Hierarchy& h);
// fine_written (nullable) is called once, on the host, right after the work
// that writes the finest level's part of the stream has been enqueued on st.
template <typename T>
void decompose(const Hierarchy& h, const T* table, const T* d_in, T* d_stream, const QuantOut* q,
               void* scratch, hipStream_t st, const std::function<void()>* fine_written = nullptr);
template <typename T>
uint64_t recompose_scratch_bytes(const Hierarchy& h);
template <typename T>
void recompose(const Hierarchy& h, const T* table, const T* d_stream, const QuantOut* q, T* d_out,
               void* scratch, hipStream_t st);

template <typename T>
void launch_thomas_strided(T* data, uint64_t outer, int n, uint64_t inner, DimConsts<T> w, hipStream_t st);

// A side stream per device (default priority, created on first use) with its
// fork and join events.  One host thread at a time enqueues work through a
// device's side stream: the lock is held from fork until the object goes away,
// after the join has been enqueued, so no call waits on another's events.
class SideStream {
 public:
  hipStream_t s = nullptr;
  void fork(hipStream_t st);   // s waits for the work enqueued on st so far
  void record_join();          // marks the end of the work enqueued on s
  void join(hipStream_t st);   // st waits for that work (no-op before a fork)

 private:
  hipEvent_t ef_ = nullptr, ej_ = nullptr;
  std::unique_lock<std::mutex> lk_;
};

// Fused 3D level kernels (transform3d.hip), used when all three sides are decomposed.
template <typename T>
bool fused3d_ok(const Hierarchy& h);
// coeff_written (nullable) is called right after the level's coefficient
// kernel has been enqueued.
template <typename T>
void fused3d_decompose_level(const Hierarchy& h, int l, const T* table, const T* u, T* ucoarse, T* g1, T* z,
                             const QuantOut* q, T* cstream, hipStream_t st,
                             const std::function<void()>* coeff_written = nullptr);
template <typename T>
void fused3d_recompose_level(const Hierarchy& h, int l, const T* table, const T* cur, T* out, T* g1, T* z,
                             const QuantOut* q, const T* cstream, hipStream_t st);
// The two halves of fused3d_recompose_level: the correction of level l (it
// reads only level l's coefficients) into z, using g1; then u_l from u_{l-1}
// (cur), z and the coefficients.
template <typename T>
void fused3d_recompose_correction(const Hierarchy& h, int l, const T* table, T* g1, T* z, const QuantOut* q,
                                  const T* cstream, hipStream_t st);
template <typename T>
void fused3d_recompose_finish(const Hierarchy& h, int l, const T* table, const T* cur, T* out, T* z,
                              const QuantOut* q, const T* cstream, hipStream_t st);
// The small levels (every side <= 17) and the coarsest grid in one workgroup:
// levels 1..lt, lt = fused3d_tail_levels (0: none).  Decomposition starts from
// u, the fine grid of level lt, and writes the stream of levels lt..0;
// recomposition reads levels 0..lt and writes the fine grid of level lt to out.
template <typename T>
int fused3d_tail_levels(const Hierarchy& h);
template <typename T>
void fused3d_tail_decompose(const Hierarchy& h, int lt, const T* table, const T* u, const QuantOut* q, T* cstream,
                            hipStream_t st);
template <typename T>
void fused3d_tail_recompose(const Hierarchy& h, int lt, const T* table, T* out, const QuantOut* q, const T* cstream,
                            hipStream_t st);

// Autotuned launch shapes (tune.hip): per knob, dtype and fine level shape.
constexpr int TUNE_COEFF_SEG = 0;       // coarse intervals of dim 0 per block, plane-marching decomposition
constexpr int TUNE_SCATTER_PLANES = 1;  // fine planes per block, recomposition scatter
constexpr int TUNE_KNOBS = 2;
int tune_get(int knob, bool f64, int n0, int n1, int n2, int fallback);
bool tune_known(int knob, bool f64, int n0, int n1, int n2);
void tune_set(int knob, bool f64, int n0, int n1, int n2, int value);
void tune_force(int knob, int value);  // this thread only; 0 clears
void tune_save();
// Times the candidates of every level of the fused 3D path on d_in (which
// also serves as each coarser level's input) and records the fastest; q
// holds the quantization buffers and bins (transform.hip).
template <typename T>
void fused3d_tune(const Hierarchy& h, const T* table, const T* d_in, const QuantOut* q, void* scratch,
                  hipStream_t st);

// Quantization helpers (quant.hip).
void launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t st);
template <typename T>
void launch_maxabs(const T* d, uint64_t n, uint64_t* d_bits, hipStream_t st);
struct BinArgs {
  double K[MAXL + 1];
  double counts[MAXL + 1];
};
void launch_bins(int f64, const uint64_t* d_maxbits, double tol, int rel, double S, int L,
                 int alloc, const BinArgs& a, double* d_bins, double* d_scalars, hipStream_t st);
template <typename T>
void launch_quantize(const T* c, uint64_t n, const uint64_t* d_level_off, int nlev,
                     const double* d_bins, int R, uint16_t* sym, int64_t* qside, hipStream_t st);
template <typename T>
void launch_dequantize(const uint16_t* sym, const int64_t* qside, uint64_t n,
                       const uint64_t* d_level_off, int nlev, const double* d_bins, int R, T* c,
                       hipStream_t st);

// The s-norm bound (norms.hip): per-level width factors g_l and the rounding
// reserve factor, computed on the host in float64.
struct SnormArgs {
  double g[MAXL + 1];
  double reserve;
};
SnormArgs snorm_args(const Hierarchy& h, double s);
uint64_t mass_norm_scratch_bytes();
// *d_out = u^T M u (float64) of the input grid; d_bands from device_mass_table.
template <typename T>
void launch_mass_norm(const Hierarchy& h, const double* d_bands, const T* u, void* scratch, double* d_out,
                      hipStream_t st);
// Widths b_l = 2 tau_eff g_l; tau = tol sqrt(*d_nrm2) (rel) or tol; scalars as launch_bins.
void launch_bins_snorm(int f64, const uint64_t* d_maxbits, const double* d_nrm2, double tol, int rel, int L,
                       const SnormArgs& a, double* d_bins, double* d_scalars, hipStream_t st);

// Refactoring into bitplane precision segments (refactor.hip).  Per level:
// stream offset and count, words per plane, the level's first word in the
// segment area (sign plane, then B planes), its first wavefront (2048
// coefficients each); for reconstruction also the exponent and planes used.
struct RfLevels {
  int nlev;
  uint64_t off[MAXL + 2], n[MAXL + 2], words[MAXL + 2], word_off[MAXL + 2], wave0[MAXL + 2];
  int exp[MAXL + 2], planes[MAXL + 2];
};
RfLevels rf_levels(const Hierarchy& h, uint32_t B);
struct RfMetaLayout {
  uint64_t exp_off, R_off, loff_off, meta_bytes, total;
};
RfMetaLayout rf_meta_layout(const Hierarchy& h, const bool* has_coords, uint32_t B, const RfLevels& lv);
std::vector<uint8_t> rf_header(const Hierarchy& h, const double* const* coords, int dtype, uint32_t B,
                               const RfLevels& lv, const RfMetaLayout& m);
struct RfParsed {
  int dtype = 0, ndim = 0, B = 0, L = 0;
  double maxabs = 0.0, l2norm = 0.0;
  uint64_t shape[MAXD] = {0, 0, 0, 0};
  bool has_coords[MAXD] = {false, false, false, false};
  std::vector<std::vector<double>> coords;
  std::vector<int> exps;
  std::vector<uint32_t> R;
  std::vector<uint64_t> loff;
  uint64_t meta_bytes = 0, need = 0;
  // coordinate pointers for get_hierarchy (NULL when every dimension is uniform)
  const double* const* coord_ptrs(const double** buf) const;
};
// false (and P.need set) when more bytes are needed; throws on malformed input
bool rf_parse(const uint8_t* b, uint64_t bytes, RfParsed& P);
void rf_check_layout(const RfParsed& P, const Hierarchy& h, RfLevels* lv);
std::vector<uint32_t> rf_request(const RfParsed& P, const Hierarchy& h, double tol, int eb, int norm, double s,
                                 const uint32_t* have, double* estimate);
template <typename T>
void launch_rf_planes(const T* cs, const RfLevels& lv, int B, const int* exps, uint32_t* seg, uint32_t* R,
                      hipStream_t st);
void launch_rf_meta(const uint64_t* lbits, const uint64_t* ubits, const double* nrm2, int f64, int nlev, int* exps,
                    void* hdr, uint64_t hdr_exp, hipStream_t st);
template <typename T>
void launch_rf_decode(const uint32_t* seg, const RfLevels& lv, int B, T* cs, hipStream_t st);

// Second-stage lossless coder (lossless.hip).
uint64_t zs_bound(uint64_t raw_bytes);
// Encodes raw_bytes of d_in (4-byte aligned) into the container at d_out and
// returns its size; d_sizes: scratch of ceil(raw_bytes / 16384) + 1 words.
// Synchronises st.
uint64_t zs_encode(const void* d_in, uint64_t raw_bytes, void* d_out, uint64_t capacity, uint32_t* d_sizes,
                   hipStream_t st);
// Fixed part of a container held on the host; false when it is not one.
bool zs_parse(const uint8_t* h, uint64_t bytes, uint64_t* raw_bytes, uint64_t* nch);
// Decodes into d_out (4 ceil(raw_bytes / 4) bytes); throws MGARD_ERR_FORMAT
// for malformed input; status: one device word of scratch.  Synchronises st.
void zs_decode(const void* d_in, uint64_t in_bytes, uint64_t raw_bytes, uint64_t nch, void* d_out, uint32_t* status,
               hipStream_t st);

// Huffman (huffman.hip).
void launch_histogram(const uint16_t* sym, uint64_t n, int dict, int chunk, uint64_t* hist,
                      uint32_t* chunk_esc, uint32_t* status, hipStream_t st);
// Chunks [k0, k1) only, adding into hist (which the caller has cleared).
void launch_histogram_chunks(const uint16_t* sym, uint64_t n, int dict, int chunk, uint64_t k0, uint64_t k1,
                             uint64_t* hist, uint32_t* chunk_esc, uint32_t* status, hipStream_t st);
// enc_scratch (nullable): the encoder's scratch, whose packed code table and
// longest length the codebook kernel then fills (see launch_encode's packed).
void launch_codebook(const uint64_t* hist, int dict, uint8_t* len, uint64_t* codes, void* enc_scratch,
                     hipStream_t st);
// The packed code table and longest-length slot inside an encoder scratch.
void encode_tables(void* enc_scratch, int dict, uint32_t** enc, uint32_t** maxlen);
void launch_chunk_bits(const uint16_t* sym, uint64_t n, int dict, int chunk, const uint8_t* len,
                       uint32_t* chunk_bits, hipStream_t st);
// exclusive scan of per-chunk words (ceil(bits/32)) -> offsets (n+1 entries, last = total)
void launch_scan_words(const uint32_t* chunk_bits, uint64_t nch, uint64_t* word_off,
                       hipStream_t st);
void launch_scan_u32(const uint32_t* v, uint64_t n, uint64_t* off, hipStream_t st);
// both at once: word offsets of the chunk bit counts and offsets of the escape counts
void launch_scan_pair(const uint32_t* chunk_bits, const uint32_t* esc, uint64_t nch, uint64_t* word_off,
                      uint64_t* esc_off, hipStream_t st);
uint64_t encode_scratch_bytes(int dict);
// With esc_off, qside and ecodes given, the code of the j-th escaped value
// (2 (|q| - R) + [q < 0], R = dict / 2) goes to ecodes[j].
void launch_encode(const uint16_t* sym, uint64_t n, int dict, int chunk, const uint8_t* len,
                   const uint64_t* codes, const uint64_t* word_off, uint32_t* payload,
                   const uint64_t* esc_off, const int64_t* qside, uint64_t* ecodes, void* scratch,
                   bool packed, hipStream_t st);
// Escaped values, packed per level (escapes.hip).  Level offsets of a stream
// by value (so that no host copy is needed inside a captured graph).
struct LevelTable {
  uint64_t off[MAXL + 2];
};
// After the encoder has written the escape codes (ecodes): per level the first
// escape index (ostart, nlev + 1), the largest code (wmax, nlev), the counts
// and widths (hdr_counts, hdr_bits: the header's arrays) and the word offsets
// (woff, nlev + 1; woff[nlev] = total words), and the packed words after the
// payload at d_out + payload_off + 4 word_off[nch].
void launch_escape_pack(const uint16_t* sym, uint64_t n, int chunk, const uint64_t* esc_off, const uint64_t* word_off,
                        uint64_t nch, const uint64_t* ecodes, int nlev, const LevelTable& lt, char* d_out,
                        uint64_t payload_off, uint64_t* hdr_counts, uint32_t* hdr_bits, uint64_t* ostart,
                        unsigned long long* wmax, uint64_t* woff, hipStream_t st);
// The per-level layout of a stored stream's escapes, from its header.
struct EscLevels {
  uint64_t ostart[MAXL + 2];  // first escape index of each level; the total last
  uint64_t woff[MAXL + 2];    // first word of each level; all words last
  uint64_t loff[MAXL + 2];    // stream offsets of the levels; n last
  uint32_t bits[MAXL + 1];
  int nlev;
};
// qside[epos[j]] = q of escape j (skipped when *status is set; sets it for an
// escape recorded outside its level).  words: the nw packed words.
void launch_escape_scatter(const uint64_t* epos, const uint32_t* words, uint64_t nw, const EscLevels& t, int R,
                           uint64_t n, int64_t* qside, uint32_t* status, hipStream_t st);

uint64_t decode_table_bytes(int dict);
// Decoding tables and the decode itself; with esc_off and epos given, the
// stream positions of the n_out escapes go to epos.
void launch_decode_full(const uint32_t* payload, uint64_t payload_words, const uint64_t* word_off,
                        const uint32_t* chunk_bits, uint64_t n, int dict, int chunk,
                        const uint8_t* len, uint16_t* sym, const uint64_t* esc_off, uint64_t n_out,
                        uint64_t* epos, void* table_scratch, uint32_t* d_status, hipStream_t st);

// Learned allocation (mlp.hip).  Parameter layout (float32): mean[4], std[4],
// W1[64][4], b1[64], W2[64][64], b2[64], W3[64], b3[1].
constexpr int MLP_IN = 4, MLP_HID = 64;
constexpr int MLP_W1 = 2 * MLP_IN;
constexpr int MLP_B1 = MLP_W1 + MLP_HID * MLP_IN;
constexpr int MLP_W2 = MLP_B1 + MLP_HID;
constexpr int MLP_B2 = MLP_W2 + MLP_HID * MLP_HID;
constexpr int MLP_W3 = MLP_B2 + MLP_HID;
constexpr int MLP_B3 = MLP_W3 + MLP_HID;
constexpr int MLP_NPARAM = MLP_B3 + 1;
constexpr int STATS_BLOCKS = 256;  // partial-sum blocks per level
template <typename T>
void launch_level_stats(const T* c, const uint64_t* d_off, int nlev, double* d_part, double* d_stats,
                        hipStream_t st);
void launch_features(const double* d_stats, const double* d_scalars, int nlev, const float* d_params,
                     float* d_x, hipStream_t st);
void launch_apply_theta(const double* d_bins, const float* d_theta, int nlev, double scale, double* d_learned,
                        hipStream_t st);
template <typename T>
void launch_linf(const T* a, const T* b, uint64_t n, unsigned long long* d_err, hipStream_t st);
void launch_select_bins(const unsigned long long* d_err, double* d_scalars, double* d_bins,
                        const double* d_learned, int nlev, hipStream_t st);
void mlp_forward(const float* params, const float* x, int B, float* out, float* cache, float* tmp,
                 hipStream_t st);
void mlp_backward(const float* params, const float* x, const float* cache, const float* dout, int B,
                  float* grads, float* tmp, hipStream_t st);
void mlp_normalize(const float* x, const float* params, int B, float* xn, hipStream_t st);
void mlp_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2,
              float eps, int step, hipStream_t st);
void mlp_mse(const float* pred, const float* target, int B, float* dout, double* loss,
             hipStream_t st);

}  // namespace mg
