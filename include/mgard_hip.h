/*
 * mgard_hip.h -- C interface of the MI355X (gfx950) multilevel lossy compressor.
 *
 * The operations follow the compression module of the paper
 * "MGARD: A multigrid framework for high-performance, error-controlled data
 * compression and refactoring":
 *   - recursive multilevel decomposition of the input into multilevel
 *     coefficients (Sec. 2, software design),
 *   - level-wise linear quantization of the coefficients by a bin width, with
 *     an error guarantee in the L-infinity norm (Sec. 2; Sec. 2.3),
 *   - lossless encoding into a self-describing buffer (Sec. 2; Sec. 2.1),
 *   - the high-level compress / decompress calls (Sec. 3, first listing) and
 *     individual stage calls in the spirit of the low-level API (Sec. 2.1).
 *
 * Conventions for every call:
 *   - Arrays are C-ordered (last dimension contiguous), 1 to 4 dimensions.
 *   - Pointers named d_* are device (HBM) pointers on the current HIP device;
 *     pointers named h_* are host pointers.  The caller owns every buffer; the
 *     library never frees caller memory.  Scratch memory is allocated by the
 *     library on first use, cached per device, and reused by later calls
 *     (mgard_release_workspace frees it).  Calls that share a device must not
 *     run concurrently: they share that scratch memory.
 *   - Work is enqueued on opts->stream (a hipStream_t, NULL = default stream).
 *     Calls that return sizes to the host synchronise that stream once.
 *   - Errors are returned as mgard_status codes; no C++ exception crosses this
 *     interface.  mgard_last_error() gives a message for the last failure on
 *     the calling thread.  On error the contents of output buffers are
 *     unspecified.
 *   - Coordinates: coords may be NULL (all dimensions uniform) or an array of
 *     ndim host pointers, each NULL (uniform) or pointing to shape[d]
 *     strictly increasing float64 values.
 */
#ifndef MGARD_HIP_H
#define MGARD_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MGARD_OK = 0,
  MGARD_ERR_ARG = -1,       /* null pointer, bad option value, bad coordinates */
  MGARD_ERR_SHAPE = -2,     /* ndim outside 1..4, a zero side, too many elements */
  MGARD_ERR_DTYPE = -3,     /* dtype is not MGARD_F32 / MGARD_F64 */
  MGARD_ERR_TOL = -4,       /* tolerance not positive / not finite, or outside the
                               supported range: the rounding reserve
                               4 (L+1) eps max|u| exceeds tau / 2, or max|u| / b_l
                               reaches 2^49 for some level */
  MGARD_ERR_NONFINITE = -5, /* the input holds a NaN or an infinity */
  MGARD_ERR_CAPACITY = -6,  /* an output buffer is smaller than required */
  MGARD_ERR_FORMAT = -7,    /* compressed buffer is malformed or truncated */
  MGARD_ERR_DEVICE = -8,    /* a HIP runtime call failed */
  MGARD_ERR_OOM = -9        /* scratch allocation failed */
} mgard_status;

typedef enum { MGARD_F32 = 0, MGARD_F64 = 1 } mgard_dtype;
/* Error bound type (Sec. 3, first listing: absolute or relative bound).
 * MGARD_REL: the bound is tol * max|u| (L-infinity) or tol * ||u|| (L2). */
typedef enum { MGARD_ABS = 0, MGARD_REL = 1 } mgard_eb;
/* Norm of the bound (Sec. 2: error estimators in several norms, chosen by the
 * smoothness parameter s).
 *   LINF  max |u - u~| <= tau (the default).
 *   S     ||u - u~||_s <= tau, where ||v||^2 = v^T M v is the L2 norm of the
 *         multilinear interpolant (M = kron of the consistent P1 mass matrices
 *         on the coordinates; sides of 1 or 2 nodes are summed over) and
 *         ||v||_s^2 = sum_l 4^(s l) ||(Q_l - Q_{l-1}) v||^2 over the levels,
 *         coarsest l = 0, Q_l the L2 projection onto level l; s = 0 is the L2
 *         norm.  Widths b_l = 2 tau_eff sqrt(N_l / (N 4^(s l) W_l)), W_l the
 *         hat-function integrals of level l's new nodes; tau_eff leaves
 *         max(1, 2^(s L)) sqrt(W_0) 4 (L+1) eps max|u| for rounding.  Plain
 *         allocation only; MGARD_REL needs s = 0; not offered by batches or
 *         the out-of-core calls (MGARD_ERR_ARG). */
typedef enum { MGARD_NORM_LINF = 0, MGARD_NORM_S = 1 } mgard_norm;
/* Bin-width allocation across levels.
 *   PLAIN   one bin width b = 2 tau_eff / S for all levels, with
 *           S = 1 + sum_l (1 + K_l) and K_l the product over dimensions of the
 *           infinity norms of the level's correction operators; this meets
 *           the L-infinity bound a priori.
 *   LEARNED per-level widths b_l = b * exp(theta_l) from a small network over
 *           per-level coefficient statistics (a project addition, not in the
 *           paper); the result is recomposed on the device and checked, and
 *           the plain widths are used instead whenever the L-infinity error
 *           exceeds the bound.
 *   COUNT   count-weighted widths b_l = 2 tau_eff N_l / ((1 + K_l) sum N)
 *           (ablation; also meets the bound a priori). */
typedef enum { MGARD_ALLOC_PLAIN = 0, MGARD_ALLOC_LEARNED = 1, MGARD_ALLOC_COUNT = 2 } mgard_alloc;

/* Second lossless stage after the entropy coder (Sec. 2: the final lossless
 * encoding).  ZS: zero suppression, see mgard_lossless_encode; mgard_compress
 * then writes the 'MGZS' container of its stream when that is smaller. */
typedef enum { MGARD_LOSSLESS_NONE = 0, MGARD_LOSSLESS_ZS = 1 } mgard_lossless;

typedef struct mgard_model mgard_model; /* device-resident network weights */

typedef struct {
  uint32_t struct_size;   /* sizeof(mgard_opts) */
  uint32_t eb;            /* mgard_eb, default MGARD_REL */
  uint32_t alloc;         /* mgard_alloc, default MGARD_ALLOC_PLAIN */
  uint32_t dict_size;     /* Huffman dictionary: power of two in [256, 8192]; 0 = 8192 */
  uint32_t chunk_symbols; /* symbols per independently decodable chunk, multiple of 256
                             in [256, 8192]; 0 = 1024 */
  uint32_t lossless;      /* mgard_lossless: second lossless stage of mgard_compress,
                             default MGARD_LOSSLESS_NONE */
  void* stream;              /* hipStream_t */
  const mgard_model* model;  /* required for MGARD_ALLOC_LEARNED */
  uint32_t norm;             /* mgard_norm, default MGARD_NORM_LINF */
  uint32_t reserved2;
  double s;                  /* smoothness of MGARD_NORM_S (finite), default 0 */
} mgard_opts;

/* Fills *opts with the defaults (REL, PLAIN, 8192, 1024, default stream, L-infinity). */
void mgard_default_opts(mgard_opts* opts);

typedef struct {
  double tol, tau_abs, maxabs;
  double bin_width[40];   /* per level, coarsest grid first; levels+1 entries used */
  double linf_err;        /* measured by the learned-allocation check, else -1 */
  uint64_t n_symbols, n_outliers, payload_words, out_bytes;
  uint32_t levels, fallback_used;
} mgard_info;

typedef struct {
  uint32_t version, dtype, ndim, eb, alloc, fallback, coord_flags, levels;
  uint32_t dict_size, chunk_symbols;
  uint64_t shape[4];
  double tol, tau_abs, maxabs;
  uint64_t n_symbols, n_chunks, n_outliers, payload_words, total_bytes;
  uint32_t norm, reserved;  /* mgard_norm */
  double s;
} mgard_header;

/* ---------------------------------------------------------------- high level */

/* Upper bound on the compressed size in bytes (header, code lengths, chunk
 * tables, worst-case payload and outliers).  Returns 0 for invalid arguments. */
uint64_t mgard_compress_bound(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                              mgard_dtype dtype, const mgard_opts* opts);

/* Compresses d_in (device, dtype, shape) under tol (Sec. 3, first listing).
 * d_out: device buffer of out_capacity bytes, at least mgard_compress_bound().
 * *out_bytes (host) receives the compressed size; info (nullable) receives
 * the bound, bin widths and counts.  Synchronises opts->stream once. */
mgard_status mgard_compress(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                            mgard_dtype dtype, double tol, const void* d_in, void* d_out,
                            uint64_t out_capacity, uint64_t* out_bytes, const mgard_opts* opts,
                            mgard_info* info);

/* Decompresses in_bytes of d_in (device) into d_out (device, out_capacity
 * bytes, at least prod(shape)*sizeof(dtype) as stored in the header).  The
 * header is read back to the host first and validated before any decoding.
 * A buffer in the 'MGZS' container of the lossless stage is decoded first.
 * hdr (nullable) receives the parsed header. */
mgard_status mgard_decompress(const void* d_in, uint64_t in_bytes, void* d_out,
                              uint64_t out_capacity, const mgard_opts* opts, mgard_header* hdr);

/* ------------------------------------------------------------- batches
 * A project addition (the paper compresses one variable per call, Sec. 3):
 * many fields of different shapes compressed by one graph launch.
 *
 * mgard_batch_create plans the compression of `nfields` fields (each with its
 * own shape, coordinates, dtype and device input; opts->alloc must be PLAIN or
 * COUNT) under one tolerance into d_out: field i is written at byte offset
 * h_offsets[i] (host array of nfields, filled by the call; slots are
 * mgard_compress_bound bytes, 256-byte aligned, in field order) and its
 * compressed size goes to d_sizes[i] (device, uint64) at each launch, or 0
 * when field i cannot be compressed (its input holds a NaN or an infinity,
 * or the tolerance is outside the supported range, see MGARD_ERR_TOL).  The
 * call allocates the plan's scratch (one device allocation, owned by the
 * plan), uploads the headers and constant tables, runs the autotuner for the
 * fields' level shapes (mgard_autotune), then captures every field's
 * compression into one HIP graph of grouped launches: every field's kernel
 * launches are recorded in order, and launches of the same kernel by many
 * fields run as one launch whose blocks find their field's arguments, grid
 * and block index in a device table (the auto-tuning and adaptive
 * scheduling layer of Sec. 2.2).  Fields whose decompositions take different
 * kernels (3D fused, generic, one-block small levels; per precision) form
 * separate chains on parallel branches of the graph.  Nothing in the graph allocates, copies
 * from host memory, sets memory or synchronises with the host.  Inputs and output are bound at creation: each launch compresses
 * the current contents of the same input buffers.  MGARD_ERR_CAPACITY when
 * out_capacity < mgard_batch_bound().
 *
 * mgard_batch_launch replays the graph on `stream` (a hipStream_t, NULL for
 * the default stream) with one hipGraphLaunch and returns without waiting.
 * Launches of one plan must not overlap; distinct plans are independent. */
typedef struct {
  uint32_t ndim;
  uint32_t dtype;             /* mgard_dtype */
  uint64_t shape[4];
  const double* coords[4];    /* host; NULL entries: uniform 0..n-1 */
  const void* d_in;           /* device, C order */
} mgard_field;

typedef struct mgard_batch mgard_batch;

uint64_t mgard_batch_bound(uint32_t nfields, const mgard_field* fields, const mgard_opts* opts);
mgard_status mgard_batch_create(uint32_t nfields, const mgard_field* fields, double tol, void* d_out,
                                uint64_t out_capacity, uint64_t* h_offsets, uint64_t* d_sizes,
                                const mgard_opts* opts, mgard_batch** plan);
mgard_status mgard_batch_launch(mgard_batch* plan, void* stream);
void mgard_batch_free(mgard_batch* plan);
/* Kernel launches in one graph launch of the plan (0 for NULL). */
uint32_t mgard_batch_launches(const mgard_batch* plan);

/* Autotuner: the auto-tuning part of the library's adaptive scheduling layer
 * (Sec. 2.2, software architecture).  For each level of the fused 3D path of this
 * shape and dtype, times the candidate launch shapes of the decomposition's
 * plane-marching kernel (coarse intervals per block) and of the
 * recomposition's scatter kernel (fine planes per block) on d_in and keeps
 * the fastest; later compressions and decompressions of that level shape use
 * them.  The choices persist in the JSON file named by the environment
 * variable MGARD_TUNE_FILE when it is set (read at the first call, rewritten
 * after each tuning).  Shapes without a fused 3D path have nothing to tune
 * (MGARD_OK).  Tuning runs kernels on opts->stream and synchronises it. */
mgard_status mgard_autotune(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                            mgard_dtype dtype, const void* d_in, const mgard_opts* opts);

/* Host-only header parser: h_buf holds at least the first `bytes` bytes of a
 * compressed buffer.  Returns MGARD_ERR_FORMAT when they do not form a valid
 * header (MGARD_ERR_CAPACITY when more bytes are needed for the full header;
 * hdr->total_bytes then holds nothing useful). */
mgard_status mgard_inspect(const void* h_buf, uint64_t bytes, mgard_header* hdr);

/* ------------------------------------------------------------ stage calls
 * The stage calls run single steps of the pipeline on caller buffers
 * (Sec. 2.1, low-level API).  The coefficient stream holds, in order, the
 * coarsest grid (C order), then levels 1..L; inside a level the sub-grids by
 * odd-dimension mask m = 1..2^D-1 ascending (bit d set: dimension d indexes
 * the new nodes of that level), each dense and C ordered. */

/* Levels and stream layout: *levels = L; level_offsets (nullable, L+2
 * entries) receives the start of each level in the stream and the total. */
mgard_status mgard_stream_layout(uint32_t ndim, const uint64_t* shape, uint32_t* levels,
                                 uint64_t* level_offsets, uint32_t max_offsets);

/* Multilevel decomposition (Sec. 2): d_in (dtype, shape) -> d_coeff (dtype,
 * prod(shape) values in stream order).  Arithmetic in dtype. */
mgard_status mgard_decompose(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                             mgard_dtype dtype, const void* d_in, void* d_coeff,
                             const mgard_opts* opts);

/* Inverse of mgard_decompose (the paper's inverse procedure). */
mgard_status mgard_recompose(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                             mgard_dtype dtype, const void* d_coeff, void* d_out,
                             const mgard_opts* opts);

/* Level-wise quantization (Sec. 2): for level l with host bin width
 * h_bins[l], q = round-half-away(float64(c) * (1/b_l)); symbol = q + dict/2
 * when |q| < dict/2, else 0 with q stored at the same index of d_qside
 * (int64, n values; only escape positions are written).  d_symbols: uint16. */
mgard_status mgard_quantize(uint32_t ndim, const uint64_t* shape, mgard_dtype dtype,
                            const void* d_coeff, const double* h_bins, uint32_t dict_size,
                            uint16_t* d_symbols, int64_t* d_qside, const mgard_opts* opts);

/* Dequantization: c = dtype(float64(q) * b_l) with q from symbols / qside. */
mgard_status mgard_dequantize(uint32_t ndim, const uint64_t* shape, mgard_dtype dtype,
                              const uint16_t* d_symbols, const int64_t* d_qside,
                              const double* h_bins, uint32_t dict_size, void* d_coeff,
                              const mgard_opts* opts);

/* Histogram of n uint16 symbols into d_hist (uint64, dict_size entries) and
 * the number of escape symbols (0) in each chunk into d_chunk_esc (uint32,
 * ceil(n/chunk) entries).  d_symbols must be 16-byte aligned; MGARD_ERR_ARG
 * for a symbol outside the dictionary. */
mgard_status mgard_histogram(const uint16_t* d_symbols, uint64_t n, uint32_t dict_size,
                             uint32_t chunk, uint64_t* d_hist, uint32_t* d_chunk_esc,
                             const mgard_opts* opts);

/* Huffman code lengths (uint8) and canonical codes (uint64, right-aligned)
 * from a device histogram: leaves sorted by (count, symbol), two-queue merge
 * with ties to the leaf, canonical order (length, symbol). */
mgard_status mgard_huffman_codebook(const uint64_t* d_hist, uint32_t dict_size,
                                    uint8_t* d_code_len, uint64_t* d_codes,
                                    const mgard_opts* opts);

/* Chunked encoding: each chunk of `chunk` symbols is packed MSB-first into
 * 32-bit words starting word-aligned; d_chunk_bits (uint32) receives its bit
 * count, d_payload the concatenated chunks.  *payload_words (host) receives
 * the payload length; payload_capacity is in words.  d_symbols must be
 * 16-byte aligned. */
mgard_status mgard_huffman_encode(const uint16_t* d_symbols, uint64_t n, uint32_t dict_size,
                                  uint32_t chunk, const uint8_t* d_code_len,
                                  const uint64_t* d_codes, uint32_t* d_chunk_bits,
                                  uint32_t* d_payload, uint64_t payload_capacity,
                                  uint64_t* payload_words, const mgard_opts* opts);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments, results and errors as mgard_huffman_encode, but its
 * scratch (chunk word offsets and the packed code table) lives in a fixed
 * array of the library that every device holds until the process ends
 * (about 16 MiB), and the call allocates nothing.  n may need at most
 * MGARD_NOALLOC_MAX_CHUNKS chunks of `chunk` symbols (MGARD_ERR_CAPACITY
 * otherwise).  All calls on one device share that array and every call
 * rewrites the part it reads before reading it, so consecutive calls are
 * independent; calls that overlap on one device (other host threads, other
 * streams) race and must not be made. */
#define MGARD_NOALLOC_MAX_CHUNKS 2097152
mgard_status mgard_huffman_encode_noalloc(const uint16_t* d_symbols, uint64_t n, uint32_t dict_size,
                                          uint32_t chunk, const uint8_t* d_code_len,
                                          const uint64_t* d_codes, uint32_t* d_chunk_bits,
                                          uint32_t* d_payload, uint64_t payload_capacity,
                                          uint64_t* payload_words, const mgard_opts* opts);

/* Inverse of mgard_huffman_encode.  d_symbols must be 16-byte aligned
 * (MGARD_ERR_ARG otherwise); MGARD_ERR_FORMAT when the payload does not
 * decode to exactly n symbols with the given bit counts. */
mgard_status mgard_huffman_decode(const uint32_t* d_payload, uint64_t payload_words,
                                  const uint32_t* d_chunk_bits, uint64_t n, uint32_t dict_size,
                                  uint32_t chunk, const uint8_t* d_code_len, uint16_t* d_symbols,
                                  const mgard_opts* opts);

/* max |u| over n values of dtype into *h_maxabs; MGARD_ERR_NONFINITE when a
 * NaN or infinity is present. */
mgard_status mgard_maxabs(mgard_dtype dtype, const void* d_in, uint64_t n, double* h_maxabs,
                          const mgard_opts* opts);

/* ||u|| = sqrt(u^T M u), the L2 norm of the multilinear interpolant of d_in
 * (dtype, shape, coordinates) as MGARD_NORM_S defines it, summed in float64
 * on the device in a fixed order, into *h_norm. */
mgard_status mgard_l2_norm(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                           mgard_dtype dtype, const void* d_in, double* h_norm,
                           const mgard_opts* opts);

/* Plain bin width and the a-priori constant S for a shape (host only). */
mgard_status mgard_plain_constant(uint32_t ndim, const uint64_t* shape,
                                  const double* const* coords, double* h_S, double* h_K,
                                  uint32_t max_levels);

/* ----------------------------------------------------- learned allocation
 * A project addition (the paper defines no learned component; it motivates
 * higher-ratio compression for AI workloads, Sec. 1).  A small network maps
 * four features of a level's coefficients -- log(rms/tau), log(max|c|/tau),
 * log(count / stream length), l/L, normalised by a stored mean and standard deviation -- to
 * theta_l; the level's bin width is b_plain * exp(s * clamp(theta_l, -3, 5)).
 * With opts->alloc = MGARD_ALLOC_LEARNED and opts->model set, mgard_compress
 * decomposes, evaluates the network, quantizes, recomposes on the device and
 * measures max|u - u~| (the bound check), first with s = 1 and, if that exceeds
 * tau, again with s = 1/2; when both exceed tau the plain widths are used
 * (mgard_info.fallback_used = 1, header fallback byte set).  The check's
 * result is read back once between the two attempts.
 *
 * Parameters: MGARD_MLP_NPARAM float32 values, layout mean[4], std[4],
 * W1[64][4], b1[64], W2[64][64], b2[64], W3[64], b3[1] (y = x W^T + b,
 * Linear(4,64)-ReLU-Linear(64,64)-ReLU-Linear(64,1)). */
#define MGARD_MLP_NPARAM 4553
#define MGARD_MLP_IN 4
#define MGARD_MLP_HID 64
#define MGARD_MLP_CACHE_PER_ROW 260 /* floats of d_cache per batch row */

/* Copies h_params (n_params == MGARD_MLP_NPARAM) to the current device.
 * MGARD_ERR_ARG for non-finite values or non-positive feature scales. */
mgard_status mgard_model_create(const float* h_params, uint64_t n_params, mgard_model** out);
void mgard_model_free(mgard_model* model);

/* Per level of a coefficient stream (stream order as above): h_stats[3l] =
 * count, h_stats[3l+1] = sum of squares (float64), h_stats[3l+2] = max |c|. */
mgard_status mgard_level_stats(uint32_t ndim, const uint64_t* shape, mgard_dtype dtype,
                               const void* d_coeff, double* h_stats, const mgard_opts* opts);

/* The network's raw input rows for a coefficient stream (stream order as
 * above): h_x[4l .. 4l+3] = log(rms_l/tau_abs), log(max_l |c|/tau_abs),
 * log(count_l / stream length), l/L, computed on the device by the same
 * kernels as the learned compression (before the stored normalisation).
 * max_rows: capacity of h_x in rows (MGARD_ERR_CAPACITY below levels + 1). */
mgard_status mgard_level_features(uint32_t ndim, const uint64_t* shape, mgard_dtype dtype,
                                  const void* d_coeff, double tau_abs, float* h_x,
                                  uint32_t max_rows, const mgard_opts* opts);

/* The a-priori bin widths (opts->alloc PLAIN or COUNT, opts->eb) of d_in under
 * tol, computed on the device by the kernels of mgard_compress: max|u|, then
 * tau, the rounding reserve and the widths (Sec. 2: bin widths from an error
 * estimator).  h_bins receives levels + 1 widths, coarsest grid first
 * (max_bins: its capacity); *h_tau_abs (nullable) the absolute bound.  Fails
 * as mgard_compress does for non-finite input or an unsupported tolerance. */
mgard_status mgard_bin_widths(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                              mgard_dtype dtype, double tol, const void* d_in, double* h_bins,
                              uint32_t max_bins, double* h_tau_abs, const mgard_opts* opts);

/* max |a_i - b_i| over n values of dtype, evaluated in float64, into *h_err. */
mgard_status mgard_linf_error(mgard_dtype dtype, const void* d_a, const void* d_b, uint64_t n,
                              double* h_err, const mgard_opts* opts);

/* Network forward over `batch` rows of raw features d_x (batch x 4, float32)
 * into d_out (batch).  d_cache (nullable, batch x MGARD_MLP_CACHE_PER_ROW)
 * keeps the normalised input and the activations for mgard_mlp_backward.
 * Sums run in a fixed order; the results are reproducible. */
mgard_status mgard_mlp_forward(const float* d_params, const float* d_x, uint32_t batch,
                               float* d_out, float* d_cache, const mgard_opts* opts);

/* Gradients of the loss with respect to the weights (same layout as the
 * parameters; the mean/std entries are set to 0) from d_dout = dLoss/dout. */
mgard_status mgard_mlp_backward(const float* d_params, const float* d_cache, const float* d_dout,
                                uint32_t batch, float* d_grads, const mgard_opts* opts);

/* Mean squared error 1/B sum (pred - target)^2 into *h_loss and its gradient
 * 2/B (pred - target) into d_dout. */
mgard_status mgard_mlp_mse(const float* d_pred, const float* d_target, uint32_t batch,
                           float* d_dout, double* h_loss, const mgard_opts* opts);

/* One Adam step (bias-corrected, step counts from 1) on the weights; the
 * feature normalisation entries are left unchanged.  d_m, d_v: moment
 * buffers of MGARD_MLP_NPARAM floats, zero before the first step. */
mgard_status mgard_mlp_adam(float* d_params, const float* d_grads, float* d_m, float* d_v,
                            uint32_t step, float lr, float beta1, float beta2, float eps,
                            const mgard_opts* opts);

/* ----------------------------------------------------------- out-of-core
 * Compression of a host-resident array larger than device memory (Sec. 2.1,
 * high-level APIs: out-of-core processing; Sec. 2.2, software architecture:
 * the array is partitioned into chunks that fit on the device).
 *
 * Chunks are slabs of slab_planes planes (>= 3) along dimension 0; a last
 * slab of fewer than 3 planes joins the one before it.  Every slab is
 * compressed as a field of its own, in the format of mgard_compress, at the
 * absolute tolerance of the whole array (MGARD_REL: tol * max |u| over the
 * array, found in a first streaming pass), so the L-infinity bound holds on
 * every slab and on the array.  A nonuniform dimension 0 gives each slab its
 * own coordinates.  Slab k + 1 is copied to the device while slab k is
 * compressed and slab k - 1 is copied back; h_in and h_out should be pinned
 * host memory (hipHostMalloc) for the copies to overlap (pageable memory
 * works, with copies that wait).  Device memory: two slabs, two slab bounds,
 * and the scratch of one slab, allocated and freed by each call.  The
 * learned allocation is not offered here (MGARD_ERR_ARG).
 *
 * Container (little-endian): 'MGCK', u32 version 1, u32 ndim, u32 dtype,
 * u64 shape[4] (unused 0), u64 slab_planes, u64 n_slabs, f64 tol, u32 eb,
 * u32 0, f64 tau_abs, u64 offsets[n_slabs + 1] (byte offset of each slab's
 * stream; the last is the container's length), then the slab streams.
 */
uint64_t mgard_chunked_bound(uint32_t ndim, const uint64_t* shape, const double* const* coords, mgard_dtype dtype,
                             uint64_t slab_planes, const mgard_opts* opts);

/* h_in: the C-ordered host array; h_out: host buffer of out_capacity bytes
 * (MGARD_ERR_CAPACITY with *out_bytes = mgard_chunked_bound when short);
 * *out_bytes: the container's length. */
mgard_status mgard_compress_chunked(uint32_t ndim, const uint64_t* shape, const double* const* coords,
                                    mgard_dtype dtype, double tol, const void* h_in, uint64_t slab_planes,
                                    void* h_out, uint64_t out_capacity, uint64_t* out_bytes,
                                    const mgard_opts* opts);

/* Inverse of mgard_compress_chunked into the host array h_out;
 * MGARD_ERR_FORMAT for a malformed container or slab stream. */
mgard_status mgard_decompress_chunked(const void* h_in, uint64_t in_bytes, void* h_out, uint64_t out_capacity,
                                      const mgard_opts* opts);

/* ------------------------------------------------------- lossless stage
 * The final lossless stage (Sec. 2: quantized integers and precision
 * segments "are compressed through lossless encoding"), as zero
 * suppression, the redundancy this pipeline leaves after its entropy coder
 * (the all-zero shortest code of a dominant symbol, the mostly-zero high
 * bitplanes of the refactoring), in chunks coded independently:
 *   the input bytes, zero-padded to whole little-endian 32-bit words, in
 *   chunks of 4096 words (the last may be shorter, m words); level-1 bitmap:
 *   bit 31 - i%32 of word i/32 set when word i is nonzero; level-2 bitmap:
 *   the same over the level-1 words; a coded chunk is the level-2 bitmap,
 *   the nonzero level-1 words, the nonzero words, each in order, and the
 *   chunk is stored raw when that is not shorter than m words (a stored
 *   length of m means raw).
 * Container (little-endian): 'MGZS', u16 version 1, u16 0, u64 raw bytes,
 * u64 chunks, u64 word offsets[chunks + 1] of the stored chunks, then the
 * stored chunks.  mgard_decompress reads it as well as a plain stream. */

/* Largest container for raw_bytes of input. */
uint64_t mgard_lossless_bound(uint64_t raw_bytes);

/* Encodes raw_bytes of d_in (device, 4-byte aligned) into d_out (device,
 * out_capacity >= mgard_lossless_bound); *out_bytes receives the container's
 * size.  Synchronises opts->stream. */
mgard_status mgard_lossless_encode(const void* d_in, uint64_t raw_bytes, void* d_out, uint64_t out_capacity,
                                   uint64_t* out_bytes, const mgard_opts* opts);

/* Decodes a container (in_bytes at d_in, device) into d_out (device;
 * out_capacity >= the raw size rounded up to a multiple of 4: whole words
 * are written); *raw_bytes receives the raw size.  MGARD_ERR_FORMAT when the
 * offsets or a chunk's bitmaps do not match its stored length (checked
 * before any data word is read).  Synchronises opts->stream. */
mgard_status mgard_lossless_decode(const void* d_in, uint64_t in_bytes, void* d_out, uint64_t out_capacity,
                                   uint64_t* raw_bytes, const mgard_opts* opts);

/* ----------------------------------------------------------- refactoring
 * The refactoring module (Sec. 2, software design: multilevel coefficients
 * encoded into precision segments of different significance per level by
 * bitplane encoding, the error of each segment accumulated, retrieval that
 * fetches segments greedily by the error estimators; Sec. 3, second listing:
 * refactor, request a tolerance, fetch the needed components, reconstruct,
 * tolerance after tolerance).
 *
 * Per level l of the coefficient stream (stream order as for the stage
 * calls), with e_l the integer for which max|c| = f 2^e_l, 1/2 <= f < 1, and
 * B planes: m = floor(|c| 2^(B - e_l)) < 2^B and the sign bit c < 0.  The
 * level's segments are its sign plane, then planes k = 0..B-1 holding bit
 * B-1-k of every m, each packing the level's coefficients most significant
 * bit first into 32-bit words (coefficient i at bit 31 - i%32 of word i/32).
 * R_l[k] = max(m mod 2^(B-k)), k = 0..B, is the residual table; with the
 * first k planes, c^ = dtype(+-(m with its low B-k bits cleared) 2^(e_l-B))
 * and |c - c^| <= E_l[k] = (R_l[k]+1) 2^(e_l-B) + [k > 0] eps 2^e_l.
 *
 * Buffer (little-endian): 'MGRF', u16 version 1, u8 dtype, u8 ndim, u8 B,
 * u8 coordinate flags, u16 0, u32 L, f64 max|u|, f64 ||u|| (the L2 norm of
 * MGARD_NORM_S), u64 shape[ndim], f64 coordinates of each flagged dimension,
 * i32 e_l[L+1] (-2^31 for an all-zero level), u32 R[(L+1)(B+1)] level-major,
 * u64 level offsets[L+2] (bytes, in the segment area), zero padding to a
 * multiple of 8 bytes (the metadata ends there), then the segment area: per
 * level the sign plane and planes 0..B-1, ceil(N_l/32) words each. */

/* Exact size of the refactored buffer (0 for invalid arguments). */
uint64_t mgard_refactor_bound(uint32_t ndim, const uint64_t* shape, const double* const* coords, mgard_dtype dtype,
                              uint32_t planes);

/* Decomposes d_in (device) and writes the metadata and every segment of
 * `planes` (1..32) bitplanes per level into d_out (device, out_capacity >=
 * mgard_refactor_bound).  *out_bytes receives the size.  MGARD_ERR_NONFINITE
 * for a NaN or an infinity in the input.  Synchronises opts->stream. */
mgard_status mgard_refactor(uint32_t ndim, const uint64_t* shape, const double* const* coords, mgard_dtype dtype,
                            uint32_t planes, const void* d_in, void* d_out, uint64_t out_capacity,
                            uint64_t* out_bytes, const mgard_opts* opts);

/* Host only.  h_meta holds the first `bytes` bytes of a refactored buffer;
 * *meta_bytes receives the metadata's size (also, with MGARD_ERR_CAPACITY,
 * the bytes needed when they are too few); levels, planes and total_bytes
 * (nullable) receive L, B and the buffer's size.  MGARD_ERR_FORMAT for
 * malformed metadata. */
mgard_status mgard_refactor_inspect(const void* h_meta, uint64_t bytes, uint64_t* meta_bytes, uint32_t* levels,
                                    uint32_t* planes, uint64_t* total_bytes);

/* Host only: the retrieval plan.  From the planes already held per level
 * (h_have, L+1 entries; NULL = none), adds one plane at a time to the level
 * whose estimator term falls the most per byte fetched (a level's sign plane
 * counts with its first plane; ties to the lowest level) until the estimate
 * meets tau, and writes the planes to hold into h_want (max_levels >= L+1).
 * Estimators: MGARD_NORM_LINF (opts->norm): 4 (L+1) eps max|u| + E_0[k_0] +
 * sum_{l>=1} (1 + K_l) E_l[k_l] (K_l as for MGARD_ALLOC_PLAIN);
 * MGARD_NORM_S: max(1, 2^(sL)) sqrt(W_0) 4 (L+1) eps max|u| +
 * sqrt(sum_l 4^(s l) W_l E_l[k_l]^2).  tau = tol for MGARD_ABS, tol max|u|
 * (L-infinity) or tol ||u|| (s = 0) for MGARD_REL.  *h_estimate (nullable)
 * receives the estimate of h_want; when every plane is held and the estimate
 * still exceeds tau, h_want holds all planes and the call succeeds. */
mgard_status mgard_refactor_request(const void* h_meta, uint64_t bytes, double tol, const uint32_t* h_have,
                                    uint32_t* h_want, uint32_t max_levels, double* h_estimate,
                                    const mgard_opts* opts);

/* Host only: the byte ranges of a refactored buffer to fetch to go from
 * h_have to h_want planes per level (n_levels = L+1 entries each; NULL
 * h_have = none): at most one contiguous range per level, level by level,
 * offsets from the start of the buffer, into h_offsets / h_lengths (n_levels
 * entries each); *count receives the number of ranges. */
mgard_status mgard_refactor_ranges(const void* h_meta, uint64_t bytes, const uint32_t* h_have,
                                   const uint32_t* h_want, uint32_t n_levels, uint64_t* h_offsets,
                                   uint64_t* h_lengths, uint32_t* count);

/* Reconstruction from the first h_planes[l] planes of every level (n_levels
 * = L+1 entries, each <= B): d_in (device) holds a buffer of the full size
 * whose metadata and those segments are filled in (the rest is not read);
 * d_out (device) receives prod(shape) values of the stored dtype.  The
 * metadata is read back to the host and checked first. */
mgard_status mgard_reconstruct(const void* d_in, uint64_t in_bytes, const uint32_t* h_planes, uint32_t n_levels,
                               void* d_out, uint64_t out_capacity, const mgard_opts* opts);

/* ----------------------------------------------------------- measurement
 * Kernel timing with HIP events recorded on each launch's stream.
 * mgard_timing(1) clears earlier records and starts recording; (0) clears and
 * stops.  mgard_timing_report waits for the recorded events and writes one
 * line per kernel name, "name launches total_milliseconds", into h_buf
 * (capacity bytes, NUL-terminated); *needed receives the size required. */
mgard_status mgard_timing(int enable);
mgard_status mgard_timing_report(char* h_buf, uint64_t capacity, uint64_t* needed);

/* ----------------------------------------------------------- miscellaneous */
const char* mgard_last_error(void);
mgard_status mgard_release_workspace(void);
const char* mgard_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MGARD_HIP_H */
