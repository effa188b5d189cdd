/*
 * rdct.h -- C-ABI of the MI355X (gfx950) round-off DCT library (librdct.so).
 *
 * Method: R. J. Cintra and F. M. Bayer, "A DCT Approximation for Image
 * Compression".  An 8-bit greyscale plane is split into 8x8 blocks A (Section 3);
 * each block is transformed by the 2-D separable transform T A T^T with
 * T = C0 = [2 C], the element-wise round-off of twice the DCT matrix, whose
 * entries are 0 and +-1 (Section 2).  The orthogonalising diagonal S (Section 2,
 * S = sqrt((C0 C0^T)^-1) = diag(1/sqrt(g)), g = (8,6,4,6,8,6,4,6)) is never
 * applied to pixels: it is folded into the step that follows the transform,
 * either the retention of the first r zig-zag coefficients (Section 3) or a
 * quantisation table (Section 2 folds S into the quantisation).  The
 * inverse runs through the transpose, since C_orth = S C0 is orthogonal
 * (Section 2), and the result is scored by SSE / MSE / PSNR (Section 3).
 *
 * Conventions for every entry point
 *  - Buffer pointers are DEVICE pointers owned by the caller unless a comment
 *    says "host".  The library keeps no reference after the call returns,
 *    except for the plan and server objects, which document their own.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Every
 *    compute call is asynchronous on it: arguments are validated synchronously,
 *    before any launch; faults inside kernels surface at the caller's next
 *    synchronisation of the stream.
 *  - Hot-path calls (forward, inverse, compress_eval, batch_run) allocate no
 *    memory.  Plan and server creation allocate and say so.
 *  - Planes are W x H uint8 with a row pitch in bytes >= W.  Sides that are not
 *    multiples of 8 are padded by replicating the last row / column; metrics
 *    cover only the plane's own pixels.
 *  - Coefficients are block-major: block (by, bx) (raster order over
 *    ceil(H/8) x ceil(W/8) blocks) holds 64 consecutive values in natural order
 *    k * 8 + l, k = vertical and l = horizontal frequency.
 *  - Zig-zag order is the JPEG sequence starting (0,0), (0,1), (1,0), (2,0), ...
 *  - Return value: RDCT_OK or an error code; no global error state.
 */
#ifndef RDCT_H_
#define RDCT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RDCT_OK = 0,
  RDCT_ERR_INVALID_ARG = 1, /* null pointer, bad size/pitch/r/quality/table, bad enum */
  RDCT_ERR_UNSUPPORTED = 2, /* valid but not provided (see each call) */
  RDCT_ERR_HIP = 3,         /* a HIP runtime call or launch failed */
  RDCT_ERR_NO_MEMORY = 4,   /* plan / server creation could not allocate */
  RDCT_ERR_BUDGET = 5,      /* server: request larger than the whole device budget */
  RDCT_ERR_NOT_FOUND = 6,   /* server: unknown ticket */
  RDCT_ERR_BUSY = 7,        /* server: queue or staging full (non-blocking submit) */
  RDCT_ERR_CANCELLED = 8    /* server: the request was cancelled before admission */
} rdct_status_t;

/* Element type of a coefficient buffer. */
typedef enum {
  RDCT_COEF_I32 = 0, /* int32: integer Y = C0 A C0^T, or quantised q          */
  RDCT_COEF_I16 = 1, /* int16: same values; exact since |Y| <= 16320          */
  RDCT_COEF_F32 = 2  /* float: scaled C_orth coefficients Z = S Y S           */
} rdct_coef_t;

/* What follows the transform. */
typedef enum {
  RDCT_SEL_NONE = 0,   /* keep all 64 coefficients                                   */
  RDCT_SEL_ZIGZAG = 1, /* keep the first r zig-zag coefficients, zero the rest (Sec. 3) */
  RDCT_SEL_QUANT = 2   /* q = round(Z / Q), halves away from zero, decided exactly     */
} rdct_sel_mode_t;

typedef struct {
  int32_t mode;            /* rdct_sel_mode_t                                          */
  int32_t r;               /* ZIGZAG: coefficients kept, 1..64 (the paper uses 1..45)  */
  int32_t quality;         /* QUANT: 1..100, IJG scaling of the JPEG luminance table   */
  int32_t level_shift;     /* 0..255 subtracted from every pixel before the transform
                              and added back after the inverse (JPEG uses 128)         */
  const uint16_t* qtable;  /* QUANT: optional HOST pointer to 64 entries (1..255),
                              natural order; NULL = derive from `quality`              */
} rdct_select_t;

/* ------------------------------------------------------------------------- */
/* Core path                                                                  */
/* ------------------------------------------------------------------------- */

/*
 * Forward transform of one plane (Section 3: T A T^T on every 8x8 sub-block,
 * T = C0; 22 additions per 8-point pass, Section 2 / Table 1).
 *   src        plane, `height` rows of `src_pitch` bytes (>= width).
 *   sel        host pointer.  NONE: coef = Y.  ZIGZAG: Y (I32/I16) or Z (F32)
 *              with positions of zig-zag rank >= r set to 0.  QUANT: q (I32/I16).
 *   coef       ceil(H/8) * ceil(W/8) * 64 elements of `coef_type`.
 *   F32 output is fl32 of the exact s_k s_l Y_kl (error <= 3.1e-5).
 * Errors: INVALID_ARG (nulls, sizes <= 0, pitch < width, r or quality out of
 * range, F32 with QUANT), HIP.
 */
rdct_status_t rdct_forward(const uint8_t* src, int32_t width, int32_t height,
                           int64_t src_pitch, const rdct_select_t* sel,
                           void* coef, rdct_coef_t coef_type, void* stream);

/*
 * Inverse transform (Section 3 inverts the kept coefficients; C_orth^-1 = C_orth^T,
 * Section 2) of block-major coefficients back to a float plane.
 *   coef_type I32/I16 with NONE or ZIGZAG: integer Y, positions of rank >= r
 *     ignored; A' = C0^T D' Y D' C0 / 576 (D' = diag(24/g)), exact integer
 *     numerator, one rounding to float.
 *   coef_type F32 with NONE or ZIGZAG: Z; A' = C_orth^T Z C_orth in float64.
 *   coef_type I32/I16 with QUANT: q; A' = C_orth^T (q . Q) C_orth in float64.
 *   `level_shift` is added back.  dst: height rows of dst_pitch floats.
 * Errors: INVALID_ARG, HIP.
 */
rdct_status_t rdct_inverse(const void* coef, rdct_coef_t coef_type,
                           int32_t width, int32_t height, const rdct_select_t* sel,
                           float* dst, int64_t dst_pitch, void* stream);

/*
 * Fused compress-and-evaluate (Section 3: transform, keep r or quantise,
 * inverse, squared error) in one launch.
 *   sel->mode ZIGZAG: r_count >= 1 values r = sel->r .. sel->r + r_count - 1
 *     (all <= 64) are scored; sse_out[i] = sum over the plane of (576 A - R)^2
 *     for r = sel->r + i, exact, in units of 1/576^2 (SSE = sse_out / 331776).
 *     r_count > 1 needs width and height to be multiples of 8 (else
 *     UNSUPPORTED); it uses the identity sum (576A - R)^2 = 576 sum over the
 *     dropped positions of d'_k d'_l Y_kl^2, which holds because C_orth is
 *     orthogonal.
 *   sel->mode QUANT: r_count must be 1; sse_out[0] = sum over blocks of
 *     round(2^20 * block SSE), the block SSE taken in float64 (SSE =
 *     sse_out / 2^20).
 *   sel->mode NONE: as ZIGZAG with r = 64, r_count = 1.
 *   coef_out   optional (NULL = not written): the coefficients at r = sel->r
 *              (ZIGZAG: masked Y or Z; QUANT: q).
 *   recon_out  optional float plane at r = sel->r (same as rdct_inverse would
 *              give on coef_out), recon_pitch floats per row.
 *   sse_out    device, r_count uint64 entries, overwritten.
 * Planes of up to 6,000,000 blocks are accepted (the uint64 sums cannot wrap).
 */
rdct_status_t rdct_compress_eval(const uint8_t* src, int32_t width, int32_t height,
                                 int64_t src_pitch, const rdct_select_t* sel,
                                 int32_t r_count, void* coef_out, rdct_coef_t coef_type,
                                 float* recon_out, int64_t recon_pitch,
                                 uint64_t* sse_out, void* stream);

/* Units of sse_out for a selection mode: 1/576^2 (NONE, ZIGZAG) or 2^-20 (QUANT). */
double rdct_sse_unit(int32_t mode);

/* PSNR in dB of a plane from its sse_out value: 10 log10(255^2 / MSE),
   MSE = sse_out * rdct_sse_unit(mode) / (width * height); +inf when 0. */
double rdct_psnr(uint64_t sse, int32_t mode, int32_t width, int32_t height);

/*
 * PSNR of many planes at once (Section 3: PSNR per image, and the average PSNR
 * over images as the mean of their dB values).  HOST arrays.
 *   sse       n * r_count raw sums in units of rdct_sse_unit(mode): plane i's
 *             r_count sums at sse[i * r_count ...] (a sweep; r_count = 1 otherwise).
 *   widths, heights   n plane sizes.
 *   psnr_out  n * r_count values in the layout of sse (+inf for an exact
 *             reconstruction).
 *   mean_out  optional (NULL = not written): r_count means over the n planes.
 * Errors: INVALID_ARG (null arrays, n < 0, r_count < 1, a size <= 0, bad mode).
 */
rdct_status_t rdct_psnr_planes(const uint64_t* sse, int32_t n, int32_t r_count, int32_t mode,
                               const int32_t* widths, const int32_t* heights, double* psnr_out,
                               double* mean_out);

/*
 * rdct_psnr_planes on the device, asynchronous on `stream`: the decibels are
 * formed where the sums are, so a caller that reads results back copies them
 * and does no per-value arithmetic on the host.  DEVICE arrays:
 *   sse       n * r_count raw sums (layout of rdct_psnr_planes);
 *   pixels    n plane sizes in pixels (width * height);
 *   psnr_out  n * r_count values, +inf for an exact reconstruction;
 *   mean_out  optional: r_count means over the n planes (NaN when n = 0).
 * No allocation.  Errors: INVALID_ARG (null or misaligned arrays, n < 0,
 * r_count < 1, bad mode), UNSUPPORTED (more than 2^31 values), HIP.
 */
rdct_status_t rdct_psnr_device(const uint64_t* sse, int32_t n, int32_t r_count, int32_t mode,
                               const int64_t* pixels, double* psnr_out, double* mean_out,
                               void* stream);

/* Number of 8x8 blocks of a plane: ceil(h/8) * ceil(w/8). */
int64_t rdct_num_blocks(int32_t width, int32_t height);

/* ------------------------------------------------------------------------- */
/* Batched planes: one persistent launch over a device-side block work list   */
/* ------------------------------------------------------------------------- */

/* One plane of a batch.  Pointers are DEVICE pointers that must stay valid
   while the plan exists (the plan records them). */
typedef struct {
  const uint8_t* src;      /* plane, height rows of src_pitch bytes              */
  int32_t width, height;
  int64_t src_pitch;
  rdct_select_t sel;       /* per-plane r / quality / table / level shift; the
                              mode (ZIGZAG or QUANT; NONE = ZIGZAG with r = 64)
                              must be the same for every plane of a plan          */
  void* coef_out;          /* block-major coefficients (nullable; null for all
                              planes or for none)                                 */
  float* recon_out;        /* reconstruction (nullable; null for all or none)     */
  int64_t recon_pitch;     /* floats per reconstruction row                       */
} rdct_plane_desc_t;

/* Launch geometry of a batch plan. */
typedef enum {
  RDCT_LAYOUT_DEFAULT = 0,    /* from the tuning cache, else STRIDED                  */
  RDCT_LAYOUT_STRIDED = 1,    /* persistent workgroups stride over every plane's work
                                 items; a clearing launch, then sums added atomically */
  RDCT_LAYOUT_PER_PLANE = 2   /* one workgroup per plane, its waves striding over the
                                 plane's items; sums stored, no clearing launch
                                 (wgs_per_cu unused); suits many similar planes      */
} rdct_layout_t;

typedef struct {
  int32_t waves_per_wg;    /* 1, 2 or 4; 0 = from the tuning cache or default      */
  int32_t wgs_per_cu;      /* resident workgroups per compute unit, 1..16; 0 = same */
  int32_t use_graph;       /* 1: runs replay a captured hipGraph; 0: plain launches
                              (the default with a NULL tuning: measured faster)      */
  int32_t layout;          /* rdct_layout_t                                         */
  int32_t xcd_ranges;      /* STRIDED: 1 = workgroups remapped so that each of the
                              eight XCDs (each with its own L2) takes a contiguous
                              range of work items, so neighbouring items share an
                              L2 (the default, and the order the autotuner times);
                              0 = the hardware's round-robin order                  */
  int32_t strip;           /* STRIDED: consecutive 128-block work items a wave takes
                              before striding, 1, 2, 4 or 8; 0 = from the tuning
                              cache or default (explicit tunings only)              */
} rdct_tuning_t;

typedef struct rdct_batch_plan rdct_batch_plan_t;

/*
 * Build a plan over n planes (Section 3's per-block procedure applied to every
 * block of every plane): a device work list of 128-block items, the per-plane
 * descriptors and quantisation tables are uploaded once.  Each run computes,
 * for every plane, what rdct_compress_eval computes with r_count = 1 (same
 * kernels, identical per-block results): coefficients, reconstruction and
 * sse_out[i] (units of rdct_sse_unit(mode)), overwritten.
 * Allocates device memory (the plan's tables) -- not a hot call.
 * tuning: NULL = tuning cache or defaults (a cache entry that is not a valid
 * geometry is ignored); zero fields of a given tuning take the same sources.
 * Errors: INVALID_ARG (any plane invalid, mixed modes or output nullness, a
 * tuning field out of range -- checked before anything is allocated),
 * UNSUPPORTED, NO_MEMORY, HIP.
 */
rdct_status_t rdct_batch_plan_create(const rdct_plane_desc_t* planes, int32_t n,
                                     rdct_coef_t coef_type, uint64_t* sse_out,
                                     const rdct_tuning_t* tuning, rdct_batch_plan_t** out);

/*
 * A batched retention sweep (Section 3, keep the r initial zig-zag coefficients,
 * for a range of r): every plane's sel has mode ZIGZAG and gives the first r,
 * and each run writes sse_out[i * r_count + j] = the error of plane i at
 * r = sel.r + j (units of rdct_sse_unit(RDCT_SEL_ZIGZAG)), exactly what
 * rdct_compress_eval gives for that plane alone with the same r_count.  The
 * sums come from coefficient energies (Parseval through the exact inverse), so
 * every plane must consist of whole blocks (width and height multiples of 8);
 * coefficients and reconstruction (kept at r = sel.r) are optional as in
 * rdct_batch_plan_create.  sse_out holds n * r_count entries.
 * Errors: INVALID_ARG (r_count < 1, a mode other than ZIGZAG with r_count > 1,
 * sel.r + r_count - 1 > 64, or any error of rdct_batch_plan_create),
 * UNSUPPORTED (a plane with a partial block), NO_MEMORY, HIP.
 */
rdct_status_t rdct_batch_plan_create_sweep(const rdct_plane_desc_t* planes, int32_t n,
                                           int32_t r_count, rdct_coef_t coef_type,
                                           uint64_t* sse_out, const rdct_tuning_t* tuning,
                                           rdct_batch_plan_t** out);

/* Run the plan on `stream` (asynchronous; no allocation).  STRIDED layout: a
   launch that clears sse_out, then the persistent kernel; PER_PLANE: one launch.
   With use_graph the first run captures the launches into a hipGraph; later runs
   replay it.  Runs of one plan must not overlap (on two streams at once): they
   share the plan's outputs. */
rdct_status_t rdct_batch_run(rdct_batch_plan_t* plan, void* stream);

/* Run the plan with this geometry from now on (every field given, none taken
   from the cache, except that strip 0 means 1; not stored in the cache).
   Errors: INVALID_ARG (not a valid geometry: waves_per_wg 1, 2 or 4,
   wgs_per_cu 1..16, a known layout, xcd_ranges 0 or 1, strip 1, 2, 4 or 8). */
rdct_status_t rdct_batch_plan_set_tuning(rdct_batch_plan_t* plan, const rdct_tuning_t* tuning);

/* Blocks and work items of a plan, and the geometry it runs with (any pointer
   may be NULL). */
rdct_status_t rdct_batch_plan_info(const rdct_batch_plan_t* plan, int64_t* n_blocks,
                                   int32_t* n_items, rdct_tuning_t* used);

/* Tune the plan's geometry by timing it on the plan (synchronous).  Timing:
   five rounds that each queue reps launches of every candidate in turn, back
   to back, with HIP events between candidates; a candidate's median round is
   its time.  Stage 1 times both layouts over waves per workgroup and resident
   waves per CU (strip 1) and takes, among the candidates within 2% of the
   fastest, the one with the fewest resident waves per CU (then the faster);
   for a strided pick, stage 2 times strips 1, 2, 4 and 8 and takes the
   fastest.  The result is adopted, stored in the tuning cache (file named by
   RDCT_TUNING_CACHE, default ~/.cache/rdct_tuning.json, keyed by architecture,
   path variant, size class and plane-count class) and returned in *best. */
rdct_status_t rdct_batch_autotune(rdct_batch_plan_t* plan, int32_t reps, void* stream,
                                  rdct_tuning_t* best);

/* Release the plan's device memory and graph (synchronises its internal stream). */
void rdct_batch_plan_destroy(rdct_batch_plan_t* plan);

/* ------------------------------------------------------------------------- */
/* Codec output: run-length coded kept coefficients and 8-bit pixels          */
/* ------------------------------------------------------------------------- */

/* Number of 64-block groups of a plane: ceil(ceil(W/8) ceil(H/8) / 64). */
int64_t rdct_codec_groups(int32_t width, int32_t height);

/*
 * Store what Section 3's procedure keeps: for every block, the kept
 * coefficients in zig-zag order as (run, value) pairs -- run = zeros before a
 * non-zero value, trailing zeros implied by the pair count, the DC coded like
 * the rest -- and optionally the 8-bit reconstruction clamp(round(A'), 0, 255)
 * (round half away from zero).
 *   sel         ZIGZAG: ranks 0 .. r-1 of Y are kept (NONE: all 64); the pixels
 *               come from the exact numerator, floor((R + 288) / 576).  QUANT: all
 *               64 values q are kept; A' in float64 plus the level shift.
 *   counts      device, ceil(W/8) ceil(H/8) uint16: pairs per block.
 *   group_pairs device, rdct_codec_groups uint32: pairs per 64-block group.
 *   slots       device, rdct_codec_groups * 4096 int32: group g's pairs, in block
 *               order, at slots + 4096 g.  A pair is (run << 16) | (uint16)value
 *               (|Y| <= 16320 and |q| < 2^15 fit in 16 bits).
 *   recon_u8    optional 8-bit plane, recon_pitch bytes per row.
 * Planes up to 2^22 blocks.  No allocation.
 * Errors: INVALID_ARG, UNSUPPORTED (size), HIP.
 */
rdct_status_t rdct_codec_encode(const uint8_t* src, int32_t width, int32_t height,
                                int64_t src_pitch, const rdct_select_t* sel, uint16_t* counts,
                                uint32_t* group_pairs, int32_t* slots, uint8_t* recon_u8,
                                int64_t recon_pitch, void* stream);

/*
 * Concatenate the groups written by rdct_codec_encode into one stream:
 * offsets[b] = index in `packed` of block b's first pair (nblocks + 1 entries,
 * offsets[nblocks] = total), packed = all pairs in block order.  Pairs at
 * index >= capacity are not written (compare offsets[nblocks] with capacity;
 * 64 pairs per block always suffice).  workspace: rdct_codec_groups uint32.
 * No allocation.  Errors: INVALID_ARG, UNSUPPORTED (size), HIP.
 */
rdct_status_t rdct_codec_pack(const uint16_t* counts, const uint32_t* group_pairs,
                              const int32_t* slots, int32_t width, int32_t height,
                              uint32_t* offsets, int32_t* packed, int64_t capacity,
                              uint32_t* workspace, void* stream);

/*
 * rdct_codec_pack without a caller workspace, for callers that cannot allocate
 * or pass scratch memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments and results as
 * rdct_codec_pack minus `workspace`: the chunk prefixes go to a fixed device
 * array of the library's own (256 KiB per GPU, held until the process ends),
 * which covers the largest plane the codec accepts (2^22 blocks); larger
 * planes return UNSUPPORTED.  Allocates nothing.  Every call on one GPU uses
 * that GPU's one array, so calls that overlap on one GPU (two streams, or two
 * host threads) race and must be serialised by the caller; nothing in the
 * array needs to start at zero.  The first call on a device looks the array's
 * address up.  Errors: INVALID_ARG, UNSUPPORTED (size), HIP.
 */
rdct_status_t rdct_codec_pack_noalloc(const uint16_t* counts, const uint32_t* group_pairs,
                                      const int32_t* slots, int32_t width, int32_t height,
                                      uint32_t* offsets, int32_t* packed, int64_t capacity,
                                      void* stream);

/* Decode n pair words of the packed stream (HOST arrays): run_out[i] = word >> 16,
   value_out[i] = the signed 16-bit low half.  Errors: INVALID_ARG (null arrays
   with n > 0, n < 0). */
rdct_status_t rdct_codec_unpack_pairs(const int32_t* words, int64_t n, int32_t* run_out,
                                      int32_t* value_out);

/* ------------------------------------------------------------------------- */
/* Comparison transforms and image-quality metrics (Sections 2-4)             */
/* ------------------------------------------------------------------------- */

/* An 8x8 transform T applied to every block as T A T^T (Section 3); the keep-r
   reconstruction is A' = T^-1 (M_r . T A T^T) T^-T. */
typedef enum {
  RDCT_T_RDCT = 0,       /* C_orth = S C0, C0 = [2 C] (Section 2)                       */
  RDCT_T_DCT = 1,        /* the exact DCT C, the reference of Section 3's comparison     */
  RDCT_T_SDCT = 2,       /* signed DCT sign(C) / sqrt(8) (Section 2); not orthogonal:
                            the inverse is the matrix inverse (8 sign(C)^-1 is integral) */
  RDCT_T_RDCT_CEIL = 3,  /* (C0 C0^T)^(-1/2) C0 with C0 = ceil(2 C) (Section 4: ceiling in
                            place of the round-off; C0 C0^T is a full matrix)            */
  RDCT_T_RDCT_FLOOR = 4  /* C0 = floor(2 C): its first row is zero and C0 C0^T singular,
                            so no approximation exists -- every call returns UNSUPPORTED */
} rdct_transform_t;

/*
 * Keep-r sweep of one plane under one transform (Section 3), scored by SSE and
 * by the universal quality index (UQI; the index of Wang and Bovik that
 * Section 3 uses, evaluated over every 8x8 window at stride 1).  For every r in
 * r_first .. r_first + r_count - 1 (1 <= r, last <= 64):
 *   sse_out[i]  sum over the plane of (A - A'_r)^2 in units of
 *               rdct_quality_sse_unit(transform): exact for RDCT (1/576^2) and
 *               SDCT (1/64^2); for DCT and RDCT_CEIL float64 sums rounded to
 *               2^-20 per 32 x 32 tile of windows.
 *   uqi_out[i]  sum over the (H - 7)(W - 7) windows of
 *               Q = [2 s_xy / (s_x^2 + s_y^2)] [2 xbar ybar / (xbar^2 + ybar^2)]
 *               (a factor whose denominator is 0 counts as 1; so that float64
               noise in exactly flat blocks cannot decide it, a reconstruction
               window with variance <= 2^-32 grey levels^2 counts as flat and a
               window mean of magnitude <= 2^-32 as 0; both bounds lie below
               the resolution of the RDCT and SDCT integer numerators, so for
               those only exactly flat or zero-mean windows qualify), as int64 in units
 *               of 2^-32 (float64 per tile, then rounded); mean UQI =
 *               uqi_out * 2^-32 / rdct_quality_windows(width, height).  For RDCT and
 *               SDCT the window sums are exact integers, so only each window's
 *               final quotient rounds (its two factors are formed as one
 *               product over one product, then divided once).
 * The reconstruction is real-valued (no rounding or clipping).  Width and height
 * must be multiples of 8 (else UNSUPPORTED); planes up to 2^20 blocks.  Both
 * outputs are device arrays of r_count entries, overwritten.  No allocation.
 * Errors: INVALID_ARG, UNSUPPORTED (sizes, RDCT_T_RDCT_FLOOR), HIP.
 */
rdct_status_t rdct_quality_sweep(const uint8_t* src, int32_t width, int32_t height,
                                 int64_t src_pitch, int32_t transform, int32_t r_first,
                                 int32_t r_count, uint64_t* sse_out, int64_t* uqi_out,
                                 void* stream);

/* Units of rdct_quality_sweep's sse_out: 1/576^2 (RDCT), 1/64^2 (SDCT), 2^-20
   (DCT, RDCT_CEIL); 0 for an invalid transform. */
double rdct_quality_sse_unit(int32_t transform);

/* Number of 8x8 windows at stride 1: (width - 7) * (height - 7), 0 if smaller. */
int64_t rdct_quality_windows(int32_t width, int32_t height);

/*
 * Metrics of one plane from rdct_quality_sweep's raw sums (Section 3: MSE and
 * the mean UQI over the plane's windows).  HOST arrays of n entries:
 *   mse_out[i] = sse[i] * rdct_quality_sse_unit(transform) / (width * height)
 *   uqi_out[i] = uqi[i] * 2^-32 / rdct_quality_windows(width, height)
 * Errors: INVALID_ARG (null arrays with n > 0, n < 0, an invalid transform, a
 * plane smaller than one 8x8 window).
 */
rdct_status_t rdct_quality_metrics(const uint64_t* sse, const int64_t* uqi, int32_t n,
                                   int32_t transform, int32_t width, int32_t height,
                                   double* mse_out, double* uqi_out);

/* One plane of a quality plan (DEVICE pointer, valid while the plan exists). */
typedef struct {
  const uint8_t* src;
  int32_t width, height;
  int64_t src_pitch;
} rdct_quality_desc_t;

typedef struct rdct_quality_plan rdct_quality_plan_t;

/*
 * Plan over n planes and one transform: every run computes rdct_quality_sweep
 * for each plane in one launch (a device list of 32 x 32 window tiles).  Plane i
 * writes sse_out[i * r_count + j] and uqi_out[i * r_count + j].  Allocates
 * device memory (tile list and descriptors) -- not a hot call.
 * Errors: as rdct_quality_sweep, plus NO_MEMORY.
 */
rdct_status_t rdct_quality_plan_create(const rdct_quality_desc_t* planes, int32_t n,
                                       int32_t transform, int32_t r_first, int32_t r_count,
                                       uint64_t* sse_out, int64_t* uqi_out,
                                       rdct_quality_plan_t** out);

/* Run the plan on `stream` (asynchronous; no allocation). */
rdct_status_t rdct_quality_plan_run(rdct_quality_plan_t* plan, void* stream);

void rdct_quality_plan_destroy(rdct_quality_plan_t* plan);

/* ------------------------------------------------------------------------- */
/* Compression server: admission by device-memory budget, continuous batching */
/* ------------------------------------------------------------------------- */

typedef struct rdct_server rdct_server_t;

typedef struct {
  int64_t budget_bytes;     /* device memory for admitted requests (planes, descriptors,
                               error sums); the server allocates it once at creation     */
  int64_t staging_bytes;    /* pinned host staging for submitted requests (0 = budget/4,
                               at most 2 GiB)                                             */
  int32_t max_inflight;     /* requests admitted and not yet completed (0 = 4096)         */
  int32_t max_batch_planes; /* planes per launch (0 = 4096)                               */
  int32_t n_streams;        /* device streams, batches in flight at once: 1..4 (0 = 2)    */
  int32_t plain;            /* 1: no batching -- each plane runs alone (copy, launch,
                               synchronise) in submission order; the comparison path      */
} rdct_server_cfg_t;

/* A request: 1..3 planes of one picture (e.g. Y, Cb, Cr of 4:2:0), all scored with
   the same selection.  The planes are HOST pointers; submit copies them, so the
   caller may reuse its buffers as soon as submit returns. */
typedef struct {
  const uint8_t* planes[3];
  int32_t width[3], height[3];
  int64_t pitch[3];         /* bytes per host row (>= width)                            */
  int32_t n_planes;
  rdct_select_t sel;        /* ZIGZAG (r) or QUANT; no coefficient output               */
  uint64_t user_tag;
} rdct_request_t;

typedef struct {
  uint64_t ticket;
  uint64_t user_tag;
  int32_t status;           /* RDCT_OK, RDCT_ERR_CANCELLED or RDCT_ERR_HIP              */
  int32_t n_planes;
  uint64_t sse[3];          /* raw error sums, units rdct_sse_unit(mode)                */
  double psnr[3];           /* dB, +inf for an exact reconstruction                     */
  double t_submit_us;       /* times in microseconds since the server was created       */
  double t_launch_us;       /* when its batch was launched                               */
  double t_done_us;         /* when the server saw the batch complete                    */
  int32_t batch_planes;     /* planes in the launch that carried it                      */
  int32_t reserved;
} rdct_completion_t;

typedef struct {
  int64_t submitted, completed, cancelled, rejected;
  int64_t batches, planes, blocks;
  int64_t peak_device_bytes;   /* high-water mark of the budget in use */
  int64_t device_bytes_in_use;
  int32_t pending, inflight;
} rdct_server_stats_t;

/* Create a server (allocates the device budget and pinned staging; starts one
   scheduler thread).  Errors: INVALID_ARG, NO_MEMORY, HIP. */
rdct_status_t rdct_server_create(const rdct_server_cfg_t* cfg, rdct_server_t** out);

/* Queue a request without blocking.  Errors: INVALID_ARG (bad plane or selection),
   BUDGET (the request alone exceeds the device budget: it could never be admitted),
   BUSY (staging full -- retry later). */
rdct_status_t rdct_server_submit(rdct_server_t* srv, const rdct_request_t* req, uint64_t* ticket);

/* Move up to `max` completions into out[]; waits up to wait_us microseconds for the
   first one (0 = do not wait).  *n receives the count. */
rdct_status_t rdct_server_poll(rdct_server_t* srv, rdct_completion_t* out, int32_t max,
                               int32_t* n, int32_t wait_us);

/* Cancel a request that has not been admitted yet: it completes with
   RDCT_ERR_CANCELLED.  NOT_FOUND if the ticket is unknown, BUSY if already admitted. */
rdct_status_t rdct_server_cancel(rdct_server_t* srv, uint64_t ticket);

/* Block until every submitted request has completed (or timeout_ms passes:
   RDCT_ERR_BUSY). */
rdct_status_t rdct_server_drain(rdct_server_t* srv, int32_t timeout_ms);

rdct_status_t rdct_server_stats(rdct_server_t* srv, rdct_server_stats_t* out);

/* Stop the scheduler, wait for launched work, free everything.  Pending requests
   are dropped. */
void rdct_server_destroy(rdct_server_t* srv);

/* ------------------------------------------------------------------------- */
/* Bandwidth calibration (no part of the method)                              */
/* ------------------------------------------------------------------------- */

/* Read:write patterns of rdct_stream, per unit of one wave. */
typedef enum {
  RDCT_STREAM_READ = 0,      /* 8 KiB read                                   */
  RDCT_STREAM_WRITE = 1,     /* 16 KiB written                               */
  RDCT_STREAM_COPY = 2,      /* 8 KiB read, 8 KiB written                    */
  RDCT_STREAM_R1W2 = 3,      /* 8 KiB read, 16 KiB written (frame quantiser) */
  RDCT_STREAM_R1W6 = 4       /* 4 KiB read, 24 KiB written (batch with
                                int16 coefficients and float reconstruction) */
} rdct_stream_pattern_t;

/* Bytes one unit of `pattern` reads and writes (either pointer may be NULL). */
rdct_status_t rdct_stream_unit_bytes(int32_t pattern, int64_t* read_bytes, int64_t* write_bytes);

/*
 * Move `units` units of `pattern` from src to dst (DEVICE pointers, 16-byte
 * aligned): the streaming reference the HBM rooflines of the transform kernels
 * are read against.  Each wave instruction reads or writes 1 KiB (16 bytes per
 * lane).  src holds units * read bytes; dst holds units * written bytes (at
 * least 1 KiB for RDCT_STREAM_READ, where it is written only for one value of
 * the data).  flags: bit 0 = nontemporal loads, bit 1 = nontemporal stores,
 * bit 2 = workgroups remapped so that each XCD takes a contiguous range.
 * wgs_per_cu: 0 = one unit per wave (the grid covers the units), else that many
 * persistent 4-wave workgroups per compute unit (1..32) stride over them.
 * Asynchronous on `stream`; no allocation.
 * Errors: INVALID_ARG, UNSUPPORTED (more than 2^34 units), HIP.
 */
rdct_status_t rdct_stream(const void* src, void* dst, int64_t units, int32_t pattern,
                          int32_t flags, int32_t wgs_per_cu, void* stream);

const char* rdct_status_string(rdct_status_t status);

/* Library version string and the GPU architecture it was built for. */
const char* rdct_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RDCT_H_ */
