/*
 * sprintz.h -- C ABI of the MI355X (gfx950) Sprintz codec.
 *
 * Sprintz (Blalock, Madden & Guttag, IMWUT 2018) compresses a multivariate
 * integer time series: T samples (rows) of D columns, every element an
 * integer of bitwidth w = 8 or 16 stored row-major (Section 2.1,
 * Definitions). Per column a forecaster predicts each sample (delta coding,
 * Section 4.2.1, or FIRE, Section 4.2.2 / Algorithm 3); the errors are
 * zigzag coded, every block of 8 rows gets one bit width per column, the
 * block is bit packed behind a header of log2(w)-bit width codes, and runs of
 * all-zero blocks become a single run-length record (Algorithm 1, Section
 * 4.3). Decompression inverts this (Algorithm 2).
 *
 * For parallelism the series is cut into independently coded segments of
 * seg_rows rows; every segment restarts the forecaster state at zero, exactly
 * as the paper starts a stream. The container is self-describing:
 *
 *   64-byte header | (nseg+1) x u64 segment offsets | pad to 16 | segments
 *   segment = u32 nrec | header groups | raw tail rows | pad to 16
 *
 * Conventions for every entry point below:
 *   - Pointers named d_* are device pointers (HIP global memory) on the
 *     current device; h_* are host pointers. The caller owns every buffer;
 *     the library never allocates, frees or retains caller memory.
 *   - Work is enqueued on `stream` and is asynchronous; nothing is
 *     synchronised. Host-detectable argument errors are returned at once
 *     and then nothing is enqueued.
 *   - Device-detected problems (a corrupt container, an internal size
 *     mismatch) are ORed into *d_status as nonzero bits; *d_status must be 0
 *     on entry and may be NULL to skip device-side reporting. The kernels
 *     never trap and never write outside [d_dst, d_dst + dst_cap).
 *   - int8/uint8 (and int16/uint16) produce identical bytes: the codec works
 *     on w-bit patterns modulo 2^w. The dtype is recorded only so that the
 *     decoder can report it.
 *   - GPU limits: 1 <= D <= 128, 8 <= seg_rows <= 2^20 with seg_rows % 8 == 0,
 *     hdr_group <= 255, learn_shift <= 8. Outside them the call returns
 *     SPZ_EUNSUPPORTED (D) or SPZ_EINVAL (the rest).
 */
#ifndef SPRINTZ_H_
#define SPRINTZ_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPZ_OK = 0,
    SPZ_EINVAL = -1,        /* bad argument */
    SPZ_ENOSPC = -2,        /* destination or workspace too small */
    SPZ_ECORRUPT = -3,      /* container header invalid */
    SPZ_EUNSUPPORTED = -4,  /* valid request outside the GPU limits */
    SPZ_EHIP = -5,          /* a HIP runtime call failed */
    SPZ_ENOMEM = -6
} spz_status;

typedef enum { SPZ_INT8 = 1, SPZ_UINT8 = 2, SPZ_INT16 = 3, SPZ_UINT16 = 4 } spz_dtype;

/* Section 4.2: delta coding or FIRE (Fast Integer REgression). */
typedef enum { SPZ_DELTA = 0, SPZ_FIRE = 1 } spz_forecaster;

typedef struct {
    uint32_t struct_size;  /* sizeof(spz_params) */
    uint32_t forecaster;   /* spz_forecaster */
    uint32_t seg_rows;     /* rows per independently coded segment (multiple of 8);
                              0 = autotuned (compression only: see sprintz_autotune) */
    uint32_t hdr_group;    /* records whose headers are stored together (Section 4.3,
                              last paragraph); 0 = one group per segment */
    uint32_t learn_shift;  /* FIRE learning rate eta = 2^-learn_shift (paper: eta = 1/2) */
    uint32_t entropy;      /* 0 = none; 1 = Huffman coding of every segment's packed
                              bytes (Section 4.4, Entropy Coding; the coder and its format
                              are this library's: one canonical code of at most 11-bit
                              codes per segment, 16 sub-streams). Compression needs
                              a plain container's space in the workspace; the coded
                              segment image must fit 60 KiB of LDS
                              (SPZ_EUNSUPPORTED otherwise) */
} spz_params;

typedef struct {
    uint64_t rows;
    uint32_t D;
    uint32_t dtype;             /* spz_dtype */
    spz_params params;
    uint64_t compressed_size;   /* total container bytes */
    uint64_t decompressed_size; /* rows * D * (w / 8) */
    uint32_t nseg;
    uint32_t w;                 /* 8 or 16 */
} spz_info;

/* Fill *p with the defaults: FIRE, seg_rows 1024, hdr_group 0, learn_shift 1,
 * entropy 0. */
void spz_params_default(spz_params *p);

/* Largest container sprintz_compress can write for this shape: every block
 * at full width plus headers, padding and the offset table. 0 if the
 * arguments are invalid. */
size_t sprintz_compress_bound(uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p);

/* Bytes of device workspace for the fastest compression of this shape. With
 * hdr_group 0 and D <= 16 that is the single-pass encoder's: every segment
 * is coded once into a slot of the workspace (its largest size) and then
 * copied to its place, plus 16 bytes per segment. Otherwise 8 bytes per
 * segment (two passes over the input). With entropy = 1 also the plain
 * container, its workspace and 256 bytes per segment for the code records. */
size_t sprintz_workspace_size(uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p);

/* Smallest workspace sprintz_compress accepts: 8 bytes per segment + 8 (the
 * two-pass encoder, which reads the input twice; the same bytes). Equal to
 * sprintz_workspace_size when entropy = 1. 0 if the arguments are invalid. */
size_t sprintz_workspace_size_min(uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p);

/* Compress d_src, a row-major (rows, D) array of `dtype` (alignment: the
 * element size), into the container d_dst (16-byte aligned, dst_cap >=
 * sprintz_compress_bound). The container's byte count is written to the
 * device word *d_out_size (required). d_ws (8-byte aligned, ws_size >=
 * sprintz_workspace_size_min) holds the segments' sizes (and with the
 * single-pass encoder their coded bytes) between the kernels; the
 * single-pass encoder runs when ws_size >= sprintz_workspace_size, d_ws and
 * d_src are 16-byte aligned and seg_rows * D * w/8 is a multiple of 16. The
 * container is the same either way.
 * Algorithm 1 (encodeBlock) per block, forecasters of Section 4.2, bit
 * packing of Section 4.3. */
spz_status sprintz_compress(const void *d_src, uint64_t rows, uint32_t D, spz_dtype dtype,
                            const spz_params *p, void *d_dst, size_t dst_cap, uint64_t *d_out_size,
                            void *d_ws, size_t ws_size, int32_t *d_status, hipStream_t stream);

/* The autotuner behind seg_rows = 0. It compresses the first min(rows, 2^20)
 * rows of d_src at the reference segment size (one segment over them, the
 * paper's unsegmented stream) and at each candidate 256, 512, 1024, 2048 and
 * 4096 below it, and times the decoding of each container (best of three,
 * HIP events). The reference only sets the bar: the choice is the fastest
 * decode among the candidates whose container stays within 1 % of the
 * reference's bytes; if none does, the candidate with the smallest container
 * (its loss is above 1 %); the reference itself only when there is no
 * candidate below it. Only the segment size is searched: waves per segment
 * and LDS tiles are fixed by the kernels. The result goes to *seg_rows_out
 * and to a host cache (mutex-protected, keyed by D, w, forecaster,
 * learn_shift, hdr_group, entropy and the power-of-two size class of the
 * reference size) that
 * sprintz_compress with seg_rows = 0 reads; a shape class that is not cached
 * yet is tuned on the first such call. Synchronous: it allocates scratch
 * device memory (hipMalloc), waits for `stream` and frees it again.
 * sprintz_compress_bound and sprintz_workspace_size with seg_rows = 0 hold
 * for every candidate. */
spz_status sprintz_autotune(const void *d_src, uint64_t rows, uint32_t D, spz_dtype dtype, const spz_params *p,
                            uint32_t *seg_rows_out, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * sprintz_compress without a workspace argument. The workspace is a static
 * device array of 4 MiB (4,194,304 bytes) inside the library, one per GPU, held until the process ends; its address
 * is looked up once per device on the first call there. The call allocates
 * nothing and otherwise behaves exactly as sprintz_compress (same kernels,
 * same bytes, same argument checks, except that seg_rows 0 is refused with
 * SPZ_EINVAL because the autotuner allocates); the single-pass encoder when its
 * workspace fits the array, else the two-pass one. Requests whose
 * sprintz_workspace_size_min exceeds the array (more than 524,287 segments,
 * or entropy = 1 beyond a small shape) return SPZ_ENOSPC before anything is
 * enqueued. All calls on
 * one GPU share its array: calls that overlap in time on that GPU (on
 * different streams, or from different threads) race and must not be
 * issued; calls ordered on one stream are fine. */
spz_status sprintz_compress_noalloc(const void *d_src, uint64_t rows, uint32_t D, spz_dtype dtype,
                                    const spz_params *p, void *d_dst, size_t dst_cap, uint64_t *d_out_size,
                                    int32_t *d_status, hipStream_t stream);

/* Parse the 64-byte container header from a host copy of at least 64
 * bytes. SPZ_ECORRUPT if it is not a valid header. */
spz_status sprintz_get_info(const void *h_src, size_t n, spz_info *out);

/* Decompress the container d_src (16-byte aligned, src_size bytes, described
 * by *info from sprintz_get_info) into d_dst, a row-major (rows, D) array
 * (dst_cap >= info->decompressed_size, aligned to the element size).
 * Algorithm 2 (decodeBlock) per record. Corrupt segments set bit 1 in
 * *d_status; their output rows are then unspecified. */
spz_status sprintz_decompress(const void *d_src, size_t src_size, const spz_info *info, void *d_dst,
                              size_t dst_cap, int32_t *d_status, hipStream_t stream);

/* Entropy-coded containers (info->params.entropy = 1): bytes of device
 * workspace sprintz_decompress_ws needs -- a plain container whose segments
 * sit at a fixed stride (the largest plain segment of the shape). 0 for
 * plain containers. */
size_t sprintz_decompress_workspace_size(const spz_info *info);

/* sprintz_decompress with a caller workspace (16-byte aligned, ws_size >=
 * sprintz_decompress_workspace_size; ignored for plain containers). Each
 * segment is Huffman-decoded into the workspace (the inverse of Section 4.4,
 * Entropy Coding), then decoded as by sprintz_decompress. A corrupt coded segment
 * sets bit 2 of *d_status. sprintz_decompress on an entropy-coded container
 * does the same with a stream-ordered allocation (hipMallocAsync /
 * hipFreeAsync) of the workspace. Batched plans take entropy-coded
 * containers too (their plain containers live in the plan's workspace). */
spz_status sprintz_decompress_ws(const void *d_src, size_t src_size, const spz_info *info, void *d_dst,
                                 size_t dst_cap, int32_t *d_status, void *d_ws, size_t ws_size, hipStream_t stream);

/* ---- Batched decompression ------------------------------------------------
 *
 * Decodes many containers (streams) in one go. The segments of all streams
 * become one work list per class (w, forecaster, D); for each class one
 * persistent grid of workgroups pulls groups of segments from a device queue,
 * so thousands of small and large streams fill the GPU together instead of
 * one launch each (the paper's method is unchanged: every segment is decoded
 * exactly as by sprintz_decompress, Algorithm 2 per record).
 *
 * Streams outside the batched kernels (hdr_group != 0, D > 16, output not
 * 16-byte aligned, seg_rows * D * w/8 not a multiple of 16) are decoded by
 * the single-container path inside the same call. Entropy-coded containers
 * (params.entropy = 1, Section 4.4) are first Huffman-decoded, all their
 * segments in one launch, into plain containers in the plan's workspace
 * (sprintz_decompress_workspace_size bytes each, rounded up to 256), which
 * then take the same batched or single-container path. */
typedef struct {
    const void *d_src;   /* container, 16-byte aligned, src_size bytes */
    size_t src_size;
    void *d_dst;         /* output rows (rows, D); dst_cap bytes */
    size_t dst_cap;
} spz_batch_item;

/* Opaque plan: device copies of the stream descriptors and work lists. */
typedef struct spz_batch spz_batch;

/* Validate n items (infos[i] from sprintz_get_info of item i) and build a
 * plan. Allocates device memory (hipMalloc) and copies the work lists to it
 * synchronously; returns the first item's error (SPZ_EINVAL, SPZ_ENOSPC,
 * SPZ_EUNSUPPORTED) if any item is invalid, SPZ_ENOMEM / SPZ_EHIP on
 * allocation or copy failure. The plan keeps the item pointers; the caller
 * keeps the buffers alive and unchanged in size while the plan is used. */
spz_status sprintz_batch_create(const spz_batch_item *items, const spz_info *infos, uint32_t n, spz_batch **out);

/* Device bytes of the plan for these items: the plain containers of
 * entropy-coded items, then the tables (0 if an item is invalid). */
size_t sprintz_batch_workspace_size(const spz_batch_item *items, const spz_info *infos, uint32_t n);

/* As sprintz_batch_create, but the tables go to the caller's device workspace
 * d_ws (16-byte aligned, ws_size >= sprintz_batch_workspace_size) with an
 * asynchronous copy on `stream`, so that plans can be made while other work
 * runs (the serving loop does this). Allocates no device memory; the plan
 * keeps the host copy of the tables until sprintz_batch_destroy, which the
 * caller calls once that copy and every use of the plan have completed.
 * SPZ_ENOSPC if ws_size is too small. */
spz_status sprintz_batch_create_in(const spz_batch_item *items, const spz_info *infos, uint32_t n, void *d_ws,
                                   size_t ws_size, hipStream_t stream, spz_batch **out);

/* Enqueue the decoding of every item of the plan on `stream`: a tiny kernel
 * resets the per-class queues, then one launch per nonempty class, then the
 * fallback streams. The class launches run concurrently on up to four
 * streams: `stream` and three side streams of the device that the library
 * creates once (default priority) and keeps, forked from `stream` and joined
 * back into it with the plan's events, so all work stays ordered after
 * earlier work on `stream` and before later work on it, also under graph
 * capture. d_status: n int32 device words (zero on entry, or NULL); corrupt
 * data in item i sets bit 1 of d_status[i]. Allocates nothing and never
 * synchronizes, so the call can be captured into a HIP graph. Calls that
 * overlap on one plan race on its queues and events. */
spz_status sprintz_batch_decompress(const spz_batch *b, int32_t *d_status, hipStream_t stream);

/* Free a plan (NULL is ignored). The caller makes sure no enqueued work uses it. */
void sprintz_batch_destroy(spz_batch *b);

/* ---- Batched compression --------------------------------------------------
 *
 * Compresses many series in one go. Series with hdr_group 0, D <= 16, entropy
 * 0, 16-byte aligned input, seg_rows * D * w/8 a multiple of 16 and a
 * workspace of at least sprintz_workspace_size bytes are coded
 * by the single-pass encoder in one persistent grid per class (w,
 * forecaster, D) that pulls groups of a series' segments from a device queue
 * (every segment exactly as by sprintz_compress: Algorithm 1 per block), then
 * one offset scan per series and one compaction launch over all of them; the
 * other series are compressed one call each inside the same batch call. */
typedef struct {
    const void *d_src;     /* (rows, D) row-major input, aligned to the element size */
    uint64_t rows;
    uint32_t D;
    uint32_t dtype;        /* spz_dtype */
    spz_params params;     /* seg_rows must be set (0 is refused: tune first with sprintz_autotune) */
    void *d_dst;           /* container, 16-byte aligned */
    size_t dst_cap;        /* >= sprintz_compress_bound */
    uint64_t *d_out_size;  /* device word: container bytes, 8-byte aligned */
    void *d_ws;            /* the series' workspace, 16-byte aligned; the batched encoder takes it when */
    size_t ws_size;        /* ws_size >= sprintz_workspace_size, else the series takes one call (>= the minimum) */
} spz_compress_item;

/* Opaque plan of a compression batch. */
typedef struct spz_cbatch spz_cbatch;

/* Device bytes of a batch's plan tables (0 if an item is invalid); every
 * series brings its own workspace in its item. */
size_t sprintz_compress_batch_workspace_size(const spz_compress_item *items, uint32_t n);

/* Validate n items and build a plan in the caller's workspace d_ws
 * (256-byte aligned, ws_size >= sprintz_compress_batch_workspace_size): the
 * tables go up with an asynchronous copy on `stream`; no device memory is
 * allocated. The first invalid item's status is returned (SPZ_EINVAL,
 * SPZ_ENOSPC, SPZ_EUNSUPPORTED). The plan keeps the item pointers and its
 * host copy of the tables until sprintz_compress_batch_destroy. */
spz_status sprintz_compress_batch_create_in(const spz_compress_item *items, uint32_t n, void *d_ws, size_t ws_size,
                                            hipStream_t stream, spz_cbatch **out);

/* Enqueue the compression of every item on `stream`. The class launches of
 * the batched encoder run concurrently on `stream` and the device's side
 * streams, joined back into `stream` before the offset scan (as for
 * sprintz_batch_decompress). d_status: n int32 device words (zero on entry,
 * or NULL); a size problem of item i sets bit 2 of d_status[i]. Allocates
 * nothing and never synchronizes, so the call can be captured into a HIP
 * graph. Calls that overlap on one plan race on its queues, events and
 * workspace. */
spz_status sprintz_compress_batch(const spz_cbatch *b, int32_t *d_status, hipStream_t stream);

/* Free a plan (NULL is ignored); its device tables are the caller's memory. */
void sprintz_compress_batch_destroy(spz_cbatch *b);

/* Static description of a status code. */
const char *sprintz_strerror(spz_status s);

/* Container format version this library writes and reads (1). */
int sprintz_format_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPRINTZ_H_ */
