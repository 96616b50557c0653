/*
 * mont.h -- C ABI of a gfx950 (MI355X) library for batched Montgomery-type
 * modular reduction, multiplication and exponentiation over arrays of
 * residues.
 *
 * The operations follow Xu, Jia and Yang, "Chinese Remainder Theorem
 * Approach to Montgomery-Type Algorithms" (arXiv 2402.00675):
 *
 *   MONT_CLASSIC              Montgomery's REDC (Section 1): T R^{-1} mod N,
 *                             R = 2^w, for 0 <= T < R N; result in [0, N).
 *   MONT_SIGNED               signed Montgomery (Section 3.1, Algorithm 1),
 *                             R = 2^w, odd N with 2N < R, |T| < N R / 2;
 *                             result r = T R^{-1} (mod N), -N < r < N, the
 *                             unique such r with T/R - N/2 < r <= T/R + N/2
 *                             (quotient digit N^{-1} a0 mods R taken in
 *                             [-R/2, R/2), Section 2).
 *   MONT_PLANTARD             Plantard (Section 3.2, Algorithm 2), R = 2^(2w),
 *                             N < 2^w / phi, 0 <= T <= N^2;
 *                             result -T R^{-1} mod N in [0, N).
 *   MONT_SIGNED_PLANTARD      signed Plantard (Section 3.2, Algorithm 3),
 *                             R = 2^(2w), N < 2^(w-1), |T| <= 2^(2w-2);
 *                             result -T R^{-1} mods N in [-(N-1)/2, (N-1)/2].
 *   MONT_SIGNED_PLANTARD_ALPHA
 *                             Huang's signed Plantard (Section 3.3,
 *                             Algorithm 4) with the context's alpha >= 1,
 *                             R = 2^(2w), N < 2^(w-alpha-1),
 *                             |T| <= 2^(2 alpha) N^2; same result as
 *                             MONT_SIGNED_PLANTARD.  alpha = 0 is refused:
 *                             the paper's Example 3.1 shows it is wrong.
 *
 * Word sizes w = 16, 32, 64.  Element types:
 *   w = 16: residues uint16_t / int16_t (signed variants), T uint32_t / int32_t
 *   w = 32: residues uint32_t / int32_t,                   T uint64_t / int64_t
 *   w = 64: residues uint64_t / int64_t,                   T 128-bit: (lo, hi)
 *           pairs of uint64_t, little-endian, two's complement when signed.
 * Signed variants read and write the signed types; the others the unsigned.
 *
 * Memory and streams.  Every array argument is a DEVICE pointer that the
 * caller owns (for example a torch tensor's storage); the library never
 * allocates or frees caller buffers.  `stream` is a hipStream_t (NULL = the
 * legacy default stream).  Calls enqueue work on that stream and return
 * without waiting; results are ready once the stream is synchronised.
 * In-place operation (out == an input of the same width) is allowed; other
 * overlaps are not.  n == 0 returns MONT_OK and launches nothing.
 * Alignment: elements must be naturally aligned.  mont_mul, mont_mul_const,
 * mont_redc and mont_mul_rns stream 16-byte chunks when every pointer is
 * 16-byte aligned, or when all of them become so after the same first h
 * elements (slices of aligned arrays at one offset): the 16-byte body then
 * starts at element h (on a 128-byte line when every pointer allows it) and
 * the same launch computes the h elements before it.  Other pointers take
 * an element-wise path with the same results.
 *
 * Errors.  Argument and domain errors are found on the host before any
 * launch and returned synchronously; nothing is enqueued then.  A HIP
 * error while launching returns MONT_E_DEVICE; the message is available
 * from mont_last_error() (thread-local).  Nothing aborts or throws across
 * this interface.  Residues outside a variant's input range are a
 * precondition violation: the output is then unspecified (but the kernels
 * stay in bounds and terminate).
 *
 * Contexts are plain values: immutable after mont_setup, safe to share
 * across threads and streams, and copied by value into kernel arguments.
 *
 * Environment (read at each use):
 *   MONT_LOG         diagnostics on stderr: unset or 0 silent; 1 or "error":
 *                    the message of every error a call returns; 2 or "info":
 *                    also tuning decisions, hipGraph rebuilds and serving
 *                    events (deadline expiries, retired slots, cancellation
 *                    requests); 3 or "debug": also one line per batch run.
 *   MONT_TUNE        unset: MONT_BATCH_TUNE and mont_tune_mul behave as
 *                    documented; 0: never tune (the flag is ignored and
 *                    mont_tune_mul keeps the current shape); 1: every batch
 *                    whose shape was not fixed by mont_batch_set_shape is
 *                    tuned on its first run, flag or not.
 *   MONT_TUNE_CACHE  JSON-lines file of tuned shapes (see mont_tune_mul).
 *   MONT_LIBRARY     (Python binding only) path of the library to load.
 */
#ifndef MONT_H
#define MONT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mont_status_t;
#define MONT_OK 0
#define MONT_E_INVAL (-1)       /* null pointer, even N, N < 3, N >= 2^w, bad w, bad enum */
#define MONT_E_DOMAIN (-2)      /* the variant's precondition on N (or alpha) fails */
#define MONT_E_UNSUPPORTED (-3) /* combination not provided (see each call) */
#define MONT_E_NOMEM (-4)       /* library-owned device/host memory could not be allocated */
#define MONT_E_DEVICE (-5)      /* HIP runtime error; see mont_last_error() */
#define MONT_E_BUSY (-6)        /* resource held by another call (serving loop) */
#define MONT_E_CANCELED (-7)    /* serving job cancelled before its launch */

typedef enum {
    MONT_CLASSIC = 0,
    MONT_SIGNED = 1,
    MONT_PLANTARD = 2,
    MONT_SIGNED_PLANTARD = 3,
    MONT_SIGNED_PLANTARD_ALPHA = 4
} mont_variant_t;

/*
 * Per-modulus constants (Section 1 and Section 3).  Filled by mont_setup;
 * callers treat it as opaque but may copy it freely (64 bytes).
 */
typedef struct mont_ctx {
    uint64_t N;        /* odd modulus, 3 <= N < 2^w */
    uint32_t w;        /* word size: 16, 32 or 64 */
    uint32_t valid;    /* bit v set iff variant v's precondition on N holds */
    uint64_t nprime;   /* N' = 2^w - (N^{-1} mod 2^w), REDC's multiplier (Section 1) */
    uint64_t ninv;     /* N^{-1} mod 2^w; read as w-bit two's complement it is
                          N^{-1} mods 2^w (Algorithm 1) */
    uint64_t ninv2_lo; /* N^{-1} mod 2^(2w), low 64 bits (Algorithms 2-4) */
    uint64_t ninv2_hi; /* N^{-1} mod 2^(2w), high 64 bits (w = 64 only, else 0) */
    uint64_t r_mod_n;  /* 2^w mod N  (Montgomery form of 1) */
    uint64_t r2_mod_n; /* 2^(2w) mod N (maps x to its Montgomery form x R mod N) */
    uint32_t alpha;    /* Algorithm 4 parameter (default 1 where valid, else 0) */
    uint32_t reserved;
} mont_ctx_t;

/*
 * mont_setup -- per-modulus constants for modulus N and word size
 * log2R = w in {16, 32, 64} (Section 1: N' = R - (N^{-1} mod R); Theorem 2.1
 * is checked on the result).  Host only, synchronous, no device use.
 * Classic and signed reduce modulo R = 2^w, the Plantard family modulo
 * 2^(2w).  Returns MONT_E_INVAL for an even N, N < 3, N >= 2^w or a bad w.
 * A variant whose precondition fails is cleared in ctx->valid (calls with it
 * return MONT_E_DOMAIN).
 */
mont_status_t mont_setup(uint64_t N, uint32_t log2R, mont_ctx_t *ctx);

/*
 * mont_set_alpha -- choose Algorithm 4's alpha (Section 3.3).  Requires
 * alpha >= 1 and N < 2^(w - alpha - 1); alpha = 0 returns MONT_E_DOMAIN.
 */
mont_status_t mont_set_alpha(mont_ctx_t *ctx, uint32_t alpha);

/*
 * mont_redc -- out[i] = REDC_variant(T[i]) for i < n (Section 1; Algorithms
 * 1-4).  T holds 2w-bit integers (see the element types above); out holds
 * w-bit residues.  The Require range of the variant applies to each T[i].
 */
mont_status_t mont_redc(const mont_ctx_t *ctx, const void *T, void *out, size_t n, mont_variant_t variant,
                        void *stream);

/*
 * mont_mul -- out[i] = REDC_variant(a[i] * b[i]) (the Montgomery product,
 * Section 1).  Unsigned variants take residues in [0, N); signed variants
 * take centred residues |a|, |b| <= (N - 1)/2 (any inputs whose product meets
 * the variant's Require range are valid).
 */
mont_status_t mont_mul(const mont_ctx_t *ctx, const void *a, const void *b, void *out, size_t n,
                       mont_variant_t variant, void *stream);

/*
 * mont_mul_const -- out[i] = REDC_variant(a[i] * b) for one fixed operand b
 * (a w-bit residue; two's complement for the signed variants), bit-identical
 * to mont_mul with b broadcast.  The quotient digit m = T N^{-1} is formed as
 * a (b N^{-1}) from a constant precomputed on the host, so the Plantard forms
 * never form the product a b: the saving Section 3.2 credits to Plantard's
 * algorithm (a 2w x w multiplication becomes w x w).  MONT_E_DOMAIN when b is
 * outside [0, N) (unsigned variants) or |b| >= N (signed variants).
 */
mont_status_t mont_mul_const(const mont_ctx_t *ctx, const void *a, uint64_t b, void *out, size_t n,
                             mont_variant_t variant, void *stream);

/*
 * mont_mul_rns -- the Montgomery product over k residue rows ("limbs"), row
 * j reduced with ctxs[j] (all of one word size w).  a, b, out are limb-major
 * [k][ld] arrays; the first n entries of each row are processed.
 * 1 <= k <= MONT_RNS_MAX, n <= ld.  ctxs is a HOST array.
 */
#define MONT_RNS_MAX 32
mont_status_t mont_mul_rns(const mont_ctx_t *ctxs, uint32_t k, const void *a, const void *b, void *out, size_t n,
                           size_t ld, mont_variant_t variant, void *stream);

/*
 * mont_crt -- integer reconstruction from residue rows: for pairwise coprime
 * odd moduli N_j = ctxs[j].N (64-bit word contexts, 1 <= k <= 16) and
 * residues x[j][i] in [0, N_j) (limb-major [k][ld], uint64), writes the
 * unique X_i in [0, N_0 ... N_{k-1}) with X_i = x[j][i] (mod N_j) as k
 * little-endian uint64 words at out[i*k .. i*k + k) (out 16-byte aligned).
 * The multi-modulus Chinese Remainder Theorem (Section 2 derives the two-
 * modulus case from Theorem 2.1), computed by Garner's mixed-radix
 * conversion: products by the constants N_j^{-1} mod N_i are Montgomery
 * products, or Shoup's precomputed-quotient products when every modulus is
 * below 2^62 and below twice every other one (below 2^61 with a quotient from
 * three partial products; results are identical).
 * ctxs is a HOST array.  MONT_E_DOMAIN if two moduli share a factor;
 * MONT_E_UNSUPPORTED for contexts that are not 64-bit; MONT_E_INVAL for k
 * outside [1, 16], n > ld, or a null or misaligned pointer.
 */
#define MONT_CRT_MAX 16
mont_status_t mont_crt(const mont_ctx_t *ctxs, uint32_t k, const void *res, size_t n, size_t ld, void *out,
                       void *stream);

/*
 * mont_ntt -- in-place number-theoretic transforms of `batch` polynomials of
 * n = 2^log2n residues in [0, N) (1 <= log2n <= 12), stored contiguously,
 * natural order in and out:
 *   forward  X_k = sum_j x_j root^(j k) mod N,
 *   inverse  x_j = n^{-1} sum_k X_k root^(-j k) mod N   (inverse != 0),
 * for a root with root^(n/2) = -1 (mod N) (else MONT_E_DOMAIN).  The
 * butterflies multiply by twiddles with the classic Montgomery product
 * (MONT_CLASSIC) or with Plantard's product by a fixed operand
 * (MONT_PLANTARD, Section 3.2); other variants return MONT_E_UNSUPPORTED.
 * Twiddle tables are built once per (N, root, n, variant, direction) and
 * kept in library-owned device memory for the life of the process.  The
 * coefficients are words of the context's width; with a 16-bit context,
 * transforms of length 16 or more whose 16-bit butterflies would need a
 * reduction between stages are computed with the 32-bit reductions of the
 * same modulus (16-bit words in and out, the same results).
 */
mont_status_t mont_ntt(const mont_ctx_t *ctx, void *data, size_t batch, uint32_t log2n, uint64_t root, int inverse,
                       mont_variant_t variant, void *stream);

/*
 * mont_pow -- out[i] = x[i]^e[i] mod N for residues x[i] in [0, N) and
 * unsigned 64-bit exponents e[i] (x^0 = 1, including 0^0).  Ordinary
 * residues in and out; inside, x is mapped to x R mod N with one REDC of
 * x (R^2 mod N), raised with Montgomery products (classic REDC, R = 2^w) and
 * mapped back with REDC (Section 1: the representation x -> x R mod N and
 * REDC's "pull back").  Valid for every odd N < 2^w.
 */
mont_status_t mont_pow(const mont_ctx_t *ctx, const void *x, const uint64_t *e, void *out, size_t n,
                       void *stream);

/*
 * mont_redc_range -- out[i] = REDC_variant(T0 + i) for i < n, with T
 * generated in the kernel (no input array): exhaustive sweeps of the input
 * space.  Unsigned variants (classic, Plantard) at w = 16 and 32; the last
 * input T0 + n - 1 must stay in the variant's Require range.
 */
mont_status_t mont_redc_range(const mont_ctx_t *ctx, uint64_t T0, void *out, size_t n, mont_variant_t variant,
                              void *stream);

/* --------------------------------------------------------------------------
 * Ragged batches: many independent vectors, each with its own modulus,
 * length and operation, processed by ONE persistent launch.  Elements of a
 * vector live in the caller's pool of its word size at offset `off`.
 */
#define MONT_OP_MUL 0  /* out = REDC_variant(in0 * in1) */
#define MONT_OP_REDC 1 /* out = REDC_variant(in0), in0 holds 2w-bit T */
#define MONT_OP_POW 2  /* out = in0 ^ in1 mod N, in1 the uint64 exponent pool; classic only */

typedef struct mont_seg {
    uint32_t ctx;     /* index into the batch's context table */
    uint16_t op;      /* MONT_OP_* */
    uint16_t variant; /* mont_variant_t */
    uint64_t n;       /* element count (0 allowed) */
    uint64_t off;     /* offset of the segment in in0 and out, in their element units */
    uint64_t off1;    /* offset in in1, in its element units (w-bit b, or uint64_t
                         exponents); for MONT_OP_MUL, (off1 - off) must be a multiple
                         of 128 / w so that both operands stay 16-byte aligned */
} mont_seg_t;

/*
 * Device pools, indexed by word-size class: [0] w = 16, [1] w = 32,
 * [2] w = 64.  in0 holds a (w-bit), x (w-bit) or T (2w-bit, for
 * MONT_OP_REDC); in1 holds b (w-bit) or exponents (uint64_t); out holds
 * w-bit results.  Pool pointers must be 16-byte aligned; unused entries may
 * be NULL.  The caller keeps the segments' byte ranges disjoint inside each
 * pool (a MONT_OP_REDC segment's T range is twice as wide as its out range).
 */
typedef struct mont_pools {
    const void *in0[3];
    const void *in1[3];
    void *out[3];
} mont_pools_t;

typedef struct mont_batch mont_batch_t;

/* batch flags */
#define MONT_BATCH_GRAPH 1u   /* replay the launch from a hipGraph */
#define MONT_BATCH_DYNAMIC 2u /* tiles taken from an atomic counter (else static round-robin) */
#define MONT_BATCH_TUNE 4u    /* autotune tile size and grid on the first run; the candidate
                                 runs read the caller's input pools and write library-owned
                                 output pools, so in-place batches stay exact */
#define MONT_BATCH_NONTEMPORAL 8u /* reported by mont_batch_info: the launch uses non-temporal
                                     loads and stores (chosen by the tuner; set by default) */

/*
 * mont_batch_create -- validates every segment (context valid for its
 * variant, op/variant pair supported), splits the segments into tiles, and
 * uploads the context, segment and tile tables to library-owned device
 * memory on `stream`.  ctxs and segs are HOST arrays, copied.  Returns
 * MONT_E_DOMAIN / MONT_E_INVAL / MONT_E_UNSUPPORTED with the offending
 * segment index in mont_last_error().
 */
mont_status_t mont_batch_create(const mont_ctx_t *ctxs, uint32_t nctx, const mont_seg_t *segs, uint32_t nseg,
                                uint32_t flags, mont_batch_t **out, void *stream);

/*
 * mont_batch_run -- performs every segment's operation in one launch (a
 * hipGraph replay with MONT_BATCH_GRAPH).  A batch is used by one stream at
 * a time; runs on one batch must not overlap.
 */
mont_status_t mont_batch_run(mont_batch_t *batch, const mont_pools_t *pools, void *stream);

/* Ragged forms of mont_mul / mont_redc / mont_pow: mont_batch_run for a
 * batch whose segments all have that op (else MONT_E_INVAL). */
mont_status_t mont_mul_ragged(mont_batch_t *batch, const mont_pools_t *pools, void *stream);
mont_status_t mont_redc_ragged(mont_batch_t *batch, const mont_pools_t *pools, void *stream);
mont_status_t mont_pow_ragged(mont_batch_t *batch, const mont_pools_t *pools, void *stream);

/*
 * mont_batch_run_pervector -- the same work as mont_batch_run, issued the
 * conventional way: one mont_mul / mont_redc / mont_pow launch per segment,
 * from a host loop.  A reference schedule for measuring what the persistent
 * launch saves.
 */
mont_status_t mont_batch_run_pervector(mont_batch_t *batch, const mont_pools_t *pools, void *stream);

/* Tiles and launch shape chosen for the batch (for reports). */
typedef struct mont_batch_info {
    uint64_t ntiles;
    uint64_t elements;
    uint32_t tile_elems; /* elements per tile for 32-bit mul/redc (others scale by bytes) */
    uint32_t grid;       /* workgroups of the launch */
    uint32_t block;
    uint32_t flags;      /* the batch's flags, plus MONT_BATCH_NONTEMPORAL when it applies */
    uint32_t blocks_per_cu; /* 0: one workgroup per tile; else the persistent grid is CUs x this */
    uint32_t pow_tile;   /* elements per exponentiation tile */
    uint32_t counters;   /* tile counters of a dynamic schedule (1 or 8), 0 when static */
} mont_batch_info_t;
mont_status_t mont_batch_info(const mont_batch_t *batch, mont_batch_info_t *info);

/*
 * mont_batch_set_shape -- fixes the launch shape of a batch, in place of (or
 * after) MONT_BATCH_TUNE, and rebuilds its tile table on `stream` (the call
 * waits for that upload):
 *   tile_elems     elements per tile of 32-bit products and reductions
 *                  (16-bit tiles hold twice as many, 64-bit tiles half), a
 *                  power of two in [256, 2^20];
 *   blocks_per_cu  0: one pass, one workgroup per tile; 1..64: a persistent
 *                  grid of (compute units x blocks_per_cu) workgroups, capped
 *                  at the tile count, each looping over tiles;
 *   dynamic        0: static round-robin over the tile table; 1: each
 *                  workgroup takes its next tile from one atomic counter; 8:
 *                  from one counter per XCD (tiles x, x+8, ... for XCD x),
 *                  moving on to the next XCD's counter once its own is used up
 *                  (one counter when the grid is not a multiple of 8).  The
 *                  kernel leaves the counters zeroed for the next run;
 *   nontemporal    1: non-temporal loads and stores;
 *   block          lanes per workgroup: 64 or 256 (0 = 256).
 * Results do not depend on the shape.  MONT_E_INVAL for values outside these
 * ranges; the batch must not be running (its earlier runs completed).
 */
typedef struct mont_batch_shape {
    uint32_t tile_elems;
    uint32_t blocks_per_cu;
    uint32_t dynamic;
    uint32_t nontemporal;
    uint32_t block;
} mont_batch_shape_t;
mont_status_t mont_batch_set_shape(mont_batch_t *batch, const mont_batch_shape_t *shape, void *stream);

/* Frees the batch's device tables and graph (after its runs completed). */
void mont_batch_destroy(mont_batch_t *batch);
/*
 * mont_batch_run_noalloc -- for callers that cannot allocate device memory
 * (code under stream capture that must not call hipMalloc, tight serving
 * loops, harnesses that forbid allocation): the work of mont_batch_create
 * followed by one mont_batch_run, with the same results, that allocates
 * nothing.  The batch's constant and tile tables go to a fixed device array
 * of MONT_NOALLOC_SCRATCH_BYTES that the library holds on each device it
 * runs on until the process ends; the launch is the one-pass shape (one
 * workgroup per tile of tile_elems 32-bit elements, 0 = 4096; a power of two
 * in [256, 2^20]), non-temporal.  ctxs, segs and pools are HOST structures
 * with the meaning of mont_batch_create and mont_batch_run; segments are
 * validated the same way, with the same errors.  Tables larger than the
 * array (64 bytes per context, 32 per segment and 32 per tile, 64 more)
 * return MONT_E_INVAL before any device use; a larger tile_elems or
 * mont_batch_create serves such batches.  The tables are copied to the
 * device on `stream` and the call waits for that copy (and so for the
 * stream's earlier work) before it returns; the kernel itself runs
 * asynchronously.  Every call on one device shares that device's array:
 * calls that overlap on one device (on other streams or from other threads)
 * race and must not be issued; calls in order on one stream are safe.
 */
#define MONT_NOALLOC_SCRATCH_BYTES (16u << 20)
mont_status_t mont_batch_run_noalloc(const mont_ctx_t *ctxs, uint32_t nctx, const mont_seg_t *segs, uint32_t nseg,
                                     const mont_pools_t *pools, uint32_t tile_elems, void *stream);


/* --------------------------------------------------------------------------
 * Launch-shape tuning for the streaming kernels.
 */
typedef struct mont_launch {
    uint32_t unroll;     /* 16-byte chunks per thread per iteration: 1, 2 or 4 */
    uint32_t nontemporal;/* 1: non-temporal loads/stores */
    uint32_t blocks_per_cu; /* 0: one pass over the data; else grid = CUs * this */
    uint32_t block;      /* lanes per workgroup of mont_mul / mont_redc's 16-byte path: 64
                            or 256 (default 64); exponentiation ignores it */
} mont_launch_t;

/*
 * mont_tune_mul -- times the candidate launch shapes of mont_mul (unroll x
 * non-temporal x grid) for this (w, variant) on n elements of the given
 * device buffers with HIP events, keeps the fastest for later calls in this
 * process, and appends it to the JSON-lines file named by $MONT_TUNE_CACHE
 * (if set).  A shape already recorded there (or, with no file named,
 * earlier in this process) for the same device architecture, library
 * version, w, variant and size class (floor(log2 n)) is applied without
 * timing; ragged batches under MONT_BATCH_TUNE use the same cache.  The candidates write a
 * library-owned buffer (MONT_E_NOMEM if it cannot be allocated): a and b are
 * only read, and out receives one mont_mul of the chosen shape, so
 * out == a or out == b is allowed.  *best (may be NULL) gets the shape.
 */
mont_status_t mont_tune_mul(const mont_ctx_t *ctx, const void *a, const void *b, void *out, size_t n,
                            mont_variant_t variant, mont_launch_t *best, void *stream);

/* Sets / reads the launch shape used for (op, w, variant). */
mont_status_t mont_set_launch(uint32_t op, uint32_t w, mont_variant_t variant, const mont_launch_t *l);
mont_status_t mont_get_launch(uint32_t op, uint32_t w, mont_variant_t variant, mont_launch_t *l);

/* --------------------------------------------------------------------------
 * Serving loop: a request loop with continuous batching.  Jobs (a vector
 * product or a vector exponentiation, classic REDC, each with its own odd
 * modulus) are queued as they arrive, admitted in FIFO order while their
 * operands and results fit a fixed device-memory budget, and fused into
 * ragged batches that run as one persistent launch each; up to `streams`
 * batches are in flight at once, so work that arrives while the device is
 * busy joins the next batch.  Per-modulus constants stay resident in a
 * device table that the batches' segment descriptors index: a modulus's
 * constants are computed and uploaded once, when it is first seen (or seen
 * again after its entry was reused for another modulus).  A service thread
 * does the admission, copies, launches and completion polling.
 *
 * A batch not finished deadline_us after its launch is given up: its jobs
 * complete with MONT_E_DEVICE, the stream is replaced by a new one, and the
 * batch's device memory stays reserved until the abandoned work is seen to
 * end (a stream that cannot be replaced leaves service; with none left,
 * every waiting job completes with MONT_E_DEVICE).
 */
typedef struct mont_server mont_server_t;

typedef struct mont_server_cfg {
    uint64_t hbm_budget_bytes; /* device memory for job operands and results, split
                                  evenly between 32-bit and 64-bit jobs (0: 8 GiB) */
    uint32_t max_jobs_in_flight; /* admitted, unfinished jobs (0: 4096) */
    uint32_t streams;            /* batches in flight, one HIP stream each (0: 3) */
    uint32_t max_batch_jobs;     /* jobs fused into one launch (0: 512) */
    uint32_t tile_elems;         /* 32-bit product tile in elements (0: 8192) */
    uint32_t deadline_us;        /* per-batch completion deadline, microseconds (0: 30 s) */
    uint32_t reserved;
} mont_server_cfg_t;

typedef struct mont_job {
    uint64_t id;     /* caller's id, echoed in the completion */
    uint64_t N;      /* odd modulus, 3 <= N < 2^w */
    uint32_t w;      /* 32 or 64 */
    uint32_t op;     /* MONT_OP_MUL (out = REDC(a b), classic) or MONT_OP_POW (out = x^e mod N) */
    uint64_t n;      /* elements */
    const void *in0; /* HOST: a or x, n w-bit residues in [0, N) */
    const void *in1; /* HOST: b (n w-bit residues) or e (n uint64_t exponents) */
    void *out;       /* HOST: n w-bit results.  All three stay valid until the job's
                        completion is returned; pinned memory gives asynchronous copies */
} mont_job_t;

typedef struct mont_completion {
    uint64_t id;
    int32_t status;  /* MONT_OK; MONT_E_DEVICE if the batch failed or missed its deadline;
                        MONT_E_CANCELED after mont_serve_cancel */
    uint32_t reserved;
    double t_submit; /* mont_serve_now() clock, seconds */
    double t_admit;  /* device memory reserved */
    double t_launch; /* batch enqueued */
    double t_done;   /* results copied to job.out and seen complete */
} mont_completion_t;

typedef struct mont_server_stats {
    uint64_t submitted, completed, rejected, launches, jobs_launched;
    uint64_t queued, staged, in_flight;
    uint64_t bytes_in_use, peak_bytes_in_use;
    uint64_t enqueue_ns; /* service-thread time spent enqueueing batches (copies, tables, launch) */
    uint64_t canceled;   /* jobs completed by mont_serve_cancel */
    uint64_t timed_out;  /* jobs of batches that missed the deadline */
    uint64_t quarantined_bytes; /* device memory of abandoned batches not yet seen to end */
    uint64_t dead_streams;      /* streams that could not be replaced */
    uint64_t ctx_uploads;       /* per-modulus constant entries uploaded to the resident table */
    uint64_t ctx_hits;          /* jobs whose modulus was already resident */
} mont_server_stats_t;

/* Allocates the device arena and starts the service thread on the current device. */
mont_status_t mont_serve_create(const mont_server_cfg_t *cfg, mont_server_t **out);
/* Queues one job.  MONT_E_INVAL for a malformed job, MONT_E_DOMAIN for one that
 * can never fit the budget (no completion is produced for either). */
mont_status_t mont_serve_submit(mont_server_t *s, const mont_job_t *job);
/* Declares [ptr, ptr + bytes) as pinned host memory mapped for the device
 * (allocated with hipHostMalloc; verified with hipPointerGetAttributes, never
 * registered here).  Jobs whose buffers lie in declared regions are staged by
 * two copy kernels per batch instead of DMA copies per job.  MONT_E_INVAL for
 * memory that is not such pinned memory, or that overlaps a declared region
 * without being inside it.  Regions stay declared for the server's life. */
mont_status_t mont_serve_host_region(mont_server_t *s, void *ptr, size_t bytes);
/* Submits jobs[i] when mont_serve_now() reaches t0 + arrival_s[i] (blocking;
 * arrival_s non-decreasing, t0 = the clock at the call).  Returns the number
 * accepted, or a negative status. */
int64_t mont_serve_submit_timed(mont_server_t *s, const mont_job_t *jobs, const double *arrival_s, uint64_t n);
/* Moves up to max completions into out, waiting up to wait_ms for the first;
 * returns the count (>= 0) or a negative status. */
int64_t mont_serve_poll(mont_server_t *s, mont_completion_t *out, uint32_t max, int32_t wait_ms);
/* Waits until every accepted job has completed (timeout_ms < 0: no limit);
 * MONT_E_BUSY on timeout. */
mont_status_t mont_serve_drain(mont_server_t *s, int32_t timeout_ms);
mont_status_t mont_serve_stats(const mont_server_t *s, mont_server_stats_t *st);
/* Cancels the job with this id if it has not been launched yet (still queued,
 * or admitted and waiting for a launch slot): it completes with
 * MONT_E_CANCELED, its device memory is released and its out buffer is not
 * written.  MONT_E_BUSY if it is in a launched batch (it completes normally),
 * MONT_E_INVAL if no job with this id is waiting.  Blocks until the service
 * thread has handled the request. */
mont_status_t mont_serve_cancel(mont_server_t *s, uint64_t id);
double mont_serve_now(void);
/* Stops the service thread after in-flight batches finish and frees the arena. */
void mont_serve_destroy(mont_server_t *s);

/* --------------------------------------------------------------------------
 * Measurement aid.
 */

/*
 * mont_stream_ref -- out = a XOR b over `bytes` bytes (a multiple of 16, all
 * three pointers 16-byte aligned device memory): the access pattern and
 * launch shape of mont_mul with no arithmetic, so its bandwidth is the
 * practical HBM ceiling for a 2-read/1-write stream.  Not part of the
 * paper's method.
 */
mont_status_t mont_stream_ref(const void *a, const void *b, void *out, size_t bytes, void *stream);

/*
 * mont_valu_ref -- issue-rate reference for one integer VALU instruction:
 * kind 0 v_mad_u64_u32, 1 v_mul_lo_u32, 2 v_mul_hi_u32, 3 v_mul_u32_u24,
 * 4 v_add_u32, 5 v_lshl_add_u64, 6 v_cndmask_b32, 7 v_cmp_le_u64,
 * 8 v_lshrrev_b64, 9 v_sub_u32, 10 v_min_u32, 11 v_mov_b32, 12 v_and_or_b32,
 * 13 v_add3_u32, 14 v_add_co_u32, 15 v_addc_co_u32, 16 v_or_b32, 17 v_and_b32,
 * 18 v_lshlrev_b32, 19 v_alignbit_b32, 20 v_cmp_ne_u32, 21 v_mad_i64_i32.
 * `blocks` workgroups of 256 lanes each run iters x 32 instances of it in
 * eight independent chains per lane and write one uint64_t per lane to `out`
 * (device memory, blocks * 256 entries).  A kind above 21 returns
 * MONT_E_INVAL.  Not part of the paper's method.
 */
mont_status_t mont_valu_ref(uint32_t kind, uint32_t iters, uint32_t blocks, void *out, void *stream);

/* --------------------------------------------------------------------------
 * Misc.
 */
const char *mont_last_error(void);
/* Library version (ABI revision in the low 16 bits). */
uint32_t mont_version(void);

/*
 * mont_debug_violations -- precondition counter of the MONT_DEBUG build
 * (libmont_debug.so, same interface).  That build checks, ahead of each
 * call's own kernels and on the same stream, every input element against the
 * range its algorithm is defined on (the Require lines of Algorithms 1-4;
 * 0 <= T < N R for classic REDC, Section 1): a product a b of mont_mul,
 * mont_mul_const and the ragged products, a T of mont_redc and the ragged
 * reductions; bases of mont_pow, coefficients of mont_ntt and residues of
 * mont_crt must lie below their modulus; serving jobs are checked on the
 * host at submission.  Results are unchanged (out-of-range elements still get
 * an unspecified value).  Synchronises the current device, stores the number
 * of violating elements counted since the last reset in *count (may be NULL),
 * and resets the count if `reset` is non-zero.  The release library returns
 * MONT_E_UNSUPPORTED and *count = 0.
 */
mont_status_t mont_debug_violations(uint64_t *count, int reset);

#ifdef __cplusplus
}
#endif

#endif /* MONT_H */
