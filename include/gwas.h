/*
 * libgwas: the GLS grid of multi-trait GWAS on one AMD MI355X (gfx950).
 *
 * For every SNP i and trait j the library computes the generalized
 * least-squares estimate of the paper's Section 2, Eq. (1),
 *
 *     b_ij = (X_i^T M_j^{-1} X_i)^{-1} X_i^T M_j^{-1} y_j,   X_i = [X_L | x_i],
 *
 * with the covariance of Eq. (2) without its scale factor,
 * M_j = h2_j Phi + (1 - h2_j) I (b is invariant to the scale sigma2_j of M_j).
 * It follows the paper's final algorithm (Section 3.2, Algorithm 5): Phi is
 * given through its eigendecomposition Phi = Z diag(w) Z^T (computed by the
 * caller in FP64), X_L, the SNPs and the traits are rotated once by Z^T, and
 * every (i, j) problem then costs O(p n) work plus a p x p SPD solve.
 *
 * Conventions for every call
 *   - n samples, p columns per design matrix (2 <= p <= 20, Section 3.3);
 *   - matrices are column-major: Z is n x n (eigenvector k is the contiguous
 *     column k), X_L is n x (p-1), a SNP block is n x mb (SNP-major: the n
 *     genotypes of one SNP are contiguous), a trait block is n x tb;
 *   - b is m x tb x p with p fastest: b[(i * tb + j) * p + q];
 *   - "stream" is a hipStream_t passed as void* (NULL: the null stream); the
 *     calls enqueue work and return; the caller synchronises that stream.
 *     Calls on one context must be issued from one thread on one stream;
 *   - the caller owns every buffer it passes; the library copies what it keeps
 *     and owns the resident cohort (Z, w, rotated X_L and SNPs) and its scratch;
 *     buffers handed to an enqueuing call (SNP blocks, Y, h2, b) must stay
 *     valid and unmodified until that stream has completed the call's work;
 *   - every call returns a gwas_status; on failure gwas_last_error() holds a
 *     message (thread-local) and nothing has been enqueued unless stated.
 */
#ifndef GWAS_H
#define GWAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gwas_status;
#define GWAS_OK 0
#define GWAS_EINVAL 1  /* bad argument: size, range, pointer, dtype, form */
#define GWAS_ENOMEM 2  /* device or pinned-host allocation failed        */
#define GWAS_EHIP 3    /* a HIP runtime call failed (message has the code) */
#define GWAS_EBUSY 4   /* serving: no free slot or memory, try again       */
#define GWAS_ESTATE 5  /* call not valid in the object's current state     */

/* element types of SNP blocks handed to gwas_rotate */
#define GWAS_DT_F64 0
#define GWAS_DT_F32 1
#define GWAS_DT_U8 2   /* genotype counts 0, 1, 2 (any byte value is taken as a number) */

/* precision forms of the O(m t p n) contractions (the Gram assembly and the
 * p x p solve are FP64 in every form) */
#define GWAS_FORM_F64 0    /* FP64 operands, FP64 MFMA accumulation; b in FP64          */
#define GWAS_FORM_F32 1    /* FP32 operands, FP32 MFMA accumulation added to FP64 sums
                              (gwas_options.f32_flush); b in FP32                       */
#define GWAS_FORM_BF16X3 2 /* split BF16 operands x = hi + lo, hi*hi + hi*lo + lo*hi,
                              FP32 MFMA accumulation; b in FP32                          */
#define GWAS_FORM_BF16X6 3 /* split BF16 in three pieces x = hi + mid + lo (the FP32 value
                              exactly), six products hi*hi + hi*mid + mid*hi + hi*lo +
                              lo*hi + mid*mid on the BF16 MFMAs, FP32 accumulation added
                              to FP64 sums every 32 samples; b in FP32                   */
#define GWAS_FORM_BIT(f) (1u << (f))

typedef struct gwas_ctx gwas_ctx;

typedef struct gwas_options {
    int64_t m_capacity;  /* SNPs the cohort holds (> 0)                                 */
    uint32_t forms;      /* OR of GWAS_FORM_BIT(): rotated SNP copies kept resident;
                            0 means FP64, FP32 and BF16X3                             */
    int32_t device;      /* HIP device ordinal; -1: the current device                 */
    int32_t max_traits;  /* traits handled per internal trait sub-block; 0: 1024       */
    int32_t slab_snps;   /* SNPs per D2H slab when b goes to the host; 0: 16384        */
    int32_t f32_flush;   /* FP32 form: 2 (default) adds the FP32 accumulators to FP64
                            sums: for b_B (the sum X_R^T D y, which cancels) four
                            chains of 8 samples each per 32 samples, for the others
                            every 64 samples; 0 never; other values are rejected
                            with GWAS_EINVAL                                       */
    int32_t timing;      /* nonzero: time every fused and rotation launch with HIP
                            events on its stream (read back by gwas_stats)           */
    int32_t ring_slots;  /* gwas_solve_stream: pinned host slots of the b ring; 0: 4  */
    int32_t host_threads;/* gwas_solve_stream: threads per slab checksum; 0: 8        */
    int32_t geno_chunk_snps; /* genotype (GWAS_DT_U8) rotation: SNPs per chunk repacked
                            on the device before the int8 kernels, a multiple of 256;
                            the context holds a buffer of this many rows of n rounded
                            up to 64 bytes; 0: the rows that fit 256 MiB (at least 256) */
    int32_t reserved[5];
} gwas_options;

typedef struct gwas_stats_t {
    int64_t non_spd;        /* problems whose S_ij was not numerically SPD (b = NaN)   */
    int64_t snps_rotated;   /* SNP columns rotated so far                              */
    int64_t problems;       /* (SNP, trait) problems solved so far                     */
    int64_t bytes_h2d;      /* bytes the library copied host -> device                 */
    int64_t bytes_d2h;      /* bytes the library copied device -> host                 */
    int64_t resident_bytes; /* device memory held by the context                       */
    int64_t fused_launches; /* timed launches of the fused kernel (timing option)        */
    double fused_ms;        /* their summed duration, ms                                 */
    int64_t rotate_launches;/* timed rotations: per device block of gwas_rotate (and per
                               streamed SNP block), the repack and int8 launches of
                               its chunks together                                     */
    double rotate_ms;       /* their summed duration, ms                                 */
    int64_t dot_launches;   /* launches of the dot-product kernel: FP64 and FP32 solve
                               calls with at most 3 traits (whose (p+1) x t x n_pad
                               panels fit 160 KB) use it instead of the MFMA tiles     */
    int64_t reserved[5];
} gwas_stats_t;

/* Fill *opt with defaults (m_capacity must still be set). */
void gwas_default_options(gwas_options *opt);

/*
 * Eigendecomposition of the kinship matrix on the device, for setup (the
 * eigendecomposition before the loops of Algorithm 5; Section 3.1):
 * Phi = Z diag(w) Z^T in FP64, by Householder tridiagonalisation and divide and
 * conquer (rocSOLVER dsyevd, loaded on the first call; not on the solve path).
 *   n          1 <= n <= 16384
 *   Phi        n x n symmetric FP64, column-major; only its lower triangle is read
 *   Z          out: n x n column-major, column k = unit eigenvector k (the layout
 *              gwas_setup takes)
 *   w          out: the n eigenvalues, ascending
 *   on_device  nonzero: Phi, Z and w are device memory of the current device;
 *              zero: host memory
 *   stream     HIP stream for the device work (NULL: the default stream)
 * Phi and Z may be the same buffer. Temporary device memory of about
 * 8 n^2 bytes is allocated and freed. Synchronous: returns once Z and w hold
 * the result.
 * Errors: GWAS_EINVAL (n out of range, NULL pointers), GWAS_ENOMEM, GWAS_EHIP
 * (runtime failure, solver library not found, or no convergence; the message
 * of gwas_last_error says which).
 */
gwas_status gwas_eigh(int32_t n, const double *Phi, double *Z, double *w, int32_t on_device, void *stream);

/*
 * Create a context: upload the eigendecomposition of the kinship matrix and
 * the covariates, rotate the covariates (Algorithm 5, preloop: X'_L = Z^T X_L,
 * in FP64), and allocate the resident rotated-SNP store for m_capacity SNPs in
 * each requested form.
 *   ctx   out: the new context (NULL on failure)
 *   n     samples, 1 <= n <= 16384
 *   p     design width, 2 <= p <= 20 (X_L has p-1 columns; put the intercept there)
 *   Z     host, n x n column-major, orthogonal eigenvectors of Phi
 *   w     host, n eigenvalues of Phi, finite (gwas_solve requires
 *         h2_j w_k + 1 - h2_j > 0 for every k, i.e. M_j SPD)
 *   X_L   host, n x (p-1) column-major
 *   opt   options (m_capacity required)
 * Errors: GWAS_EINVAL (sizes, NULL pointers, non-finite Z, w or X_L),
 * GWAS_ENOMEM, GWAS_EHIP. Synchronous.
 */
gwas_status gwas_setup(gwas_ctx **ctx, int32_t n, int32_t p, const double *Z, const double *w,
                       const double *X_L, const gwas_options *opt);

/*
 * Rotate SNPs [m0, m0 + mb) into the resident store: X'_R = Z^T X_R
 * (Algorithm 5, preloop); the result is kept in every resident form (FP64;
 * rounded to FP32; split to BF16 hi/lo and hi/mid/lo). FP64 and FP32 X_R: an
 * FP64 MFMA GEMM. Genotype bytes (GWAS_DT_U8): int8 MFMAs against Z in
 * fixed point sliced into int8 digits, with exact integer sums recombined in
 * FP64: six digits (47 bits per eigenvector, relative to its largest entry;
 * about 3e-14 of the row's maximum from the FP64 GEMM) when the context keeps
 * the FP64 form, else the leading four (about 4e-8 of the row's maximum, at
 * the FP32 rounding of the stored values). The genotype rows are repacked on
 * the device, geno_chunk_snps at a time, into the context's buffer in the
 * MFMA operand order; any row length, stride and alignment is accepted.
 *   X_R        n x mb, SNP-major, element type dtype (GWAS_DT_*)
 *   on_device  nonzero: X_R is device memory; zero: host memory (copied in
 *              bounded chunks through a device staging buffer)
 * Errors: GWAS_EINVAL (range beyond m_capacity, dtype, NULL), GWAS_EHIP.
 */
gwas_status gwas_rotate(gwas_ctx *ctx, int64_t m0, int64_t mb, const void *X_R, int32_t dtype,
                        int32_t on_device, void *stream);

/*
 * Solve the grid of SNPs [i0, i0 + mi) x the tb traits of Y (Algorithm 5,
 * loops): rotate the traits (y' = Z^T y, FP64), form the per-trait weights
 * d_jk = 1 / (h2_j w_k + 1 - h2_j) and the trait-only quantities in FP64
 * (S_TL_j, b_T_j and the Cholesky factor of S_TL_j), then, in one fused
 * kernel per trait sub-block, the p+1 contractions of length n per (i, j)
 * (S_BR, S_BL, b_B) in the chosen form and the FP64 p x p solve.
 *   tb          traits in the block (1 <= tb)
 *   Y           n x tb, column-major FP64 (device memory if y_on_device)
 *   h2          host, tb values in [0, 1); h2 = 1 is accepted when min w > 0
 *   form        GWAS_FORM_*; its SNP copy must be resident (gwas_options.forms)
 *   b           mi x tb x p, FP64 for GWAS_FORM_F64 else FP32; device memory if
 *               b_on_device, else host memory (pinned memory gives overlapped
 *               copies: b is produced in SNP slabs into two device buffers and
 *               copied out on a second stream while the next slab computes)
 * A problem whose Gram matrix S_ij is not numerically SPD (the SNP column is,
 * to the working precision, a combination of the covariates) gets b_ij = NaN
 * and is counted in gwas_stats_t.non_spd; when the covariates themselves are
 * dependent, so are all problems of every trait.
 * Errors: GWAS_EINVAL (range, tb, h2 out of range, form not resident),
 * GWAS_EHIP. The SNPs in range must have been rotated before.
 */
gwas_status gwas_solve(gwas_ctx *ctx, int64_t i0, int64_t mi, int32_t tb, const double *Y,
                       int32_t y_on_device, const double *h2, int32_t form, void *b,
                       int32_t b_on_device, void *stream);

/*
 * gwas_solve for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and the same b, bitwise, but every per-call device buffer (staged
 * and rotated traits, h2, trait panels, factors, tile counters) lives in a
 * fixed 32 MiB array of the library in device memory, one per device, held
 * until the process ends. The call allocates nothing, host or device.
 * Arguments as gwas_solve, except that b must be device memory (mi x tb x p,
 * FP64 for GWAS_FORM_F64 else FP32). The traits are processed in sub-blocks of
 * as many traits as the array holds (at most the context's max_traits):
 * about 56 KB per trait at n = 1000, p = 4, FP64 form. Every call on a device
 * shares that device's array and leaves its last contents there: calls that
 * overlap on one device (two host threads, or two streams not ordered by the
 * caller) race and give wrong results. Statistics count the call's problems
 * and non-SPD problems; its launches are not timed.
 * Errors: as gwas_solve; GWAS_EINVAL if b is not device memory, or if a single
 * trait's buffers exceed the array (not reachable for n <= 16384, p <= 20).
 */
gwas_status gwas_solve_noalloc(gwas_ctx *ctx, int64_t i0, int64_t mi, int32_t tb, const double *Y,
                               int32_t y_on_device, const double *h2, int32_t form, void *b, void *stream);

/*
 * Streamed solve (the b sink of the paper's double-buffering scheme, Section 4,
 * applied to the device->host link): the grid of SNPs [i0, i0 + mi) x the tb
 * traits of Y is solved as in gwas_solve, in slabs of gwas_options.slab_snps
 * SNPs per trait sub-block. Each slab's b is computed into one of two device
 * buffers while the previous one is copied, on a second stream, into a slot
 * of a library-owned ring of pinned host memory (gwas_options.ring_slots
 * slots). The calling thread then waits for the copy, computes the slab's
 * checksum and, when fn is not NULL, calls fn(user, slab); the slot is reused
 * once fn returns, so a slow consumer throttles the producer. The call returns
 * when every slab has been consumed (synchronous).
 *   checksums   nullable; receives the slab checksums in issue order (up to
 *               max_checksums of them); *n_slabs receives the slab count
 * The checksum of a slab is the sum over its 32-bit words w_k (k from 0, in
 * memory order) of (k + 1) * w_k, modulo 2^64.
 * Errors: as gwas_solve; GWAS_ENOMEM if the pinned ring cannot be allocated.
 */
typedef struct gwas_slab {
    int64_t index;      /* slab number in issue order                              */
    int64_t i0, count;  /* SNP range of the slab                                   */
    int32_t j0, tb;     /* trait range (within the call's traits)                   */
    int32_t p, form;
    const void *b;      /* pinned host memory: count x tb x p, p fastest            */
    int64_t bytes;
    uint64_t checksum;
} gwas_slab;
typedef void (*gwas_slab_fn)(void *user, const gwas_slab *slab);

gwas_status gwas_solve_stream(gwas_ctx *ctx, int64_t i0, int64_t mi, int32_t tb, const double *Y,
                              int32_t y_on_device, const double *h2, int32_t form, gwas_slab_fn fn,
                              void *user, uint64_t *checksums, int64_t max_checksums, int64_t *n_slabs,
                              void *stream);

/*
 * Genotype stream: solve the grid of m SNPs that are not resident, held in host
 * (or device) memory as X_R, n x m SNP-major of element type dtype, against the
 * tb traits of Y. The SNPs pass through the context's rotated store in blocks
 * of m_capacity / 2: block k is copied to the device and rotated by Z^T
 * (Algorithm 5, preloop) into store half k % 2 on the library's own stream
 * while block k - 1 is solved from the other half on `stream`, and b leaves
 * slab by slab through the pinned ring exactly as in gwas_solve_stream (slab
 * i0 is the SNP's index in X_R). This is the paper's streaming of the SNP
 * matrix through memory (Section 4), with HBM as the buffer and the host as
 * the backing store; m is unbounded by m_capacity. Overwrites the resident
 * store. X_R is read by hipMemcpyAsync (any memory kind); pinned host memory
 * lets the copies overlap the kernels. Same outputs as rotating all m SNPs and calling
 * gwas_solve_stream (bitwise). Errors: those of gwas_solve_stream, and
 * GWAS_EINVAL for m < 0, an unknown dtype or m_capacity < 2; GWAS_ENOMEM for
 * the two block staging buffers (2 x m_capacity / 2 x n x element size).
 */
gwas_status gwas_solve_snp_stream(gwas_ctx *ctx, const void *X_R, int32_t dtype, int64_t m, int32_t tb,
                                  const double *Y, int32_t y_on_device, const double *h2, int32_t form,
                                  gwas_slab_fn fn, void *user, uint64_t *checksums, int64_t max_checksums,
                                  int64_t *n_slabs, void *stream);

/* The checksum used by gwas_solve_stream, over bytes (a multiple of 4) at p. */
uint64_t gwas_checksum(const void *p, int64_t bytes);

/*
 * Copy rotated SNP columns [i0, i0 + mi) out of the resident store, n values
 * each (FP64 for GWAS_FORM_F64, FP32 for GWAS_FORM_F32), into dst (device
 * memory if dst_on_device, else host; synchronous on stream for host).
 * For inspection and tests. Errors: GWAS_EINVAL, GWAS_EHIP.
 */
gwas_status gwas_copy_rotated(gwas_ctx *ctx, int64_t i0, int64_t mi, int32_t form, void *dst,
                              int32_t dst_on_device, void *stream);

/*
 * Copy an internal buffer of the most recent gwas_solve (or of the cohort) to
 * host memory, for inspection and tests (synchronises the device):
 *   GWAS_DBG_XL      rotated covariates X'_L: (p-1) x n_pad FP64 (n_pad = n
 *                    rounded up to 64, zeros beyond n)
 *   GWAS_DBG_YT      rotated traits y' of the last trait sub-block: tcap x n_pad FP64
 *   GWAS_DBG_FAC     per-trait factors of the last sub-block: tcap x S FP64 with
 *                    S = even(q(q+1)/2 + q), q = p-1: packed L_j^{-1} (row-major
 *                    lower), then z_j = L_j^{-1} b_T_j
 *   GWAS_DBG_PANELS  trait panels of the last sub-block in the form's layout:
 *                    per plane max_traits rounded up to 16 rows of n_pad values,
 *                    row-major (FP64, FP32) or, for the split-BF16 forms, in MFMA
 *                    fragment order (1 KB block (row / 16, k / 32) holds lane
 *                    L = (k mod 32) / 8 * 16 + row mod 16 at bytes 16 L .. 16 L + 15)
 * bytes must equal the buffer's size (gwas_debug_size reports it).
 */
#define GWAS_DBG_XL 0
#define GWAS_DBG_YT 1
#define GWAS_DBG_FAC 2
#define GWAS_DBG_PANELS 3
int64_t gwas_debug_size(gwas_ctx *ctx, int32_t what, int32_t form);
gwas_status gwas_debug_copy(gwas_ctx *ctx, int32_t what, int32_t form, void *dst, int64_t bytes);

/* Counters of the context (synchronises the device to read them). */
gwas_status gwas_stats(gwas_ctx *ctx, gwas_stats_t *out);

/* Zero the counters and the timing record of the context (synchronises). */
gwas_status gwas_reset_stats(gwas_ctx *ctx);

/* Release the context and all its device memory (synchronises first). */
void gwas_destroy(gwas_ctx *ctx);

/* Message of the last failure on this thread ("" if none). */
const char *gwas_last_error(void);

/*
 * Serving: continuous batching of trait-block requests over a resident cohort.
 *
 * A server owns a scheduler thread and a consumer thread. Submitted requests
 * wait in FIFO order until a slot is free and their device memory (rotated
 * traits, panels, factors, four b staging buffers) fits in the server's HBM
 * budget; they are then admitted, their traits rotated and prepared, and
 * their SNP range is cut into work items (slabs). Every scheduling round
 * takes each admitted request's slabs that can start (a free staging buffer
 * and, for ring output, a free ring slot) and runs all of them in one launch,
 * whatever their trait count and covariate count; a round is built when the
 * previous round's kernel has finished, so slabs that become ready meanwhile,
 * and requests that arrive meanwhile, join the next round. Each slab's b is copied to the host
 * on a second stream: into the request's own buffer when it gave one, else
 * through a ring of pinned host slots where a worker thread checksums it (the
 * checksum of gwas_solve_stream) and passes it to the request's callback, if
 * any (callbacks of one request may run concurrently, in any slab order).
 * A request's results do not depend on what else is in flight: every problem
 * is computed by the same tile code in the same order, alone or in a mix.
 * Requests use covariate-count prefixes of the cohort's covariates: a request
 * with p columns uses the intercept-first X_L columns 0 .. p-2.
 */
typedef struct gwas_server gwas_server;

typedef struct gwas_server_options {
    int64_t hbm_budget;  /* device bytes admitted requests may hold at once; 0: 8 GiB      */
    int32_t max_slots;   /* requests in flight at once, 1..32; 0: 8                        */
    int32_t form;        /* GWAS_FORM_F64, _F32, _BF16X3 or _BF16X6, used for every request
                            (must be resident)                                            */
    int32_t item_problems; /* target problems (SNPs x traits) per work item; 0: 4194304    */
    int32_t max_traits;  /* largest request trait count accepted; 0: 1024                  */
    int32_t ring_slots;  /* pinned host ring slots; 0: 2 x max_slots                       */
    int32_t host_threads;/* checksum worker threads (one ring slab each at a time); 0: 8    */
    int32_t skip_checksum; /* nonzero: ring slabs are handed to the callback unchecksummed */
    int32_t grid_wgs;    /* persistent workgroups per launch; 0: as many as fit a compute unit
                            at once, at most two per unit (the copy kernels still get
                            their share)                                                  */
    int32_t reserved[4];
} gwas_server_options;

typedef struct gwas_server_stats_t {
    int64_t rounds;          /* grouped launches                                          */
    int64_t items;           /* work items (slabs) launched                               */
    int64_t ring_stalls;     /* items deferred because no pinned ring slot was free        */
    int64_t stage_stalls;    /* items deferred because the request's staging was busy      */
    int64_t bytes_d2h;       /* b bytes copied to the host                                 */
    double checksum_s;       /* summed checksum time of the workers                       */
    double busy_s;           /* wall time with at least one request admitted              */
    double issue_s;          /* host time the scheduler spent enqueueing launches and copies */
    double kernel_s;         /* device time of the grouped launches                        */
    int64_t reserved[6];
} gwas_server_stats_t;

typedef struct gwas_request {
    int32_t t;           /* traits, 1 .. max_traits                                       */
    int32_t p;           /* design width, 2 .. min(8, the cohort's p)                      */
    const double *Y;     /* host, n x t column-major (copied at submit)                    */
    const double *h2;    /* host, t values (copied at submit)                              */
    int64_t i0, m;       /* SNP range [i0, i0 + m); m = 0: all of [i0, m_capacity)        */
    void *b;             /* host output m x t x p (FP64 for the FP64 form, else FP32), kept
                            valid until the request completes; NULL: slabs go through the
                            pinned ring and the callback                                  */
    gwas_slab_fn fn;     /* called on the consumer thread for each ring slab; may be NULL  */
    void *user;
} gwas_request;

#define GWAS_REQ_QUEUED 0
#define GWAS_REQ_RUNNING 1
#define GWAS_REQ_DONE 2
#define GWAS_REQ_CANCELLED 3
#define GWAS_REQ_FAILED 4

typedef struct gwas_result {
    int32_t state;       /* GWAS_REQ_*                                                     */
    int32_t error;       /* gwas_status when FAILED                                       */
    double t_submit;     /* gwas_clock() at submit                                         */
    double t_admit;      /* when admitted (0 if never)                                     */
    double t_done;       /* when the last slab reached the host (0 if not done)            */
    int64_t problems;    /* m x t                                                         */
    int64_t slabs;       /* work items                                                    */
    uint64_t checksum;   /* sum of the ring slabs' checksums (0 with a caller buffer)      */
    int64_t reserved[4];
} gwas_result;

/* Seconds on the steady clock used for request timestamps. */
double gwas_clock(void);

/*
 * Create a server on a context whose cohort (rotated SNPs in opt->form) stays
 * resident. The context must outlive the server, and must not be used by
 * other calls while the server runs. Allocates the HBM budget as one arena and
 * the pinned ring up front. Errors: GWAS_EINVAL (form not resident, p of the
 * cohort above 8 is fine but requests are limited to p <= 8), GWAS_ENOMEM.
 */
gwas_status gwas_server_create(gwas_ctx *ctx, const gwas_server_options *opt, gwas_server **srv);

/* Queue a request (non-blocking); *ticket identifies it. Errors: GWAS_EINVAL
 * (t, p, range, h2, non-finite Y; or the request could never fit the budget). */
gwas_status gwas_server_submit(gwas_server *srv, const gwas_request *req, uint64_t *ticket);

/* State and timestamps of a request (non-blocking). GWAS_EINVAL for an unknown ticket. */
gwas_status gwas_server_poll(gwas_server *srv, uint64_t ticket, gwas_result *out);

/* Wait until the request is DONE, CANCELLED or FAILED, or timeout_s elapses
 * (timeout_s < 0: no limit); returns GWAS_EBUSY on timeout. */
gwas_status gwas_server_wait(gwas_server *srv, uint64_t ticket, double timeout_s, gwas_result *out);

/* Cancel a request: a queued one is dropped, a running one stops issuing
 * slabs and completes as CANCELLED once its slabs in flight have landed. */
gwas_status gwas_server_cancel(gwas_server *srv, uint64_t ticket);

/* Counters of the server (non-blocking). */
gwas_status gwas_server_stats(gwas_server *srv, gwas_server_stats_t *out);

/* Cancel what is queued, finish what is running, stop the threads, free. */
gwas_status gwas_server_destroy(gwas_server *srv);

/* Library version string. */
const char *gwas_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GWAS_H */
