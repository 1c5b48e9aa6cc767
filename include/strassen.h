/*
 * strassen.h -- C ABI of the Strassen-fused GEMM library for AMD MI355X (gfx950).
 *
 * Computes C := alpha * A * B + beta * C (Introduction, eq. "prime") with
 * zero, one or two levels of Strassen's seven-product scheme (Method section,
 * eq. "gpu_allops"; two levels as in the "Two-Level Strassen's Algorithm"
 * section).  Every product of the scheme is one instance of the general
 * primitive M = (sum of signed A blocks)(sum of signed B blocks); C_o += g_o M
 * (eq. "straprim1"): the operand sums are formed while tiles are staged into
 * LDS and the product is scattered with its signs into up to four C blocks in
 * the kernel epilogue (Strassen's Algorithm on NVIDIA GPUs section), so the
 * library needs no workspace and allocates no device memory.
 *
 * Layout: all matrices are row-major.  Element (i, j) of an r x c matrix X
 * with leading dimension ldX is X[i * ldX + j]; ldX >= max(1, c).
 *   A is m x k (lda), B is k x n (ldb), C is m x n (ldc).
 * A and B are read-only device pointers; C is an in/out device pointer.  The
 * caller owns every buffer.  A or B may not overlap C.
 *
 * Sizes that 2^levels does not divide are handled by virtual zero padding
 * inside the tiles ("Handling the Fringes" section): blocks that extend past
 * the matrix read zeros and write nothing.  Nothing outside the logical
 * matrices (the ld padding) is read or written.
 *
 * Asynchrony: calls enqueue kernels on a HIP stream and return; execution
 * errors surface at the caller's next synchronisation.  Results are
 * deterministic: the seven (or 49) products are launched in batches whose C
 * write sets are disjoint (Task Parallelism section, batching by variant), so
 * no atomics are used.
 *
 * Error convention (returned int):
 *    0              success
 *   -i              the i-th argument of the called function is invalid
 *                   (1-based, in that function's parameter order)
 *   > 0             a hipError_t reported by the HIP runtime (no device,
 *                   launch failure, ...), or STRASSEN_ERROR_SCRATCH_LIMIT
 * strassen_error_string() describes a code.  No C++ exception crosses the ABI.
 *
 * Degenerate cases (BLAS conventions; the paper fixes alpha = beta = 1):
 *   m == 0 or n == 0      nothing is done (returns 0).
 *   k == 0 or alpha == 0  C := beta * C; A and B are not read.
 *   beta == 0             C is write-only; NaN/Inf already in C do not
 *                         propagate.
 */
#ifndef STRASSEN_H
#define STRASSEN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage type of A and B.  C is always fp32 and products accumulate in
 * fp32 on the matrix cores.  For the 16-bit types the signed operand sums
 * are formed in fp32 from the stored values and rounded once (to nearest,
 * ties to even) to the operand type before the MFMA. */
typedef enum {
    STRASSEN_F32 = 0,
    STRASSEN_BF16 = 1,
    STRASSEN_F16 = 2
} strassen_dtype_t;

/* Arithmetic mode.
 *   PLAIN   products in the storage type (fp32 MFMA for fp32 operands).
 *   BF16X3  fp32 operands only: each fp32 operand sum x is split into
 *           hi = bf16(x) and lo = bf16(x - hi) and the product is
 *           hi*hi + hi*lo + lo*hi on bf16 MFMAs with fp32 accumulation. */
typedef enum {
    STRASSEN_MODE_PLAIN = 0,
    STRASSEN_MODE_BF16X3 = 1
} strassen_mode_t;

#define STRASSEN_MAX_LEVELS 2

/* C := alpha*A*B + beta*C, fp32 operands, `levels` in {0, 1, 2} (0 is the
 * plain blocked GEMM with the same kernels), enqueued on the calling
 * thread's stream (strassen_set_stream; the null stream by default).
 * Argument indices for errors: m=1 n=2 k=3 A=4 lda=5 B=6 ldb=7 C=8 ldc=9
 * alpha=10 beta=11 levels=12.  Overlap of A or B with C reports -8. */
int strassen_gemm(int64_t m, int64_t n, int64_t k,
                  const float *A, int64_t lda,
                  const float *B, int64_t ldb,
                  float *C, int64_t ldc,
                  float alpha, float beta, int levels);

/* Extended form.  a_type and b_type must be equal.  trans_a / trans_b = 1
 * reads op(A) = A^T (A stored k x m, lda >= m) / op(B) = B^T (B stored
 * n x k, ldb >= k); the product is then op(A)*op(B), m x n, and a block of
 * op(X) is the transpose of a block of X.  Transposed operands are available
 * for fp32 data (modes PLAIN and BF16X3); with bf16/fp16 data they report
 * -7 / -11.  hip_stream is a hipStream_t
 * (NULL = the null stream).
 * Argument indices: m=1 n=2 k=3 A=4 lda=5 a_type=6 trans_a=7 B=8 ldb=9
 * b_type=10 trans_b=11 C=12 ldc=13 alpha=14 beta=15 levels=16 mode=17
 * hip_stream=18.  Overlap of A or B with C reports -12. */
int strassen_gemm_ex(int64_t m, int64_t n, int64_t k,
                     const void *A, int64_t lda, strassen_dtype_t a_type, int trans_a,
                     const void *B, int64_t ldb, strassen_dtype_t b_type, int trans_b,
                     float *C, int64_t ldc,
                     float alpha, float beta, int levels,
                     strassen_mode_t mode, void *hip_stream);

/* Hybrid two-level Strassen (Two-Level Strassen's Algorithm section, the
 * hybrid variant): the top level forms each product's signed quadrant sums
 * P = sum +-A_q and Q = sum +-B_q into caller-provided workspace; the fused
 * one-level kernels then compute P*Q and scatter it, with signs, straight into
 * the sixteen C blocks of the two-level partition, so C needs no workspace and
 * each operand sum on the device side has at most two terms.  fp32, row-major,
 * same semantics and degenerate cases as strassen_gemm with levels = 2.
 * workspace: device memory of at least strassen_hybrid_workspace_size(m,n,k)
 * bytes, 16-byte aligned, not overlapping A, B or C; owned by the caller,
 * contents undefined after the call; it may be NULL when the product term is
 * absent (m, n or k = 0, or alpha = 0).  Calls that overlap on one workspace
 * race.  Enqueued on hip_stream (NULL = the null stream).
 * Argument indices: m=1 n=2 k=3 A=4 lda=5 B=6 ldb=7 C=8 ldc=9 alpha=10
 * beta=11 workspace=12 workspace_bytes=13; overlap of A or B with C -8. */
int strassen_gemm_hybrid(int64_t m, int64_t n, int64_t k,
                         const float *A, int64_t lda,
                         const float *B, int64_t ldb,
                         float *C, int64_t ldc,
                         float alpha, float beta,
                         void *workspace, int64_t workspace_bytes, void *hip_stream);

/* Workspace bytes strassen_gemm_hybrid needs for this shape:
 * 4 * ((2 sm)(2 sk) + (2 sk)(2 sn)) with sm = ceil(m/4) and sn, sk = ceil(n/4),
 * ceil(k/4) rounded up to a multiple of 4 (about (mk + kn)/4 floats).  Returns
 * the size, or a negative argument index (m=1 n=2 k=3).  Pure host
 * computation. */
int64_t strassen_hybrid_workspace_size(int64_t m, int64_t n, int64_t k);

/* One-level Strassen with the operand sums formed first (the Two-Level
 * Strassen's Algorithm section's hybrid idea applied at one level): every
 * two-term operand sum of eq. "gpu_allops" (five of A, five of B) is written
 * once into caller workspace by one streaming pass per operand that reads
 * each quadrant once; then each of the seven products runs the single-term
 * kernel on the formed sums or the quadrants themselves and scatters its
 * accumulator with signs into its C blocks, as in strassen_gemm_ex at
 * levels = 1, so C needs no workspace.  The sums are formed in the same
 * order and precision as the fused kernels form them (fp32 from the stored
 * values, 16-bit data rounded once) and the products accumulate in the same
 * order, so the result equals strassen_gemm_ex's one-level result bit for
 * bit, except on the 16-bit matrix cores with 256x256 tiles (C blocks of at
 * least 128 such tiles): there the single-output products M5 and M6 are
 * accumulated after M2 and M3 in the same workgroups and added into C3 and
 * C0 together with them (one read-modify-write of those blocks fewer each),
 * so those two blocks can differ from the fused result in the last bits.
 * Worth it where staging multi-term sums inside the product kernel is the
 * bottleneck (the BF16X3 mode).  In the BF16X3 mode the sums are stored
 * pre-split (per four consecutive elements the bf16 hi parts, then the bf16
 * lo parts, rounded as the kernels split a staged value), and so are A's two
 * single quadrants that products take as operands (A00 of M2, A11 of M3), so
 * every product stages A without splitting it, and B too where B is a sum;
 * the LDS contents, and so the results, are those of the fp32 sums.  A and B
 * as stored (no transposes);
 * a_type == b_type; modes and types as in strassen_gemm_ex; same degenerate
 * cases.
 * workspace: device memory of at least strassen_formed_workspace_size()
 * bytes, 16-byte aligned, overlapping none of A, B, C; owned by the caller,
 * contents undefined after the call; may be NULL when the product term is
 * absent (m, n or k = 0, or alpha = 0).  Calls that overlap on one workspace
 * race.  Enqueued on hip_stream (NULL = the null stream); where the chains
 * apply, B's sums are formed on a second stream of the calling thread
 * (created on first use per device, default priority, kept until the
 * thread ends) beside the products that read B as stored, ordered by
 * events, and hip_stream waits for that stream before the call returns, so
 * to the caller the call is ordered on hip_stream like any other.
 * Argument indices: m=1 n=2 k=3 A=4 lda=5 a_type=6 B=7 ldb=8 b_type=9 C=10
 * ldc=11 alpha=12 beta=13 mode=14 workspace=15 workspace_bytes=16
 * hip_stream=17.  Overlap of A or B with C reports -10. */
int strassen_gemm_formed(int64_t m, int64_t n, int64_t k,
                         const void *A, int64_t lda, strassen_dtype_t a_type,
                         const void *B, int64_t ldb, strassen_dtype_t b_type,
                         float *C, int64_t ldc,
                         float alpha, float beta, strassen_mode_t mode,
                         void *workspace, int64_t workspace_bytes, void *hip_stream);

/* Workspace bytes strassen_gemm_formed needs: e * (5 sm sk + 5 sk sn) with
 * the one-level block extents sm = ceil(m/2), sk = ceil(k/2), sn = ceil(n/2)
 * (sk and sn rounded up to the 16-byte vector width: 4 fp32 or 8 16-bit
 * elements) and e = 2 bytes for bf16/fp16 data, 4 for fp32 data in the
 * PLAIN mode; about 1.25 (mk + kn) e bytes.  BF16X3 mode: 4 * (7 sm sk +
 * 5 sk sn) (A's two single quadrants stored pre-split too).  Returns the
 * size, or a negative argument index (m=1 n=2 k=3 dtype=4 mode=5).  Pure
 * host computation. */
int64_t strassen_formed_workspace_size(int64_t m, int64_t n, int64_t k,
                                       strassen_dtype_t dtype, strassen_mode_t mode);

/* strassen_gemm_formed at zero, one or two levels (levels = 0, 1 or 2; eq.
 * "gpu_allops" applied twice, the Two-Level Strassen's Algorithm section's
 * 49 products).  Level 0 is the plain product (as strassen_gemm_ex at
 * levels = 0, bit for bit); in the BF16X3 mode A and B are first written
 * pre-split into workspace, so the product stages them without splitting
 * (the plain product with the same operand path as the formed Strassen
 * products); in the PLAIN mode nothing is formed and no workspace is
 * needed.  At two levels every multi-term operand of the 49 products
 * (25 four-term and 20 two-term sums of A, the same of B, on the 4 x 4 block
 * grid) is formed once into workspace, one launch per level-1 operand
 * reading its at most eight blocks once, with the fused kernels' arithmetic
 * (terms added in order, one fused multiply-add each, in fp32 from the
 * stored values, 16-bit data rounded once; in the BF16X3 mode stored
 * pre-split as at one level, together with the four single blocks of each
 * operand); then the 49 products run the
 * single-term kernel in the race-free batches and the launch order of
 * strassen_gemm_ex at levels = 2, so the result equals that call's bit for
 * bit.  The sum-forming launches run on the calling thread's second stream
 * (as for strassen_gemm_formed) in the order the batches first read them,
 * each batch waiting for its sums through an event, so forms overlap the
 * products of earlier batches; hip_stream waits for that stream before the
 * call returns.  At one level the same as strassen_gemm_formed.  Arguments as
 * strassen_gemm_formed with levels inserted: m=1 n=2 k=3 A=4 lda=5 a_type=6
 * B=7 ldb=8 b_type=9 C=10 ldc=11 alpha=12 beta=13 levels=14 mode=15
 * workspace=16 workspace_bytes=17 hip_stream=18. */
int strassen_gemm_formed_ex(int64_t m, int64_t n, int64_t k,
                            const void *A, int64_t lda, strassen_dtype_t a_type,
                            const void *B, int64_t ldb, strassen_dtype_t b_type,
                            float *C, int64_t ldc,
                            float alpha, float beta, int levels, strassen_mode_t mode,
                            void *workspace, int64_t workspace_bytes, void *hip_stream);

/* Workspace bytes strassen_gemm_formed_ex needs: at level 0 none (PLAIN
 * mode) or 4 (m sk + sk sn) with sk, sn = k, n rounded up to 4 (BF16X3);
 * at one level as strassen_formed_workspace_size; at two levels e * 45 (sm sk + sk sn) with
 * the two-level block extents sm = ceil(m/4), sk = ceil(k/4), sn = ceil(n/4)
 * (sk, sn rounded up as above), about 2.8 (mk + kn) e bytes; BF16X3 mode
 * 4 * 49 (sm sk + sk sn) (the four single blocks of each operand that
 * products take stored pre-split too).  Returns the
 * size, or a negative argument index (m=1 n=2 k=3 levels=4 dtype=5 mode=6).
 * Pure host computation. */
int64_t strassen_formed_workspace_size_ex(int64_t m, int64_t n, int64_t k, int levels,
                                          strassen_dtype_t dtype, strassen_mode_t mode);

/* strassen_gemm_formed without a workspace argument and without any
 * allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * operand sums go to a fixed scratch array of STRASSEN_NOALLOC_SCRATCH_BYTES
 * (256 MiB) that the library's code object holds on every GPU it runs on,
 * from module load until the process ends.  Same arguments, semantics and
 * results as strassen_gemm_formed (minus the workspace pair; argument
 * indices as there, hip_stream=15).  A call whose
 * strassen_formed_workspace_size exceeds the scratch returns
 * STRASSEN_ERROR_SCRATCH_LIMIT without launching anything (fp32 data up to
 * about m = n = k = 5180, 4730 in the BF16X3 mode, 16-bit data up to about
 * 7320).  All calls on one
 * GPU share that GPU's scratch: calls that overlap in time on one GPU (from
 * several streams or threads) race.  Nothing needs clearing between calls:
 * every scratch element a call reads was written earlier in that call.  The
 * scratch belongs to the device of hip_stream (the current device for the
 * null stream); its address is looked up on the first call per device. */
#define STRASSEN_NOALLOC_SCRATCH_BYTES ((int64_t)256 << 20)
#define STRASSEN_ERROR_SCRATCH_LIMIT 0x5c00
int strassen_gemm_formed_noalloc(int64_t m, int64_t n, int64_t k,
                                 const void *A, int64_t lda, strassen_dtype_t a_type,
                                 const void *B, int64_t ldb, strassen_dtype_t b_type,
                                 float *C, int64_t ldc,
                                 float alpha, float beta, strassen_mode_t mode,
                                 void *hip_stream);

/* Sets the stream strassen_gemm uses on the calling thread (a hipStream_t;
 * NULL = the null stream).  Always returns 0. */
int strassen_set_stream(void *hip_stream);

/* Workgroup tile of the product kernels.  AUTO (the default) picks per
 * launch: for fp32, 256x256 or 128x128 by the lower cost of the launch's waves
 * of workgroups (256 slots of 256x256, one per CU, against 512 of 128x128,
 * two per CU; per-wave costs fitted to MI355X measurements); for 16-bit
 * operands, 256x256 when every product of the launch has at least 128 such
 * tiles and the launch at least 256, else 128x128.  The others force one
 * shape for every launch (tuning, tests).  Applies to the calling thread's
 * later calls only (like the stream); returns 0 or -1 (bad value). */
#define STRASSEN_TILE_AUTO 0
#define STRASSEN_TILE_128 1
#define STRASSEN_TILE_256 2
int strassen_set_tile(int tile);

/* Schedule of the products of one call (Task Parallelism section).
 * BATCHED (the default): race-free batches of one variant, launched in a fixed
 *   order; every C element is updated by plain read-modify-writes, so results
 *   are deterministic (bitwise reproducible).
 * CONCURRENT: C := beta*C first, then the products are launched up to eight at
 *   a time whatever their variant, and outputs are added with fp32 atomics
 *   (element-wise atomic update).  Fewer, fuller launches for small problems;
 *   the order of the additions varies, so results vary in the last bits.
 *   Applies to fp32 operands as stored (mode PLAIN, no transposes) at levels
 *   >= 1; other calls keep the batched schedule.  The atomics are the
 *   hardware fp32 atomic add, which needs C in ordinary (coarse-grained)
 *   device memory: with C in fine-grained or host-coherent memory the
 *   concurrent schedule is not supported.
 * STREAMS (table "tab:gpu_streaming"): one-level calls only (strassen_gemm,
 *   strassen_gemm_ex; other calls keep the batched schedule): each product
 *   is one launch, on the call's stream or on a second stream of the calling
 *   thread (created on first use, default priority) as the table assigns it;
 *   products of one stage run at once on the two streams, and each stage
 *   waits for the previous one on both, so every C element is updated in a
 *   fixed order (deterministic; the order differs from BATCHED's, so the
 *   last bits can differ).  The call's stream waits for the second stream
 *   before the call returns.
 * Applies to the calling thread's later calls only; returns 0 or -1 (bad
 * value). */
#define STRASSEN_SCHEDULE_BATCHED 0
#define STRASSEN_SCHEDULE_CONCURRENT 1
#define STRASSEN_SCHEDULE_STREAMS 2
int strassen_set_schedule(int schedule);

/* Description of how a call of this shape is executed. */
typedef struct {
    int32_t levels;            /* 0, 1 or 2 */
    int32_t blocks_per_dim;    /* d = 2^levels */
    int64_t sub_m, sub_n, sub_k; /* extent of one block of the d x d partition
                                  * (ceil(dim/d), n and k rounded up to the
                                  * vector width for levels >= 1) */
    int32_t n_instances;       /* 7^levels products */
    int32_t n_launches;        /* race-free batches = kernel launches */
    int32_t tile_m, tile_n, tile_k; /* workgroup tile and k-tile depth of the
                                     * launch with the most operand terms,
                                     * for untransposed operands (both are
                                     * chosen per launch) */
    int32_t workgroups_per_instance;
    double executed_flops;     /* 7^L * 2 * sub_m * sub_n * sub_k */
    double classical_flops;    /* 2 * m * n * k */
} strassen_plan_info_t;

/* Fills *out for a call of this shape, dtype and mode.  Pure host
 * computation: needs no GPU.  Argument indices: m=1 n=2 k=3 levels=4
 * dtype=5 mode=6 out=7. */
int strassen_plan_info(int64_t m, int64_t n, int64_t k, int levels,
                       strassen_dtype_t dtype, strassen_mode_t mode,
                       strassen_plan_info_t *out);

/* One product of the plan.  Blocks are numbered row-major in the d x d
 * partition: block b covers block-row b / d and block-column b % d.  Signs
 * are +1 or -1.  c_first[o] = 1 marks the first update of C block c_block[o]
 * in launch order: that update applies beta (C := beta*C + g*alpha*M). */
typedef struct {
    int32_t launch;            /* index of the kernel launch (batch) */
    int32_t n_a, n_b, n_c;     /* W_A, W_B, W_C (Register Optimization section) */
    int32_t a_block[4], a_sign[4];
    int32_t b_block[4], b_sign[4];
    int32_t c_block[4], c_sign[4], c_first[4];
} strassen_instance_t;

/* Copies the plan's products, in launch order, into out[0 .. capacity-1]
 * and returns their number (7^levels), or a negative argument index
 * (levels=1 out=2 capacity=3).  Pure host computation: needs no GPU. */
int strassen_plan_instances(int levels, strassen_instance_t *out, int capacity);

/* Static description of an error code; never NULL. */
const char *strassen_error_string(int code);

/* Identifier of the sources the library was built from (hex sha256 over its
 * C++/HIP sources and this header, computed by the build script); the
 * Python binding refuses a library whose id differs from the sources beside
 * it.  Never NULL. */
const char *strassen_build_id(void);

/* ---- measurement support (Experiment section: kernels are timed with
 * device events) ----------------------------------------------------------
 * While recording is on, every kernel the library launches is bracketed by
 * two HIP events on its stream.  strassen_profile_stop() waits for those
 * events, copies at most `capacity` records into out (oldest first), turns
 * recording off and returns the number of records made (which may exceed
 * capacity), or a negative argument index (out=1 capacity=2), or a positive
 * hipError_t. */
typedef struct {
    char kernel[64];           /* kernel family and template variant */
    int32_t launch;            /* launch index within its call */
    int32_t batch;             /* products in this launch */
    int32_t workgroups;        /* total workgroups */
    float ms;                  /* device time between the two events */
    double flops;              /* executed MFMA flops of this launch */
} strassen_launch_record_t;

int strassen_profile_start(void);
int strassen_profile_stop(strassen_launch_record_t *out, int capacity);

/* The matrix cores' attainable rate, the ceiling the kernels' MFMA-busy
 * fractions are read against (Analysis section: the peak a kernel is
 * modelled against).  Enqueues one launch of `workgroups` workgroups of four
 * waves; every wave issues `iters` rounds of four independent MFMAs on
 * operands held in registers (op 0: 32x32x16 bf16, 1: 32x32x16 fp16,
 * 2: 32x32x2 fp32), with random values in [-0.5, 0.5) (random != 0) or a
 * constant 0.25, and no memory traffic but one float per thread written to
 * out (workgroups * 256 floats, device memory owned by the caller).  One
 * launch executes workgroups * 4 * iters * 4 MFMAs of 32768 (16-bit) or 4096
 * (fp32) flops each; time it with events on hip_stream.  Returns 0, a
 * negative argument index (op=1 random=2 iters=3 workgroups=4 out=5) or a
 * positive hipError_t. */
int strassen_probe_mfma(int op, int random, int64_t iters, int32_t workgroups, float *out, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* STRASSEN_H */
