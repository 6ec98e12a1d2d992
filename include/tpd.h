/*
 * tpd.h -- C ABI of libtpd, the MI355X (gfx950) implementation of the
 * Tensorized Pauli Decomposition (TPD) of Hantzko, Binkowski and Gupta,
 * "Tensorized Pauli decomposition algorithm", arXiv:2310.13421.
 *
 * The decomposition (section "Problem formulation", eq. (PauliDecomposition))
 * writes a complex 2^n x 2^n matrix A as
 *     A = sum_t w_t sigma^t,    w_t = 2^-n tr(sigma^t A),
 * over the 4^n Pauli strings sigma^t = sigma^{t_1} (x) ... (x) sigma^{t_n}
 * (eq. (PauliString)), letters I=0, X=1, Y=2, Z=3.  It is computed by n
 * slicing levels (section "Methods", eq. (CumulativeWeightsDefinition)):
 * the quadrants A11, A12, A21, A22 become the cumulative matrix weights
 * (A11+A22)/2, (A12+A21)/2, i(A12-A21)/2, (A11-A22)/2; zero blocks are
 * pruned (eq. (CumulativeWeightsFormula) and the remark after it).
 *
 * Data formats
 *   - Complex numbers are interleaved (re, im): TPD_C128 = two IEEE binary64
 *     (16 bytes), TPD_C64 = two IEEE binary32 (8 bytes).
 *   - A is row-major with leading dimension 2^n.
 *   - Real input (TPD_R64, TPD_R32): plain binary64 / binary32 entries, and
 *     real-coded coefficients (see TPD_R64 below).
 *   - Coefficients, canonical layout (default): 4^n values, the
 *     weight of string t_1..t_n at index q = sum_k t_k 4^(n-k), t_1 being the
 *     first (outermost) tensor factor.
 *   - Coefficients, matrix layout (TPD_FLAG_LAYOUT_MATRIX): the weight of t
 *     at row h, column l of a 2^n x 2^n array, where bit (n-k) of h is 1 iff
 *     t_k is Y or Z and bit (n-k) of l is 1 iff t_k is X or Z.  q and (h, l)
 *     are related by q = interleave(h, l) with the bits of h in the odd
 *     positions.
 *
 * Memory, ownership, aliasing
 *   - All matrix and coefficient pointers are DEVICE pointers owned by the
 *     caller, on the current HIP device.  Alignment: 16 bytes (C128) or 8
 *     bytes (C64, R64) or 4 bytes (R32); otherwise TPD_ERROR_INVALID_VALUE.
 *   - Out of place (coeffs != A, no overlap): A is read and not modified.
 *   - In place (coeffs == A): supported with TPD_FLAG_LAYOUT_MATRIX for every
 *     n, and in the canonical layout only for n <= 6.  Partial overlap is
 *     rejected with TPD_ERROR_INVALID_VALUE.
 *   - The library owns its workspace (pruning bitmaps, work tables); it is
 *     allocated on first use per (device, stream) and by plan creation, and
 *     released by tpd_release_workspace / tpd_plan_destroy.
 *
 * Execution and errors
 *   - Calls validate their arguments on the host, synchronously, before
 *     enqueueing anything; then they enqueue kernels on `stream` (a
 *     hipStream_t, NULL = the default stream) and return without waiting.
 *     Device-side faults surface at the caller's next synchronisation.
 *   - No C++ exception crosses this ABI.  Nothing is printed unless the
 *     environment variable TPD_LOG=1 is set.
 *   - Concurrent calls on different streams use different workspaces and do
 *     not interfere; calls on one stream are ordered by the stream.
 */
#ifndef TPD_H_
#define TPD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* tpd_stream_t; /* a hipStream_t; NULL = default stream */

typedef enum {
  TPD_C128 = 0, /* interleaved binary64 pairs */
  TPD_C64 = 1,  /* interleaved binary32 pairs */
  TPD_R64 = 2,  /* real input: binary64 entries, real-coded weights (below) */
  TPD_R32 = 3   /* real input: binary32 entries, real-coded weights (below) */
} tpd_dtype_t;

/* TPD_R64 / TPD_R32: A is a real 2^n x 2^n matrix of binary64 / binary32
 * (8 / 4 bytes per entry).  Each level of a real matrix yields values that
 * are real numbers times a power of i (only the Y output multiplies by i),
 * so the transform runs in real arithmetic, half the traffic of TPD_C128 /
 * TPD_C64.  The weight of a string with y Y letters is real for even y and
 * imaginary for odd y (sigma^t is real or imaginary as y is even or odd, and
 * w_t = 2^-n tr(sigma^t A)); coeffs holds 4^n values r_t of A's type with
 *     w_t = r_t (y even),    w_t = i r_t (y odd),
 * i.e. the weight's nonzero component, in the canonical or matrix layout.
 * Each r_t equals, up to the sign of zero, that component of the TPD_C128
 * (TPD_C64) result for the same matrix.  With TPD_FLAG_HERMITIAN (A real
 * symmetric; its odd-y weights vanish, as the footnote on real-symmetric
 * input in section "Existing algorithms" notes) the first sweep reads half
 * the input.  Every entry point takes them: tpd_decompose_partial returns
 * real-coded values (NaN for out-of-range requests), tpd_compact keeps
 * |r_t| > tol, tpd_synthesize_ex turns real-coded weights into the real
 * matrix, and the batched entry points decompose real matrices of mixed
 * sizes (2^13-element tiles for both real types).                        */

typedef enum {
  TPD_SUCCESS = 0,
  TPD_ERROR_INVALID_VALUE = 1, /* NULL/misaligned pointer, bad flags, overlap */
  TPD_ERROR_UNSUPPORTED = 2,   /* n out of range, unsupported layout/aliasing */
  TPD_ERROR_OUT_OF_MEMORY = 3, /* workspace allocation failed */
  TPD_ERROR_LAUNCH = 4,        /* a kernel launch or HIP call failed */
  TPD_ERROR_INTERNAL = 5,
  TPD_ERROR_NO_DEVICE = 6      /* no usable gfx950 device */
} tpd_status_t;

/* flags (bitwise OR) */
#define TPD_FLAG_NO_PRUNE 0x1u      /* disable the zero-block bitmap (it is on by default) */
#define TPD_FLAG_LAYOUT_MATRIX 0x2u /* coefficients in the matrix layout (see above) */
#define TPD_FLAG_TIMING 0x4u        /* plans only: record per-kernel HIP events */
#define TPD_FLAG_ORDER_BOTTOM 0x8u  /* register phases bottom level first (tuning) */
#define TPD_FLAG_HERMITIAN 0x10u    /* caller promises A = A^H (see below) */
#define TPD_FLAG_ROTATE_TILES 0x20u /* second sweep: row blocks rotate every 8 tile columns (tuning) */
#define TPD_FLAGS_ALL 0x3Fu

/* TPD_FLAG_HERMITIAN: for a Hermitian A every weight is real (section
 * "Results" discusses the real-symmetric promise; Hermitian => real follows
 * from the definition).  Entry A[r][c] is the conjugate of A[c][r], and every
 * cumulative matrix weight of a Hermitian matrix is again Hermitian, so the
 * two-sweep schedule (n >= 9) reads and writes about half of the first
 * sweep's data and half of the second sweep's input, rebuilds the rest by
 * conjugation on chip, and stores the weights with imaginary parts +0.0.
 * The real parts are bitwise those of the general schedule.  Results are
 * undefined if A is not Hermitian.  n <= 8 runs the general schedule.     */

/* Largest supported n: 16 for TPD_C128, 17 for TPD_C64, TPD_R64 and
 * TPD_R32 (288 GB of HBM: an n = 17 complex128 matrix alone takes 256 GiB;
 * n = 17 runs a first sweep of 9 levels with tiles of at most 2^5
 * XOR-diagonals).  -1 for an unknown dtype. */
int tpd_max_qubits(tpd_dtype_t dtype);

/* Decompose one matrix, complex128, canonical layout, pruning on.
 * Section "Methods"; Fig. 1, Algorithms 1 and 2.
 *   A      [in]  device, 2^n x 2^n complex128, row-major
 *   n      [in]  0 <= n <= tpd_max_qubits(TPD_C128)
 *   coeffs [out] device, 4^n complex128; may equal A only if n <= 6
 *   stream [in]  hipStream_t or NULL                                     */
tpd_status_t tpd_decompose(const void* A, int n, void* coeffs, tpd_stream_t stream);

/* Same, with the dtype (TPD_C128, TPD_C64, TPD_R64, TPD_R32) and flags
 * (TPD_FLAG_NO_PRUNE, TPD_FLAG_LAYOUT_MATRIX, TPD_FLAG_ORDER_BOTTOM,
 * TPD_FLAG_HERMITIAN, TPD_FLAG_ROTATE_TILES) chosen by the caller.  coeffs may equal A (in place)
 * for any n with TPD_FLAG_LAYOUT_MATRIX and for n <= 6 in the canonical
 * order; otherwise TPD_ERROR_UNSUPPORTED.                                 */
tpd_status_t tpd_decompose_ex(const void* A, int n, void* coeffs, tpd_dtype_t dtype, unsigned flags,
                              tpd_stream_t stream);

/* Hermitian A, real weights (section "Preliminaries": the weights of a
 * Hermitian matrix are real; TPD_FLAG_HERMITIAN above for the schedule).
 * The weights go to a separate array of real values in canonical order:
 * weights[q] = w_q (binary64 for TPD_C128, binary32 for TPD_C64), 4^n x
 * 8 (4) bytes, half the bytes of a complex output.  A is overwritten: the
 * first sweep works in place in it (matrix layout, representatives only),
 * the second reads it and writes only the weights, so the second sweep
 * stores half the bytes of the complex Hermitian mode.  The values are
 * bitwise the real parts of tpd_decompose_ex with TPD_FLAG_HERMITIAN.
 *   A       [in/out] device, 2^n x 2^n TPD_C128 or TPD_C64, row-major,
 *                    Hermitian (results undefined otherwise); destroyed
 *   weights [out]    device, 4^n reals; must not overlap A
 *   flags   [in]     0 or TPD_FLAG_NO_PRUNE
 * Other dtypes or flags, misaligned or overlapping buffers:
 * TPD_ERROR_INVALID_VALUE; n out of range: TPD_ERROR_UNSUPPORTED.  n <= 8
 * runs one sweep from A (not modified) into the weights.  Uses the
 * per-(device, stream) pruning workspace as tpd_decompose_ex.            */
tpd_status_t tpd_decompose_hermitian_real(void* A, int n, void* weights, tpd_dtype_t dtype, unsigned flags,
                                          tpd_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * decomposition as tpd_decompose_ex, with the same arguments, errors and
 * results (bitwise), but the pruning bitmap lives in a static device array
 * of 256 KiB that the library holds on each device it runs on until the
 * process ends, instead of a workspace.  The call allocates and frees
 * nothing.  The array's address on a device is looked up on the first call
 * on that device (TPD_ERROR_LAUNCH if that fails).  Every call on a device
 * shares that device's array and clears it (with a fill kernel) before use,
 * so calls that overlap on one device, e.g. on two streams, race and give
 * undefined results; calls ordered by one stream are fine.  A schedule
 * whose bitmap exceeds the array is TPD_ERROR_UNSUPPORTED (none does:
 * the largest, n = 16 at tile width 2^3 or n = 17 at 2^4, takes 2^21
 * bits).  TPD_FLAG_TIMING is TPD_ERROR_INVALID_VALUE.                   */
tpd_status_t tpd_decompose_noalloc(const void* A, int n, void* coeffs, tpd_dtype_t dtype, unsigned flags,
                                   tpd_stream_t stream);

/* Inverse transform (synthesis), eq. (PauliDecomposition) read left to
 * right: A = sum_t w_t sigma^t, by the same n levels with the inverse
 * slicing step (u, v) = (s + t conj(w), s - t conj(w)), w = i on X/Y
 * diagonals, no scaling.
 *   coeffs [in]  device, 4^n weights, canonical order or (with
 *                TPD_FLAG_LAYOUT_MATRIX) the matrix layout
 *   A      [out] device, 2^n x 2^n row-major; may equal coeffs with
 *                TPD_FLAG_LAYOUT_MATRIX (any n) or for n <= 6
 *   flags  TPD_FLAG_LAYOUT_MATRIX only (TPD_FLAG_NO_PRUNE is accepted and
 *          ignored); anything else is TPD_ERROR_INVALID_VALUE.            */
tpd_status_t tpd_synthesize_ex(const void* coeffs, int n, void* A, tpd_dtype_t dtype, unsigned flags,
                               tpd_stream_t stream);

/* Partial decomposition: the weights of requested strings only (section
 * "Methods", the partial variant of Fig. 2 / Algorithm 3).  The paper slices
 * only the children in the request tree; here the unit of skipping is a
 * tile: a first-sweep d-group (2^db XOR-diagonals, all rows; the narrowest
 * tile width is used) runs only if a requested string has its X/Y mask in
 * that group, and a second-sweep tile only if a requested string lies in it
 * (and, with pruning, its cumulative matrix weight is nonzero).  The groups
 * and tiles to run are compacted into device work lists, so the cost
 * follows the work requested.  n <= 8 computes everything.  Requested
 * values are bitwise those of tpd_decompose_ex with the same dtype and
 * flags.
 *   A      [in]  device matrix, as tpd_decompose_ex (not modified unless
 *                coeffs == A)
 *   coeffs [out] device, 4^n elements of work/output, layout per flags; on
 *                return it holds the requested weights at their positions,
 *                every other element is unspecified.  May equal A with the
 *                same rules as tpd_decompose_ex.
 *   req    [in]  device array[count] of canonical indices q, any order,
 *                repeats allowed; q >= 4^n yields NaN + NaN i
 *   count  [in]  number of requests (0: nothing is enqueued)
 *   values [out] device array[count] of the dtype, values[s] = w_req[s]
 *                (real-coded for TPD_R64 / TPD_R32; NaN for q >= 4^n)
 *   flags  TPD_FLAG_NO_PRUNE, TPD_FLAG_LAYOUT_MATRIX, TPD_FLAG_HERMITIAN,
 *          TPD_FLAG_ORDER_BOTTOM; TPD_FLAG_TIMING is TPD_ERROR_INVALID_VALUE
 * Workspace: two request bitmaps (2^(n-db) and 2^(n1+n-db) bits) and two
 * work lists (32-bit entries, one per bit) per (device, stream), plus the
 * pruning bitmap.                                                         */
tpd_status_t tpd_decompose_partial(const void* A, int n, void* coeffs, const uint64_t* req, uint64_t count,
                                   void* values, tpd_dtype_t dtype, unsigned flags, tpd_stream_t stream);

/* Sparse-list output: the nonzero weights as (q, w) pairs, the list L that
 * Algorithms 1 and 2 return (section "Methods").  Ordered stream
 * compaction of a coefficient array: an element is kept unless both |re|
 * and |im| are <= tol (real-coded dtypes: unless |r| <= tol), compared in
 * the dtype's precision, tol rounded to it; NaN is kept.  Pairs appear in storage order: ascending q for the
 * canonical layout, ascending (row h, column l) for the matrix layout.
 *   coeffs   [in]  device, 4^n coefficients (canonical, or matrix layout
 *                  with TPD_FLAG_LAYOUT_MATRIX; no other flag)
 *   tol      [in]  >= 0 (0: exact nonzeros); negative or NaN is
 *                  TPD_ERROR_INVALID_VALUE
 *   q_out    [out] device array[capacity] of canonical indices
 *   w_out    [out] device array[capacity] of the dtype
 *   capacity [in]  entries available; only the first `capacity` pairs are
 *                  written (q_out and w_out may be NULL when it is 0)
 *   count    [out] device, one uint64: the total number of kept pairs
 *                  (may exceed capacity)
 * Cost: one read of the array to count per chunk of 4096 elements, an
 * exclusive scan of the chunk counts, and a second read of the chunks that
 * hold kept elements.  Workspace: 12 bytes per chunk per (device, stream). */
tpd_status_t tpd_compact(const void* coeffs, int n, tpd_dtype_t dtype, unsigned flags, double tol, uint64_t* q_out,
                         void* w_out, uint64_t capacity, uint64_t* count, tpd_stream_t stream);

/* Decompose `count` independent matrices of mixed sizes in one persistent
 * kernel launch (the paper's motivation: many time steps of a
 * time-dependent Hamiltonian, section "Introduction").
 *   ptrs     [in] HOST array[count] of device pointers to the matrices
 *   ns       [in] HOST array[count], 0 <= ns[i] <= 9
 *   count    [in] >= 0 (0 is a no-op)
 *   out_ptrs [in] HOST array[count] of device pointers to 4^ns[i]
 *                 coefficients each, or NULL for in place (in place needs
 *                 TPD_FLAG_LAYOUT_MATRIX when any ns[i] > 6)
 * The pointer tables are copied to the device before the call returns.  */
tpd_status_t tpd_decompose_batched(const void* const* ptrs, const int* ns, int count, void* const* out_ptrs,
                                   tpd_dtype_t dtype, unsigned flags, tpd_stream_t stream);

/* ---- plans: all allocation at creation, execution is graph-capturable ---- */
typedef struct tpd_plan_s* tpd_plan_t;

/* Plan for one n-qubit matrix (flags as tpd_decompose_ex plus
 * TPD_FLAG_TIMING).  `in_place` selects the in-place schedule.           */
tpd_status_t tpd_plan_create(int n, tpd_dtype_t dtype, unsigned flags, int in_place, tpd_plan_t* plan);

/* Plan for a batch of matrices with qubit counts ns[0..count) (HOST array,
 * copied).  The work table is sorted largest-first and uploaded now.     */
tpd_status_t tpd_plan_create_batched(const int* ns, int count, tpd_dtype_t dtype, unsigned flags,
                                     int in_place, tpd_plan_t* plan);

/* Execute a single-matrix plan.  A / coeffs as in tpd_decompose_ex.
 * Allocates nothing and synchronises nothing: safe inside hipGraph capture. */
tpd_status_t tpd_plan_execute(tpd_plan_t plan, const void* A, void* coeffs, tpd_stream_t stream);

/* Execute a batched plan.  d_ptrs / d_out_ptrs are DEVICE arrays[count] of
 * device pointers (d_out_ptrs may be NULL for a plan created in place).
 * Allocates nothing: safe inside hipGraph capture.                        */
tpd_status_t tpd_plan_execute_batched(tpd_plan_t plan, const void* const* d_ptrs, void* const* d_out_ptrs,
                                      tpd_stream_t stream);

tpd_status_t tpd_plan_destroy(tpd_plan_t plan);

/* Kernels per execution of the plan and their names (for profiling). */
int tpd_plan_num_kernels(tpd_plan_t plan);

/* With TPD_FLAG_TIMING: accumulated milliseconds and launch counts of each
 * kernel of the plan since creation or the last reset.  Synchronises the
 * recorded events (call after the stream is idle).  ms/counts: arrays of
 * at least tpd_plan_num_kernels(plan) entries.                          */
tpd_status_t tpd_plan_timing(tpd_plan_t plan, double* ms, uint64_t* counts, int reset);

/* Zero-block statistics of the last execution of a single-matrix plan with
 * pruning on: second-sweep tiles that were live, the total, and the number
 * of live cumulative matrix weights after the first sweep (the paper's
 * frontier |S^{n1+1}|, Fig. 1, Algorithm 2).  Synchronises `stream`.     */
tpd_status_t tpd_plan_prune_stats(tpd_plan_t plan, uint64_t* live_tiles, uint64_t* total_tiles,
                                  uint64_t* live_prefixes, int* prefix_level, tpd_stream_t stream);

/* JSON text describing the plan (sweeps, tile shapes, layouts, bytes). */
tpd_status_t tpd_plan_describe(tpd_plan_t plan, char* buf, size_t len);

/* ---- autotuning ---- */

/* Time the candidate two-sweep schedules for (n, dtype, layout, placement,
 * TPD_FLAG_HERMITIAN) on the caller's buffers and make the fastest the one
 * every later call and plan with the same key uses on this process (and,
 * if the environment variable TPD_AUTOTUNE_CACHE names a file, appended
 * there and reloaded by later processes).  Candidates: tile widths of
 * 2^3..2^5 (complex128) or 2^4..2^6 (complex64 and the real dtypes)
 * XOR-diagonals, one workgroup per tile or a persistent grid of 1, 2, 4 or
 * 8 workgroups per CU (which load the next tile while transforming the
 * current one); then the fastest of these once more with the second
 * sweep's rotated tile order (TPD_FLAG_ROTATE_TILES: which tiles run side by
 * side, hence how their rows meet the memory channels, depends on where the
 * buffer sits in physical memory); then, outside the Hermitian mode, the
 * winner in the chunked order (sweep 1 then sweep 2 over 32 MB to 512 MB
 * of XOR-diagonal strips at a time, on one stream or pipelined over two,
 * see tpd_debug_decompose_tuned).  A pipelined choice makes later
 * calls on a stream create a second stream (default priority) and events,
 * kept until tpd_release_workspace (plans: until tpd_plan_destroy).
 * The choice never changes results (same operations in the same order).
 * Timed runs are the schedule as it will run, pruning included unless
 * TPD_FLAG_NO_PRUNE is given.  Arguments as tpd_decompose_ex; `coeffs` is
 * overwritten; with A == coeffs the matrix is destroyed: before every
 * timed run (untimed) it is refilled with seeded uniform noise in [-1, 1),
 * so that the values do not decay to zero over repeated transforms.  Allocates
 * a bitmap, synchronises `stream`.  report/len (optional): JSON of the
 * candidates' median times and the choice.  n <= 8 has nothing to tune.   */
tpd_status_t tpd_autotune(const void* A, int n, void* coeffs, tpd_dtype_t dtype, unsigned flags,
                          tpd_stream_t stream, char* report, size_t len);

/* Autotune a batched plan: for each n in the plan, time the item shapes of
 * tpd_debug_plan_batched_codes (full tile with and without prefetch, half
 * tile) on that n's matrices alone and keep the fastest; then time the
 * persistent kernel with 1, 2, 3, 4, 6 or 8 workgroups per CU, or one
 * workgroup per work item, and keep the fastest.  The choices apply to this
 * plan and become the defaults of later batched plans and calls of the
 * dtype (and, with TPD_AUTOTUNE_CACHE, of later processes).
 * d_ptrs / d_out_ptrs as tpd_plan_execute_batched; outputs are
 * overwritten.  Synchronises `stream`.                                     */
tpd_status_t tpd_autotune_batched(tpd_plan_t plan, const void* const* d_ptrs, void* const* d_out_ptrs,
                                  tpd_stream_t stream, char* report, size_t len);

/* Release the per-(device, stream) workspaces held for tpd_decompose*. */
tpd_status_t tpd_release_workspace(void);

/* ---- host helpers (no device access) ---- */
const char* tpd_status_string(tpd_status_t status);

/* "XYZI..." (first letter = first tensor factor) -> canonical q; UINT64_MAX
 * for an empty string, more than 32 letters or a letter outside IXYZ.    */
uint64_t tpd_index_from_string(const char* s);

/* canonical q -> n-letter string in buf (needs n+1 bytes); 0 on success. */
int tpd_string_from_index(uint64_t q, int n, char* buf, size_t len);

/* Describe the sweep schedule chosen for (n, dtype, flags, in_place) as
 * JSON without touching a device (used by host-side tests).             */
tpd_status_t tpd_schedule_describe(int n, tpd_dtype_t dtype, unsigned flags, int in_place, char* buf,
                                   size_t len);

/* Host replay of the exact device schedule (same tile maps, thread roles,
 * LDS exchanges and arithmetic, executed sequentially on the CPU) for
 * small n.  A debugging aid for the index algebra; the library never uses
 * it to produce results.  A / coeffs are HOST pointers.                  */
tpd_status_t tpd_debug_emulate(const void* A, int n, void* coeffs, tpd_dtype_t dtype, unsigned flags,
                               int in_place);

/* As tpd_debug_emulate with a forced two-sweep tile width 2^db (db = 0:
 * the default schedule); r must be 0 or 4 (elements per thread = 16);
 * chunk_bits > 0 (with db > 0) runs the chunked order of
 * tpd_debug_decompose_tuned, and chunk_window >= 2 replays its pipelined
 * form in one order its streams allow, checking that no element is touched
 * by two chunks.                                                          */
tpd_status_t tpd_debug_emulate_tuned(const void* A, int n, void* coeffs, tpd_dtype_t dtype, unsigned flags,
                                     int in_place, int db, int r, int chunk_bits, int chunk_window);

/* One decomposition on the device with a forced two-sweep schedule: tile
 * width 2^db, 2^r elements per thread (r = 4), grid_per_cu workgroups per
 * CU (0 = one per tile), and chunk_bits: 0 runs each sweep over the whole
 * matrix, k > 0 runs sweep 1 then sweep 2 over 2^k first-sweep d-groups
 * (XOR-diagonal strips of 2^db) at a time, 2^(n-db-k) chunks (needs
 * k < n - db, not with TPD_FLAG_HERMITIAN).  chunk_window: 0 runs the
 * chunks one after the other on `stream`; w in 2..8 (with k > 0) runs
 * sweep 2 of chunk c on a second stream while sweep 1 of the next w - 1
 * chunks runs on `stream` (sweep 1 of chunk c waits for sweep 2 of chunk
 * c - w; `stream` waits for the last sweep 2).  For tests that every
 * tunable schedule gives the same bits; arguments and errors otherwise as
 * tpd_decompose_ex, and TPD_ERROR_INVALID_VALUE for a schedule that does
 * not exist.  n <= 8 ignores the schedule arguments.                      */
tpd_status_t tpd_debug_decompose_tuned(const void* A, int n, void* coeffs, tpd_dtype_t dtype, unsigned flags,
                                       int db, int r, int grid_per_cu, int chunk_bits, int chunk_window,
                                       tpd_stream_t stream);

/* tpd_decompose_hermitian_real with a forced two-sweep tile width 2^db
 * (db = 0: the tuned or default one) and grid_per_cu workgroups per CU (0 =
 * one per tile), for tests that every schedule gives the same bits;
 * TPD_ERROR_INVALID_VALUE for a schedule that does not exist.            */
tpd_status_t tpd_debug_decompose_hermitian_real_tuned(void* A, int n, void* weights, tpd_dtype_t dtype,
                                                      unsigned flags, int db, int grid_per_cu,
                                                      tpd_stream_t stream);

/* Host replays of the partial decomposition (request marking, tile skips,
 * gather) and of the compaction (same chunks, order and clipping); HOST
 * pointers, n <= 12, otherwise the arguments of the device calls.         */
tpd_status_t tpd_debug_emulate_partial(const void* A, int n, void* coeffs, const uint64_t* req, uint64_t count,
                                       void* values, tpd_dtype_t dtype, unsigned flags, int in_place);
tpd_status_t tpd_debug_emulate_compact(const void* coeffs, int n, tpd_dtype_t dtype, unsigned flags, double tol,
                                       uint64_t* q_out, void* w_out, uint64_t capacity, uint64_t* count);

/* Autotune tpd_decompose_hermitian_real for this (n, dtype): tile widths
 * and grids as tpd_autotune, each timed on A and weights (A destroyed:
 * refilled with seeded noise before every run, as tpd_autotune does in
 * place); the choice applies to later calls of the dtype
 * and n (and, with TPD_AUTOTUNE_CACHE, of later processes).  Without a
 * choice of its own the real-weights schedule takes the in-place Hermitian
 * mode's.  Arguments and errors as tpd_decompose_hermitian_real; allocates
 * a bitmap, synchronises `stream`; report/len (optional): JSON of the
 * candidates' median times and the choice.  n <= 8 has nothing to tune.  */
tpd_status_t tpd_autotune_hermitian_real(void* A, int n, void* weights, tpd_dtype_t dtype, unsigned flags,
                                         tpd_stream_t stream, char* report, size_t len);

/* Host replay of tpd_decompose_hermitian_real (HOST pointers, n <= 12; A
 * is overwritten as on the device).                                       */
tpd_status_t tpd_debug_emulate_hermitian_real(void* A, int n, void* weights, tpd_dtype_t dtype, unsigned flags);

/* Host replay of the synthesis schedule (HOST pointers, small n). */
tpd_status_t tpd_debug_emulate_synth(const void* coeffs, int n, void* A, tpd_dtype_t dtype, unsigned flags,
                                     int in_place);

/* Host replay of the batched schedule for one batch (HOST pointer arrays);
 * codes: NULL (the tuned or default shapes) or array[10] of per-n shape
 * codes as tpd_debug_plan_batched_codes takes.                            */
tpd_status_t tpd_debug_emulate_batched(const void* const* ptrs, const int* ns, int count, void* const* out_ptrs,
                                       tpd_dtype_t dtype, unsigned flags, const int* codes);

/* Rebuild a batched plan's work table with forced per-n shape codes
 * (array[10], index n): 0 = items filling the 2^BT-element tile, with the
 * next item's loads issued before the current one is transformed; 1 = the
 * same without that prefetch; 2 (n >= 3) = items of half a tile (half as
 * many matrices per item, or d-groups half as wide), with prefetch.  For
 * tests that every shape gives the same bits.  Allocates; not
 * graph-capturable.  TPD_ERROR_INVALID_VALUE for an invalid code.          */
tpd_status_t tpd_debug_plan_batched_codes(tpd_plan_t plan, const int* codes);

#ifdef __cplusplus
}
#endif

#endif /* TPD_H_ */
