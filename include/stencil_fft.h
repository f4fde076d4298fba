/*
 * stencil_fft.h -- C ABI of the MI355X (gfx950) FFT stencil solver.
 *
 * The library evolves a grid T timesteps under a linear, constant-coefficient
 * stencil in time independent of T up to a log T factor, by the method of
 * Ahmad et al., "Fast Stencil Computations using Fast Fourier Transforms"
 * (SPAA 2021):
 *
 *   periodic  (Sec. 3, algorithm StencilFFT-P, Eq. "final_data"):
 *             a_T = F^-1 Lambda^T F a_0, with Lambda = F s the DFT of the first
 *             column s of the circulant stencil matrix (appendix, eigenvalue-FFT
 *             relation), Lambda^T by binary repeated squaring (Step 2), the
 *             product (Step 3) and the inverse transform (Step 4);
 *   aperiodic (Sec. 4, StencilFFT-A with RecursiveBoundary): the periodic solve
 *             on the interior plus a divide-and-conquer over time for the cells
 *             within radius*T of a fixed boundary frame.
 *
 * Every function is extern "C"; no C++ exception crosses the ABI.  All functions
 * return SFFT_OK (0) or a negative error code; stencil_fft_last_error() then
 * returns a message for the calling thread.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  grid    DEVICE pointer (e.g. torch.Tensor.data_ptr()) to a dense row-major
 *          array of float (SFFT_F32) or double (SFFT_F64); dims[0] is the slowest
 *          axis.  Overwritten in place with the result.  The caller owns it and
 *          must keep it alive and untouched until the work enqueued on `stream`
 *          has completed.
 *  dims    HOST pointer to ndim extents (ndim in 1..3, every extent >= 1).
 *  coeffs  HOST pointer to (2*radius+1)^ndim doubles, row-major over the offsets
 *          o_0..o_{ndim-1} in [-radius, radius]; coeffs[o] multiplies the
 *          neighbour a[(i + o) mod dims] when cell i is updated (the periodic
 *          looping algorithm's S[i, (i+j) % N] convention, Sec. 2).  Copied
 *          before the call returns.  Always FP64: the symbol and its power are
 *          evaluated in FP64 whatever the grid's dtype.
 *  T       number of timesteps, >= 0; T == 0 leaves the grid unchanged.
 *  stream  hipStream_t to enqueue on (NULL = the null stream).  Calls return
 *          once the work is enqueued; synchronise the stream to read results.
 *
 * Errors: SFFT_EINVAL (null pointer, ndim outside 1..3, an extent < 1,
 * radius < 0, T < 0, a non-finite coefficient, an unknown dtype);
 * SFFT_EUNSUPPORTED (a shape the FFT planner cannot handle: a prime factor above
 * 7 in an extent of the no-allocation entry point, a radius above 8 (periodic) or
 * above 2 (aperiodic, fields, implicit), a radius above 2 on an extent with a
 * prime factor above 7, a 7-smooth 1-D extent of the fields or implicit entry
 * points longer than one row);
 * SFFT_ENOMEM (device workspace);
 * SFFT_EHIP (a HIP runtime error; the grid is then unspecified).  When
 * validation fails the grid is untouched.
 *
 * The library owns its device workspace, FFT plans and twiddle/phase/chirp-z
 * tables, kept in an implicit per-device context and released at process exit;
 * the first call that needs a new table or a larger workspace allocates it (and
 * chirp-z tables synchronise the stream once while they are built).
 * Workspace is per (device, stream): calls on one stream are ordered by the
 * stream; calls on different streams of one device may run concurrently.
 */
#ifndef STENCIL_FFT_H
#define STENCIL_FFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { SFFT_F32 = 0, SFFT_F64 = 1 } sfft_dtype;

enum {
    SFFT_OK = 0,
    SFFT_EINVAL = -1,
    SFFT_EUNSUPPORTED = -2,
    SFFT_ENOMEM = -3,
    SFFT_EHIP = -4,
    SFFT_EBUSY = -5,
    SFFT_ENOTFOUND = -6
};

/* Boundary conditions of the aperiodic solve (Sec. 4 leaves the choice to the
 * base case of RecursiveBoundary). */
enum {
    SFFT_BC_FIXED = 0,   /* Dirichlet: the frame holds fixed boundary values        */
    SFFT_BC_REFLECT = 1  /* zero-flux (Neumann): before every step each frame cell
                            takes the value of its mirror image about the cell faces
                            (interior cell r + k for frame cell r - 1 - k along each
                            axis it lies outside of)                                 */
};

/*
 * Periodic stencil solve (Sec. 3, StencilFFT-P; d-D form in the appendix on
 * d-D grids).  grid holds prod(dims) cells; on return (once the stream has run)
 * it holds a_T = S^T a_0 with periodic wrap on every axis.  Extents smaller than
 * 2*radius+1 are legal; offsets then alias modulo the extent exactly as the
 * periodic loop's modulo does.  Any extent from 1 to 2^30 is accepted: when every
 * extent is 7-smooth (2^a 3^b 5^c 7^d) the real-to-complex pass schedule runs;
 * otherwise each axis with a prime factor above 7 takes its DFT by Bluestein's
 * chirp-z algorithm (a circular convolution of a 7-smooth length >= 2n - 1) and
 * the others complex transforms, several times slower than a 7-smooth extent.
 * Radius 0..2 runs the fused pass schedule (the symbol power inside the middle
 * pass); radius 3..8 (7-smooth extents; a 1-D extent must fit one row, n/2 <= 8192)
 * runs the forward passes, one kernel that forms the symbol of any radius and its
 * power per mode, and the inverse passes.
 * Accuracy: relative L2 error against the exact result about 1e-6 (F32) and
 * 1e-14 (F64) for stable stencils; the symbol power is always FP64.
 */
int stencil_fft_periodic(void* grid, sfft_dtype dtype, int ndim, const int64_t* dims,
                         const double* coeffs, int radius, int64_t T, void* stream);

/*
 * Aperiodic stencil solve with a fixed (Dirichlet) boundary (Sec. 4,
 * StencilFFT-A and RecursiveBoundary).  grid has extents dims[i] + 2*radius: the
 * outer radius-wide frame holds the boundary values, is only read and is left
 * unchanged; the inner prod(dims) cells are evolved T steps, each step reading
 * frame cells where the stencil reaches them (the aperiodic looping algorithm of
 * Sec. 2 with radius boundary cells on each side).  Interior extents need not
 * be 7-smooth (FFT sub-problems are zero-padded where the method allows it).
 * Independent parts of the recursion run on helper streams forked from and
 * joined back into `stream`; repeated identical calls are replayed from a
 * captured graph (option "aperiodic_graphs").  Calls that share a stream must
 * not be issued from several host threads at once.
 */
int stencil_fft_aperiodic(void* grid, sfft_dtype dtype, int ndim, const int64_t* dims,
                          const double* coeffs, int radius, int64_t T, void* stream);

/*
 * stencil_fft_aperiodic with a choice of boundary condition (Sec. 4: the FFT
 * parts of RecursiveBoundary only keep cells whose dependency cone stays inside
 * the interior, so the boundary enters through the base case alone).
 *   bc  SFFT_BC_FIXED: exactly stencil_fft_aperiodic.
 *       SFFT_BC_REFLECT: the frame's values are never read and are left
 *       unchanged; the interior evolves as if, before every step, the frame held
 *       the mirror image of the interior.  Every interior extent must be at least
 *       radius (SFFT_EINVAL otherwise).
 * Other bc values: SFFT_EINVAL.  Everything else as stencil_fft_aperiodic.
 */
int stencil_fft_aperiodic_bc(void* grid, sfft_dtype dtype, int ndim, const int64_t* dims,
                             const double* coeffs, int radius, int64_t T, int bc, void* stream);

/*
 * Vector-valued fields (the appendix on vector-valued fields): nfields scalar
 * fields on one periodic grid evolve together, field i at t+1 being the sum over j
 * of the circulant stencil (i, j) applied to field j at t.  Affine updates and
 * updates that read several earlier time steps are instances (an extra constant
 * field; earlier steps carried as fields).
 *   grid    DEVICE pointer to nfields * prod(dims) elements, field-major
 *           ([nfields][dims...]); overwritten with the fields after T steps.
 *   nfields 1..4 (SFFT_EUNSUPPORTED above 4).
 *   coeffs  HOST pointer to nfields * nfields * (2*radius+1)^ndim doubles,
 *           [i][j][offsets...]: block (i, j), laid out like the scalar
 *           coefficients, weights field j's neighbours in field i's update; copied
 *           before the call returns.
 * The forward transforms of all fields run as one batch, the m x m symbol matrix
 * of every mode is raised to the power T by repeated squaring in FP64 (deviation
 * form), and the inverse transforms follow.  Extents with a prime factor above 7
 * take the chirp-z transforms of stencil_fft_periodic along those axes (all axes
 * then complex, the symbol matrix applied over the full spectrum); a 7-smooth 1-D
 * extent must fit one row (n/2 <= 8192 for even n, n <= 8192 for odd n).  Errors
 * as for stencil_fft_periodic.
 */
int stencil_fft_periodic_fields(void* grid, sfft_dtype dtype, int nfields, int ndim, const int64_t* dims,
                                const double* coeffs, int radius, int64_t T, void* stream);

/*
 * Implicit stencils (the appendix on implicit stencils): the update
 * Q a_{t+1} = S a_t on a periodic grid, with both Q and S linear stencils.  Every
 * mode evolves by lambda_R = lambda_S / lambda_Q, and by 0 where lambda_Q vanishes
 * (the pseudo-inverse of Q; |lambda_Q| at or below 16 * DBL_EPSILON * sum |q| counts
 * as zero), raised to the power T in FP64.
 *   q_coeffs, s_coeffs  HOST pointers to (2*radius+1)^ndim doubles each, laid out
 *                       like the scalar coefficients; copied before return.
 * Other arguments, extent rules and errors as for stencil_fft_periodic_fields with
 * one field.
 */
int stencil_fft_periodic_implicit(void* grid, sfft_dtype dtype, int ndim, const int64_t* dims,
                                  const double* q_coeffs, const double* s_coeffs, int radius, int64_t T,
                                  void* stream);

/*
 * Periodic solve that allocates no device memory.  For callers that cannot
 * allocate: code under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, result and validation as stencil_fft_periodic, for
 * 7-smooth extents only (others: SFFT_EUNSUPPORTED); the result is bit-identical
 * to stencil_fft_periodic's on the same input.
 * Everything the solve needs besides the caller's grid (twiddle and phase tables,
 * the per-column symbol table, the spectrum workspace) lives in one fixed device
 * array of STENCIL_FFT_NOALLOC_MAX_BYTES per GPU, held from the first call on that
 * GPU until the process ends; the tables are regenerated by small kernels on
 * `stream` at every call, and nothing in the array needs to start at zero.
 * A shape whose tables and workspace exceed the array is rejected with
 * SFFT_ENOMEM before anything is enqueued (for instance 2048 x 2048 fits in FP32
 * and FP64; 4096 x 4096 FP64 does not).
 * Every call on one GPU uses that GPU's single array: calls whose work may
 * overlap on one GPU (different streams, or different host threads, without
 * ordering between them) race and give wrong results.  Order them, e.g. by
 * issuing all such calls on one stream.
 */
#define STENCIL_FFT_NOALLOC_MAX_BYTES (64ull << 20)
int stencil_fft_periodic_noalloc(void* grid, sfft_dtype dtype, int ndim, const int64_t* dims,
                                 const double* coeffs, int radius, int64_t T, void* stream);

/* Message describing the last failing call on this thread ("" if none).  The
 * pointer stays valid until the thread's next call into the library. */
const char* stencil_fft_last_error(void);

/*
 * Symbol and its power (Sec. 3 Steps 1(i) and 2) on their own, for inspection
 * and testing.  out: DEVICE pointer to prod(dims) interleaved (re, im) double
 * pairs in natural frequency order (row-major over k_0..k_{ndim-1}); entry k
 * receives lambda(k)^T with lambda(k) = sum_o coeffs[o] exp(+2 pi i sum_a o_a k_a / dims[a])
 * (= (F s)[k], s the first column of the stencil matrix).  Same validation as
 * stencil_fft_periodic.
 */
int stencil_fft_symbol_power(double* out, int ndim, const int64_t* dims, const double* coeffs,
                             int radius, int64_t T, void* stream);

/* One problem of a batch or a serving request.  Unused dims entries are ignored. */
typedef struct {
    void* grid;            /* DEVICE pointer, as for the single-problem calls        */
    sfft_dtype dtype;
    int ndim;
    int64_t dims[3];
    const double* coeffs;  /* HOST pointer, (2*radius+1)^ndim doubles, copied       */
    int radius;
    int64_t T;
    int aperiodic;         /* 0: periodic (dims = grid extents); 1: aperiodic with
                              a fixed frame; 2: aperiodic with a reflecting frame
                              (SFFT_BC_REFLECT)                                     */
} sfft_problem;

/*
 * Solve n independent problems of uneven shapes, dtypes and T, enqueued on one
 * stream.  Periodic problems of 7-smooth extents and radius <= 2 are packed into
 * batched launches: one launch per pass index and kernel variant runs the tiles
 * of every problem's pass of that index that uses that variant.  The others
 * (aperiodic problems, periodic ones with a prime factor above 7 in an extent or
 * a radius above 2) are solved one after another on the same stream, with the
 * rules of their single-problem entry points.
 * Validation covers every problem before anything is enqueued: on error nothing
 * runs and the message names the offending problem index.
 */
int stencil_fft_batch(const sfft_problem* probs, int n, void* stream);

/*
 * A batch of periodic problems captured once into a hipGraph and replayed with
 * one launch.  The
 * graph binds the grids, coefficients and T given at creation; each replay
 * advances every grid by its T steps again, in place.  create() plans the
 * problems, allocates the graph's own workspace and captures the batched
 * program; it must not be called while another capture is active on the
 * calling thread.  Aperiodic problems are rejected (SFFT_EUNSUPPORTED).
 */
typedef struct sfft_graph sfft_graph;
int stencil_fft_graph_create(const sfft_problem* probs, int n, sfft_graph** out);
int stencil_fft_graph_launch(sfft_graph* g, void* stream);
void stencil_fft_graph_destroy(sfft_graph* g);

/*
 * Serving loop (continuous batching).  A server owns a worker thread, a set of
 * HIP streams and an HBM budget for workspace.  submit() never blocks: it
 * copies the request (coefficients included) and returns a ticket, or
 * SFFT_EINVAL / SFFT_EUNSUPPORTED for an invalid request, or SFFT_ENOMEM if the
 * request's own workspace exceeds the whole budget.  Every device buffer of the
 * server lives in one allocation of the budget made at creation: per-stream
 * descriptor buffers, and per admitted request one block with everything its
 * solve needs (the spectrum workspace and column table of a batched periodic
 * request; every buffer of an aperiodic, chirp-z or radius > 2 request, sized at
 * submit on the host by the solver's own bookkeeping).  The worker admits queued
 * requests in arrival order while a slot is free and their block fits the
 * remaining budget, packs the admitted batchable ones into batched launches on a
 * free stream (the others run one after another on that stream), and releases
 * slot and budget when that stream's work completes, so
 * requests that arrive while others run join the next launch.  The grid of a
 * request must stay alive until poll() reports it done.
 *  create:  device = HIP device ordinal; hbm_budget_bytes = workspace budget
 *           (0 = 32 GiB); max_slots = requests in flight at most (0 = 64).
 *  poll:    *done = 1 once the result is in the grid, else 0; SFFT_ENOTFOUND
 *           for an unknown ticket; a failed request reports its error code.
 *  wait:    blocks until the ticket is done.
 *  stats:   JSON text (admitted, completed, launches, peak budget use) into buf.
 *  destroy: drains outstanding work, then frees everything.
 */
typedef struct sfft_server sfft_server;
int sfft_server_create(sfft_server** out, int device, uint64_t hbm_budget_bytes, int max_slots);
int sfft_server_submit(sfft_server* s, const sfft_problem* p, uint64_t* ticket);
int sfft_server_poll(sfft_server* s, uint64_t ticket, int* done);
int sfft_server_wait(sfft_server* s, uint64_t ticket);
int sfft_server_stats(sfft_server* s, char* buf, int64_t cap);
/* Seconds since server creation at which the ticket was submitted and found
 * complete by the worker (done_s = -1 while pending). */
int sfft_server_ticket_times(sfft_server* s, uint64_t ticket, double* submit_s, double* done_s);
void sfft_server_destroy(sfft_server* s);

/*
 * Host-side verification of the pass schedules a solve would run (no device
 * needed, nothing enqueued).  Each pass kernel's indices are affine in its loop
 * indices with non-negative strides, so the corner of each loop box bounds the
 * addresses it can touch; every pass of the solve is checked that way against
 * the buffers the solve hands it (spectrum workspace, real input and output
 * views, symbol column table, twiddle and stage tables), and row counts and
 * tile coverage against the transform extents.  kind 0: the periodic solve of
 * 7-smooth dims (stencil_fft_periodic); 1 / 2: the aperiodic solve with a fixed /
 * reflecting frame (stencil_fft_aperiodic_bc), whose whole RecursiveBoundary
 * bookkeeping (interior, slab and recursion-level solves, base-case strips) runs
 * with stand-in addresses under the current tunables.
 *   report  HOST buffer of cap bytes (may be NULL) receiving JSON
 *           {"checked": n, "failures": k, "errors": ["...", ...]} (first 64)
 * Returns the number of failures (0: every check passed) or a negative error
 * code (SFFT_EINVAL / SFFT_EUNSUPPORTED as the solve entry points would).
 */
int stencil_fft_verify(sfft_dtype dtype, int ndim, const int64_t* dims, const double* coeffs, int radius,
                       int64_t T, int kind, char* report, int64_t cap);

/*
 * Tunables (process-wide).  Names:
 *   "aperiodic_cutoff"  RecursiveBoundary recurses while T > cutoff; the base
 *                       case loops T' <= cutoff steps (default chosen per shape
 *                       when 0).
 *   "col_max"           longest sub-transform a strided pass performs (power of
 *                       two, 16..1024; default 0 = per-dtype choice).
 *   "generic_kernels"   1: run every pass on the generic (runtime-radix) kernels
 *                       instead of the power-of-two register kernels (testing).
 *   "aperiodic_graphs"  1 (default): stencil_fft_aperiodic captures the second
 *                       identical call (same grid address, shape, coefficients,
 *                       T, stream and tunables) into a graph and replays it on
 *                       later identical calls; 0: always enqueue directly.
 *   "mixed_row_q"       most points per thread of the register mixed-radix
 *   "mixed_col_q"       kernels on row / strided-axis passes (5, 10, 12, 20
 *                       or 25; 0 = default: the most the register budget
 *                       allows for the length's family and dtype).
 * Returns SFFT_EINVAL for an unknown name or an out-of-range value.
 */
int stencil_fft_set_option(const char* name, int64_t value);

/*
 * Autotuner (plans for the batched and single periodic solves).  For every
 * distinct extent of a strided axis (axes 0..ndim-2) of the given 7-smooth shape
 * it times whole solves (radius 1, T = 4096; three runs of `reps` back-to-back
 * solves per candidate, median) with each candidate factorisation of that axis into sub-transforms --
 * the planner's balanced default, the single transform when it fits (<= 1024
 * points), the most balanced two-level splits in both orders, or the orders of a
 * three-level split -- after checking each candidate's result (T = 3, every mode
 * visible) against the default schedule's to 1e-5 (F32) / 1e-12 (F64) relative
 * L2 and largest cell error; only candidates that pass may be chosen.  The
 * fastest is kept in the process-wide tuning database keyed by (extent, dtype),
 * which every later plan of that extent uses.  Allocates two grids of the shape
 * and synchronises the device while it runs.  report (may be NULL) receives JSON
 * of every candidate's time and error; returns its length or a negative code.
 * save / load write and read the database as JSON ({"version": 1, "splits":
 * [{"n": .., "f64": 0|1, "levels": [..]}, ..]}); load merges into the current
 * database; clear empties it.  (Not a step of the paper's method: plan
 * selection for the FFT passes.)
 */
int stencil_fft_tune(int ndim, const int64_t* dims, sfft_dtype dtype, int reps, char* report, int64_t cap);
int stencil_fft_tune_save(const char* path);
int stencil_fft_tune_load(const char* path);
int stencil_fft_tune_clear(void);

/*
 * Per-kernel timing with HIP events recorded on the launch stream around every
 * kernel the library enqueues.  enable != 0 clears and starts collection; 0
 * stops it.  read() writes JSON {"kernels": {name: {"launches": n, "ms": total,
 * "bytes": algorithmic bytes}}} into buf (cap bytes) after synchronising the
 * streams that were used; returns the length or a negative error.
 */
int stencil_fft_profile(int enable);
int stencil_fft_profile_read(char* buf, int64_t cap);

/*
 * The pass schedule the planner picks for a periodic problem, as JSON (passes,
 * kinds, sub-lengths, radices, tile shapes, algorithmic bytes per pass).
 * Host-only: needs no GPU.
 */
int stencil_fft_plan_describe(int ndim, const int64_t* dims, sfft_dtype dtype, char* buf, int64_t cap);

/* Library version string. */
const char* stencil_fft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STENCIL_FFT_H */
