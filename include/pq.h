/*
 * pq.h -- C ABI of the MI355X permanent engine (libpq.so).
 *
 * The engine computes Fock-basis transition amplitudes of a linear-optical
 * interferometer.  For an m-mode unitary U, input occupations S and output
 * occupations T (non-negative integers, n = sum S photons), the matrix
 * U_{T,S} is the n x n matrix whose rows are the output modes i repeated t_i
 * times and whose columns are the input modes j repeated s_j times, and
 *
 *     amp(S -> T) = perm(U_{T,S}) / sqrt(prod_j s_j! prod_i t_i!),
 *     p(S -> T)   = |amp|^2                      (Appendix, Eq. BS_prob),
 *
 * with perm(A) = sum over permutations sigma of prod_i A[sigma(i)][i]
 * (Appendix, Eq. per_def).  U_{T,S} is indexed U[output][input].
 *
 * The permanent is evaluated by the Balasubramanian-Bax-Franklin-Glynn
 * formula generalised to repeated rows and columns: the outer sum runs over
 * an n-ary Gray code whose digits range from zero to the occupation of each
 * mode (Benchmarks / Boson Sampling), with one sign fixed ("halving").
 *
 * Conventions shared by every entry point
 *   - Complex numbers are pq_c128 {double re, im}: the same bytes as
 *     torch.complex128, std::complex<double> and C99 double _Complex.
 *   - Matrices are row-major; a leading dimension counts complex elements.
 *   - Device pointers are HIP device memory on the ctx's device; occupation
 *     vectors and job descriptions are host memory (they drive planning).
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and is stream-ordered; the call returns before the GPU finishes.
 *     Device buffers must stay valid until that work completes.
 *   - Ownership: the caller owns every buffer it passes.  The library never
 *     frees caller memory; it allocates only workspace owned by the ctx.
 *   - Errors: a status code is returned synchronously; no C++ exception
 *     crosses the ABI.  Argument and planning errors leave outputs
 *     untouched.  Launch failures return PQ_EDEVICE.  pq_last_error() gives
 *     a human-readable detail for the last failing call on a ctx.
 *   - Threading: a ctx is not thread-safe and its workspace is reused by
 *     consecutive calls, so calls on one ctx must be issued on one stream
 *     (or the caller must order the streams).  Distinct ctxs are independent.
 *   - Special cases: sum S != sum T gives perm = amp = 0 with PQ_OK
 *     (a passive circuit conserves photon number); n = 0 gives perm = amp = 1.
 *     n > PQ_MAX_N, more than PQ_MAX_N distinct columns, or 2^62 or more
 *     Gray-code terms give PQ_ERANGE.
 */
#ifndef PQ_H
#define PQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } pq_c128;
typedef struct pq_ctx pq_ctx;

enum {
    PQ_OK = 0,
    PQ_EINVAL = 1,      /* invalid argument (NULL pointer, negative size or occupation, ldu < m) */
    PQ_ERANGE = 2,      /* problem too large for the engine */
    PQ_ENOMEM = 3,      /* device workspace allocation failed */
    PQ_EDEVICE = 4,     /* HIP runtime or launch error */
    PQ_ECANCELLED = 5   /* cancellation requested on the ctx (pq_cancel) */
};

#define PQ_MAX_N 48     /* photons per permanent, and distinct rows/columns */

/* Library version string, e.g. "pq 0.1 gfx950". Static storage. */
const char* pq_version(void);

/*
 * pq_device_peak -- the ctx's device as the HIP runtime reports it: compute
 * units (*cus), peak engine clock in kHz (*clock_khz), and the FP64 vector
 * peak they imply, cus x clock x 128 flops (4 SIMDs of 16 FP64 lanes per CU,
 * one FMA each per clock), in TFLOP/s (*fp64_tflops).  Host-only, no GPU
 * work.  NULL ctx or output: PQ_EINVAL.
 */
int pq_device_peak(pq_ctx* ctx, int32_t* cus, int32_t* clock_khz, double* fp64_tflops);

/* Create a context on HIP device `hip_device` (PQ_EINVAL for a bad ordinal or
 * NULL out, PQ_EDEVICE if the device cannot be queried).  *out is set only on
 * success.  The ctx owns device workspace, grown on demand.  Environment read
 * here: PQ_AUTOTUNE=1 turns chunk-policy autotuning on (pq_autotune_enable);
 * PQ_AUTOTUNE_CACHE=<file> loads this device's recorded tuning decisions from
 * that file and appends new ones to it (one JSON object per line, keyed by
 * the device's architecture and CU count and the job list's shape);
 * PQ_FAULT_INJECT (pq_fault_inject); PQ_QUEUE (pq_queue_mode); PQ_WALK
 * (pq_walk_variant); PQ_LHAF_PACK (pq_lhaf_pack); PQ_ALL_GEMM
 * (pq_all_outputs_gemm). */
int pq_create(pq_ctx** out, int hip_device);

/* Destroy a context (NULL-safe).  Waits for the device before freeing. */
void pq_destroy(pq_ctx* ctx);

/*
 * Cancellation.  pq_cancel(ctx, 1) sets a flag in pinned, device-mapped host
 * memory owned by ctx.  Work-queue launches of this ctx (pq_perm_batched)
 * poll it before every chunk they pop and stop popping once it is set: jobs
 * whose chunks were not all swept keep whatever their output buffers held.
 * Kernels of other entry points run to completion.  While the flag is set,
 * every entry point that enqueues GPU work returns PQ_ECANCELLED without
 * enqueuing anything; pq_cancel(ctx, 0) clears it.  Safe to call from another
 * thread while work is in flight (it only stores the flag).
 */
int pq_cancel(pq_ctx* ctx, int on);

/*
 * Fault injection for tests of error handling: while set, every device
 * allocation of ctx (PQ_FAULT_ALLOC: workspace, plan blocks) fails with
 * PQ_ENOMEM, or every launch check (PQ_FAULT_LAUNCH) fails with PQ_EDEVICE,
 * as if the runtime had refused it.  The ctx stays usable: clearing the
 * injection (PQ_FAULT_NONE) restores normal operation.  pq_create reads the
 * initial setting from the environment variable PQ_FAULT_INJECT (alloc |
 * launch).
 */
enum { PQ_FAULT_NONE = 0, PQ_FAULT_ALLOC = 1, PQ_FAULT_LAUNCH = 2 };
int pq_fault_inject(pq_ctx* ctx, int what);

/* Static description of a status code. */
const char* pq_strerror(int status);

/* Detail of the last failing call on ctx ("" if none); owned by ctx, valid
 * until the next call on ctx. */
const char* pq_last_error(const pq_ctx* ctx);

/*
 * pq_perm -- one amplitude (Eq. BS_prob, Eq. per_def).
 *   U      device, m x m complex, row-major, leading dimension ldu >= m.
 *   S, T   host int32[m]: input / output occupations (>= 0).
 *   perm   device, 1 complex, may be NULL: perm(U_{T,S}).
 *   amp    device, 1 complex, may be NULL: perm / sqrt(prod S! prod T!).
 * U must not be NULL when m > 0; S and T must not be NULL.
 * The sweep splits its Gray range evenly over two rounds of the resident
 * wavefronts (each at least 32 time states); with autotuning on
 * (pq_autotune_enable) the launch shape follows the autotuner instead.
 */
int pq_perm(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
            const int32_t* S, const int32_t* T,
            pq_c128* perm, pq_c128* amp, void* stream);

/*
 * pq_perm_noalloc -- pq_perm for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, and harnesses that
 * forbid allocation.  Same arguments, planning, errors and results as
 * pq_perm (the same kernels in the same launch geometry: the default, or
 * the autotuner's recorded decision for the shape), but the launch
 * sequence's scratch (compact matrix, +-2B rows, step tables, workgroup
 * partials) is a static device array of PQ_NOALLOC_SCRATCH_BYTES per GPU,
 * resolved by pq_create; the call itself allocates nothing (no hipMalloc,
 * hipFree or allocating library routine) and records no profiling events.
 *   - A permanent whose launch needs more scratch than that returns
 *     PQ_ERANGE (outputs untouched); pq_perm handles it.  Under the default
 *     launch shape every binary (collision-free) permanent up to n = 48
 *     fits; large mixed-radix ones with 4096-state step tables and 40
 *     distinct columns may not, nor may shapes the autotuner gave 4 rounds.
 *   - Every call on one GPU, from every ctx, shares that GPU's array: calls
 *     whose GPU work overlaps (other streams, other ctxs, other threads) race
 *     and give wrong results.  Calls ordered on one stream are safe; nothing
 *     in the array needs to start at zero.
 *   - PQ_EDEVICE if the array's address could not be resolved on this device.
 */
#define PQ_NOALLOC_SCRATCH_BYTES (160u * 1024u)
int pq_perm_noalloc(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
                    const int32_t* S, const int32_t* T,
                    pq_c128* perm, pq_c128* amp, void* stream);

/*
 * Batched jobs on one interferometer U (uneven sizes).  Jobs use the sparse
 * form: distinct row modes with their multiplicities (the output side) and
 * distinct column modes with theirs (the input side).
 *
 *   PQ_OP_PERM        one output: perm(U_{T,S}) (and amp) at out_offset.
 *                     Needs sum row_mult == sum col_mult (else 0, as pq_perm).
 *   PQ_OP_EXTEND_ROW  m outputs at out_offset .. out_offset+m-1:
 *                     out[l] = perm(U_{T+e_l, S}) for every mode l, i.e. the
 *                     Laplace expansion along one more output row used by
 *                     chain-rule boson sampling (Clifford-Clifford algorithm
 *                     A, Benchmarks / Boson Sampling).  Needs
 *                     sum col_mult == sum row_mult + 1; amp is not written
 *                     for this op.
 */
enum { PQ_OP_PERM = 0, PQ_OP_EXTEND_ROW = 1 };
typedef struct {
    int32_t op;
    int32_t nr, nc;              /* number of distinct rows / columns (>= 0) */
    const int32_t* row_idx;      /* host, nr mode indices in [0, m), distinct */
    const int32_t* row_mult;     /* host, nr multiplicities >= 1 */
    const int32_t* col_idx;      /* host, nc mode indices in [0, m), distinct */
    const int32_t* col_mult;     /* host, nc multiplicities >= 1 */
    int64_t out_offset;          /* element offset into perm[] / amp[] */
} pq_job;

/*
 * pq_perm_batched -- all jobs in one stream-ordered submission, scheduled as a
 * persistent work queue (the many uneven permanents of a boson-sampling run,
 * Benchmarks / Boson Sampling).  Jobs are planned and cut into chunks as in
 * pq_perm_many (identical jobs once, chunks longest first); per column class
 * one launch of resident wavefronts pops chunks from an atomic counter and
 * each chunk writes its own double-double slot; a final kernel then adds
 * every job's slots in slot order and writes its outputs.  The results equal
 * pq_perm_many's bit for bit.
 *   - The launch sequence (gather, step tables, counter reset, the class
 *     queues, the final kernel) is captured into a HIP graph the first time a plan runs with a
 *     given (U, ldu, perm, amp), and replayed on later calls (up to 4 graphs
 *     per cached plan; by default, and whatever pq_graph_enable says; calls
 *     with profiling on launch directly).  Fixed output buffers therefore
 *     replay one graph.
 *   - A plan whose every job is a single chunk (small jobs: all digits fit the
 *     lanes of one wavefront) has nothing for a queue to balance and runs the
 *     static schedule instead (one workgroup per chunk, then a final kernel).
 *   - Within a plan, a column class runs as a queue only when it has more
 *     chunks than resident wavefronts and they average at least 32 Gray time
 *     states; lighter classes take one workgroup per chunk in the same launch
 *     sequence (every pop is an atomic on one counter, and thousands of tiny
 *     chunks popped at once cost more than their sweeps).  pq_queue_mode
 *     overrides this.
 *   - Chunk sizes follow the autotuner when it is enabled (off by default: a
 *     first call then times 13 chunk policies under the queue, about 26 runs
 *     of the batch, and the kept policy under the static schedule as well;
 *     the faster schedule is recorded with the policy).  Recorded decisions
 *     (pq_autotune_enable, PQ_AUTOTUNE_CACHE) apply.  Untuned plans run the
 *     queue.
 *   - The work queue reads the ctx's cancellation word every 16 pops per
 *     wavefront (pq_cancel).
 *   perm  device, complex, large enough for every job's outputs.
 *   amp   device, may be NULL; written for PQ_OP_PERM jobs only.
 * Output ranges of different jobs must not overlap (PQ_EINVAL otherwise).
 */
int pq_perm_batched(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
                    const pq_job* jobs, int32_t njobs,
                    pq_c128* perm, pq_c128* amp, void* stream);

/*
 * pq_queue_mode -- which column classes pq_perm_batched runs as work queues:
 * PQ_QUEUE_AUTO (default: the rule above, and a tuned plan's recorded
 * schedule), PQ_QUEUE_ALWAYS (every class of a multi-chunk plan), or
 * PQ_QUEUE_NEVER (the static schedule throughout).  Results are the same bits
 * in every mode.  PQ_QUEUE=auto|always|never in the environment sets it at
 * pq_create.  NULL ctx or another value: PQ_EINVAL.
 */
enum { PQ_QUEUE_AUTO = 0, PQ_QUEUE_ALWAYS = 1, PQ_QUEUE_NEVER = 2 };
int pq_queue_mode(pq_ctx* ctx, int mode);

/*
 * pq_perm_many -- the same jobs and outputs as pq_perm_batched, scheduled
 * statically: every job's Gray-code range is cut into chunks on the host, one
 * wavefront sweeps one chunk and writes its own partial slot, and a second
 * kernel adds each job's slots in order (results do not depend on timing).
 * Plans and their device descriptors are cached per distinct job list, so a
 * repeated call with the same jobs only launches kernels.  EXTEND_ROW jobs
 * may have at most 24 distinct columns (PQ_ERANGE otherwise).
 */
int pq_perm_many(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
                 const pq_job* jobs, int32_t njobs,
                 pq_c128* perm, pq_c128* amp, void* stream);

/*
 * Chunk-size autotuning of pq_perm_many (the batched form: uneven jobs of a
 * boson-sampling run in one statically scheduled launch per column class).
 * A plan aims at num_cu * waves_per_cu * chunks_per_wave chunks per class,
 * none shorter than min_chunk Gray time states; the default policy is
 * (64, 8, 256): fine chunks for long uneven jobs (a short tail), and short
 * jobs kept whole.  It applies to pq_perm_batched as well, so the two calls
 * give the same bits on the same job list.
 *
 * pq_autotune_enable -- on (nonzero): the first pq_perm_many call on a job
 * list whose shape (m, and for every job kind and padded column count the
 * number of jobs and of Gray terms, each rounded to half an octave) has no
 * recorded policy plans and runs the job
 * list under each of 14 candidate policies (the default first), timing the
 * sweep kernels with HIP events (best of two runs each), keeps the fastest
 * plan and records its policy.  That call therefore runs the jobs about 28
 * times and synchronizes the stream; its outputs are those of the kept plan.
 * Later job lists of the same shape are planned with the recorded policy.
 * Results differ between policies only by the order of the double-double
 * partial sums.  Off (0, the default): the default policy.
 *   The same switch tunes pq_perm's launch shape: the first call on a plan
 * shape (kernel kind, column count, digit radices and column powers: n and
 * the multiplicity class) with no recorded decision runs the whole launch
 * sequence under 2, 1 and 4 rounds of the resident wavefronts (the default
 * first, best of two runs each, timed with HIP events around the sequence:
 * 6 runs, and the stream is synchronized), keeps the fastest, records it,
 * and then runs once more with it.  Later calls of that shape reuse the
 * record; pq_perm_noalloc follows a recorded decision but never times.
 * PQ_AUTOTUNE_CACHE persists these decisions too (kind "perm").
 *
 * pq_autotune_last -- the last decision: policy = {waves_per_cu,
 * chunks_per_wave, min_chunk} (for pq_perm: {wavefronts per CU, 1, 32}),
 * the kept plan's or shape's time and the default's (ms), and the number of
 * candidates timed (0: the decision came from the record).  All zero before
 * any tuning.  NULL arguments: PQ_EINVAL.
 */
/*
 * pq_graph_enable -- on (nonzero): pq_perm_many captures its launch sequence
 * for a plan (gather of the compact matrices, step tables, one sweep per
 * column class, final reduction; kernel nodes only) into a HIP graph the
 * first time it runs with a given (U, ldu, perm, amp), and afterwards
 * replays that graph on the caller's stream with one hipGraphLaunch.  Up to 4
 * graphs are kept per cached plan.  The graph reads U and writes perm/amp
 * through the captured pointers, so those buffers must stay allocated while
 * the plan is cached.  Calls with profiling on launch the kernels directly.
 * Off (0, the default): direct launches.  NULL ctx: PQ_EINVAL.
 */
int pq_graph_enable(pq_ctx* ctx, int on);

/*
 * pq_walk_variant -- the form of pq_perm_grad's reverse sweep for wide
 * collision-free patterns (16 to 32 photons, every mode at most once; the
 * differentiation of the permanent in the Goals and in the differentiable
 * Fock simulations of the Benchmarks).  register_digits (1..3): how many of
 * the lowest time digits keep their summation-by-parts accumulators in
 * registers (more registers per wavefront, fewer reductions through LDS and
 * device atomics); swizzle (0 or 1): the exchanges between the four lanes of
 * a term go through ds_swizzle instead of DPP moves.  Results agree to
 * rounding between variants (the summation order of the derivative rows
 * differs).  Applies to plans built afterwards (the variant is part of the
 * plan key).  Default 3 register digits, DPP (the fastest measured at 20 and
 * 30 photons); PQ_WALK=<digits>,<swizzle> in the environment sets it at
 * pq_create.  Out of range: PQ_EINVAL.
 */
int pq_walk_variant(pq_ctx* ctx, int register_digits, int swizzle);
int pq_autotune_enable(pq_ctx* ctx, int on);
int pq_autotune_last(pq_ctx* ctx, int32_t policy[3], double* best_ms, double* default_ms,
                     int32_t* candidates);

/*
 * pq_perm_grad -- vector-Jacobian product over a batch of patterns on one U:
 * the gradient of a cost built from transition amplitudes, which the paper
 * requires of circuit simulations used for machine learning (Goals: quantum
 * machine learning support and custom gradients in the Built-in simulators
 * section; Benchmarks / Fock-space based simulations: Differentiability,
 * one learning step of a photonic circuit's parameters).
 * perm(U_{T,S}) is a polynomial (holomorphic) in U; following the
 * conjugate-Wirtinger convention of complex autograd,
 *     dU = sum_p gperm[p] * conj( d perm(U_{T_p,S_p}) / dU ),
 * where d perm / d U_ij = t_i s_j perm(U_{T-e_i, S-e_j}) (the minor
 * permanents), computed inside the same Gray-code sweep as the forward value.
 *   S, T   host int32[batch*m], pattern p at offset p*m.
 *   gperm  device, batch complex.
 *   perm   device, batch complex, may be NULL: forward values of the sweep.
 *   dU     device, m x m, leading dimension lddu >= m; OVERWRITTEN
 *          (entries outside every pattern's support are set to 0).
 * Per pattern the compact matrix may have at most PQ_GRAD_MAX_DIM distinct
 * rows and columns; more than 24 distinct columns are supported only when
 * every occupation is 0 or 1 (collision-free patterns; PQ_ERANGE otherwise).
 * Calls that overlap on one ctx are not allowed (the ctx is not thread-safe).
 */
#define PQ_GRAD_MAX_DIM 32
int pq_perm_grad(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m,
                 int32_t batch, const int32_t* S, const int32_t* T,
                 const pq_c128* gperm, pq_c128* perm,
                 pq_c128* dU, int64_t lddu, void* stream);

/*
 * Passive-circuit simulation: every output amplitude of one input pattern
 * (the output probabilities of a linear interferometer, Eq. BS_prob / per_def
 * for every T; completeness sum_T |amp|^2 = 1 for unitary U).
 *
 * pq_perm_all_outputs -- perm(U_{T,S}) and amp = perm / sqrt(prod S! prod T!)
 * for every output pattern T with sum T = sum S = n on m modes, in ascending
 * lexicographic order of (T_0, ..., T_{m-1}): T = (0, ..., 0, n) first,
 * (n, 0, ..., 0) last; pq_fock_count(m, n) = C(n+m-1, n) outputs.  One
 * Gray-code sum over the input side serves every T: a term's m column sums
 * c_i = sum_j delta_j U[i][j] give w prod_i c_i^{t_i} for all T at once.
 *   U      device, m x m row-major, leading dimension ldu >= m.
 *   S      host int32[m] input occupations, sum n <= 48.
 *   perm   device, pq_fock_count(m, n) complex, written.
 *   amp    device, same size, may be NULL.
 * Limits (PQ_ERANGE): m <= 64; at most PQ_ALL_MAX_OUTPUTS outputs; at most
 * 2^20 Gray terms (prod over occupied input modes of (s_j + 1), halved on the
 * smallest).  n == 0 writes the single vacuum output perm = amp = 1.
 * Two forms compute the same sum (pq_all_outputs_gemm picks between them):
 *   - the sweep: one thread per output T, terms staged through LDS;
 *   - the contraction: with the output modes split into halves a and b,
 *     prod_i c_i^{t_i} = M_a(T_a) M_b(T_b) (the monomials of each half), so
 *     for each degree k = |T_a| the outputs are one complex matrix product
 *     over the terms of the weighted half-a monomials (one column per T_a of
 *     degree k) and the half-b monomials (one per T_b of degree n - k),
 *     computed by rocBLAS zgemm (the device's FP64 matrix cores; the blocks
 *     of different k side by side on four streams of the ctx; blocks with at
 *     most 8 compositions on one side by a kernel of their own).  Its tables
 *     (one complex per term and composition of at most n photons in either
 *     half) take workspace of up to 1 GiB, its products as much as the
 *     outputs.
 * The two forms agree to rounding (another order of the sum over terms).
 */
#define PQ_ALL_MAX_OUTPUTS (1ll << 31)
int pq_perm_all_outputs(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m, const int32_t* S,
                        pq_c128* perm, pq_c128* amp, void* stream);

/*
 * pq_all_outputs_gemm -- which form pq_perm_all_outputs takes:
 *   PQ_ALL_GEMM_AUTO (default): the contraction when its tables fit 1 GiB
 *     and outputs x terms >= 2^29 (below that its fixed cost, about 0.2 ms
 *     of launches, outweighs the sweep); the sweep otherwise;
 *   PQ_ALL_GEMM_ALWAYS: the contraction whenever its tables fit;
 *   PQ_ALL_GEMM_NEVER: the sweep.
 * PQ_ALL_GEMM=auto|always|never in the environment sets it at pq_create.
 * NULL ctx or another mode: PQ_EINVAL.
 */
enum { PQ_ALL_GEMM_AUTO = 0, PQ_ALL_GEMM_ALWAYS = 1, PQ_ALL_GEMM_NEVER = 2 };
int pq_all_outputs_gemm(pq_ctx* ctx, int mode);

/*
 * pq_sample_chain -- chain-rule boson sampling (Clifford & Clifford's
 * algorithm A, named in the Boson Sampling benchmark section), every sample's
 * whole draw sequence in one launch.  For sample s with input modes
 * order[s][0..n-1] (a random order of the input photons' modes: a mode with
 * s_j photons appears s_j times, so random Fock inputs with repeated modes
 * are allowed) and uniforms u = uniforms[s][0..n-1] in [0, 1), step k = 1..n
 * draws
 *     r_k = the first mode l whose cumulative weight (modes in ascending
 *           order) exceeds u_k times the total, with weights
 *           |perm(U_{r_1..r_{k-1}, l ; order[0..k-1]})|^2,
 * and writes out[s][k-1] = r_k.  Averaged over uniformly random orders and
 * uniforms, the multiset {r_k} follows the Born rule of Eq. BS_prob.
 *   U         device, m x m, leading dimension ldu >= m.
 *   order     device int32[samples * n], input modes in [0, m), repeats allowed.
 *   uniforms  device double[samples * n].
 *   out       device int32[samples * n], written.
 * Limits (PQ_ERANGE): m <= 1024, n <= 24 and n <= m.  The random numbers are
 * inputs, so a run replays exactly from its uniforms and orders.
 * The kernel checks every order entry: a sample with an entry outside
 * [0, m) reads no row of U through it, its draws are all written as -1, and
 * the call returns PQ_EINVAL.  To report that, the call waits for the
 * sampler to finish on `stream` before it returns (unlike the other entry
 * points, it is synchronous).
 */
int pq_sample_chain(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m, int32_t n, int32_t samples,
                    const int32_t* order, const double* uniforms, int32_t* out, void* stream);

/*
 * pq_loss_dilation -- lossy interferometers (the pure-loss channel of the
 * Boson Sampling section: mode i meets an inaccessible mode at a beamsplitter
 * with transmissivity eta_i, after the interferometer U; the beamsplitter is
 * the paper's [[t, -r*], [r, t]] on (i, m + i) with t = sqrt(eta_i),
 * r = sqrt(1 - eta_i)).  Writes the 2m x 2m unitary
 *     Ud = [[D U, -E], [E U, D]],  D = diag(sqrt(eta)), E = diag(sqrt(1 - eta)),
 * whose top-left block is the lossy transfer matrix A = D U (A A^dagger <= I).
 * Photons entering modes 0..m-1 and leaving through modes m..2m-1 are the
 * lost ones, so pq_sample_chain and pq_perm_all_outputs on Ud (inputs in
 * modes 0..m-1) sample and evaluate the lossy output distribution.
 *   U     device, m x m, leading dimension ldu >= m.
 *   eta   host double[m] in [0, 1] (PQ_EINVAL otherwise).
 *   Ud    device, 2m x 2m, leading dimension ldd >= 2m, written.
 */
int pq_loss_dilation(pq_ctx* ctx, const pq_c128* U, int64_t ldu, int32_t m, const double* eta, pq_c128* Ud,
                     int64_t ldd, void* stream);

/*
 * pq_loss_dilation_vw -- a general lossy interferometer in the singular value
 * form of the Boson Sampling section: A = V diag(mu) W with V, W unitary and
 * mu_i = sqrt(eta_i), eta_i in [0, 1] the transmission of the i-th singular
 * mode (A A^dagger <= I).  It is W, then a pure-loss beamsplitter on every
 * mode (as in pq_loss_dilation), then V on the system modes:
 *     Ud = (V (+) I) [[D, -E], [E, D]] (W (+) I) = [[V D W, -V E], [E W, D]],
 * a 2m x 2m unitary whose top-left block is A.  pq_sample_chain and
 * pq_perm_all_outputs on Ud (inputs in modes 0..m-1; outputs m..2m-1 are the
 * lost photons) sample and evaluate A's lossy output distribution.
 *   V, W   device, m x m, leading dimensions ldv, ldw >= m (unitarity is the
 *          caller's; the dilation is unitary exactly when V and W are).
 *   eta    host double[m] in [0, 1] (PQ_EINVAL otherwise).
 *   Ud     device, 2m x 2m, leading dimension ldd >= 2m, written.
 * With V = I it equals pq_loss_dilation(W, eta).
 */
int pq_loss_dilation_vw(pq_ctx* ctx, const pq_c128* V, int64_t ldv, const double* eta, const pq_c128* W,
                        int64_t ldw, int32_t m, pq_c128* Ud, int64_t ldd, void* stream);

/*
 * pq_lhaf -- loop hafnian with repeated modes (Appendix, Eq. loop_hafnian;
 * with gamma NULL the hafnian, Eq. haf_def), the matrix function of the
 * Gaussian Boson Sampling detection probability: lhaf(filldiag(A_r, gamma_r)),
 * where mode i is repeated reps[i] times, two copies of modes i < k are
 * joined by an edge of weight A[i][k], two copies of mode i by A[i][i], and
 * every copy of mode i carries a loop of weight gamma[i].  Only the upper
 * triangle (i <= k) of A is read.  Evaluated by a Glynn-type Gray-code sum
 * over vertex signs with repetition digits and halving (the Gaussian Boson
 * Sampling section), complex FP64, double-double reduction.
 *   A      device, d x d row-major, leading dimension lda >= d.
 *   gamma  device, d complex, or NULL (no loops: the hafnian).
 *   reps   host int32[d], >= 0; N = sum reps.
 *   out    device, 1 complex, written.
 * N == 0 writes 1; without loops an odd N writes 0.  Limits (PQ_ERANGE):
 * N <= 64, at most 48 modes with reps > 0, at most 32 of them beyond the
 * lane digits and the one register digit (for (2, ..., 2) repetitions: 37
 * modes), at most 2^52 time states.  Negative reps, NULL out/reps, or NULL A / lda < d with N > 0 give
 * PQ_EINVAL.
 */
int pq_lhaf(pq_ctx* ctx, const pq_c128* A, int64_t lda, int32_t d, const pq_c128* gamma,
            const int32_t* reps, pq_c128* out, void* stream);

/*
 * pq_lhaf_pack -- whether pq_lhaf fills idle lanes.  When the lane digits of
 * a sweep leave lanes of a wavefront idle (between 33 and 63 lane states,
 * e.g. 54 for (2, ..., 2) repetitions), the idle lanes can run lane states of
 * a second Gray segment of the same parity, so that nearly every lane does
 * useful work (378 of 384 lanes at 54 states).
 *   PQ_LHAF_PACK_AUTO (default): packed when the sweep fills every resident
 *     wavefront of the device without it (shorter sweeps gain nothing and
 *     pay the per-segment set-up);
 *   PQ_LHAF_PACK_ALWAYS / PQ_LHAF_PACK_NEVER: whenever the lane states allow
 *     it / never.
 * Results agree to rounding (the order of the partial sums differs).
 * PQ_LHAF_PACK=auto|always|never in the environment sets it at pq_create.
 * NULL ctx or another mode: PQ_EINVAL.
 */
enum { PQ_LHAF_PACK_AUTO = 0, PQ_LHAF_PACK_ALWAYS = 1, PQ_LHAF_PACK_NEVER = 2 };
int pq_lhaf_pack(pq_ctx* ctx, int mode);

/*
 * pq_lhaf_many -- pq_lhaf for npat repetition vectors on one matrix (the
 * probabilities of many output patterns of one Gaussian state), in one
 * submission: every pattern is planned on the host, its Gray range is cut
 * into chunks (four per workgroup, all of one pattern), one launch per
 * kernel variant sweeps them, and each pattern's chunk sums are added in
 * chunk order (results do not depend on timing).
 *   reps   host int32[npat * d], pattern q at offset q * d.
 *   out    device, npat complex, written (out[q] for pattern q).
 * Limits and errors as for pq_lhaf, per pattern; npat == 0 does nothing.
 */
int pq_lhaf_many(pq_ctx* ctx, const pq_c128* A, int64_t lda, int32_t d, const pq_c128* gamma,
                 const int32_t* reps, int32_t npat, pq_c128* out, void* stream);

/* Number of occupation vectors with n photons on m modes, C(n+m-1, n);
 * -1 for m < 1, n < 0, or a count above 2^62 (host, no GPU work). */
int64_t pq_fock_count(int32_t m, int32_t n);

/* T[0..m-1] = the occupation vector of rank `rank` in the order of
 * pq_perm_all_outputs (host).  PQ_EINVAL for a rank outside
 * [0, pq_fock_count(m, n)) or bad sizes, PQ_ERANGE when the count overflows. */
int pq_fock_unrank(int32_t m, int32_t n, int64_t rank, int32_t* T);

/*
 * Differentiable circuits (Beamsplitter gate section; differentiable
 * circuits in the simulator overview).
 *
 * pq_mesh_unitary -- U = B_ncell ... B_2 B_1 for cells acting on mode pairs
 * (modes[2q], modes[2q+1]) with the beamsplitter mode matrix
 * [[t, -r*], [r, t]], t = cos(theta_q), r = e^{i phi_q} sin(theta_q)
 * (row = output mode, column = input mode); cell q applies first when q is
 * smallest.  angles: device, 2*ncell doubles (theta_q, phi_q).  modes: host.
 * U: device m x m, leading dimension ldu.  1 <= m <= 32, ncell <= 512.
 *
 * pq_mesh_unitary_vjp -- gradient of a real loss with respect to the angles
 * given its gradient gU with respect to U in the conjugate-Wirtinger
 * convention of complex autograd (gU = dL/dRe U + i dL/dIm U):
 * gangles[2q] = dL/dtheta_q, gangles[2q+1] = dL/dphi_q (device, overwritten).
 */
int pq_mesh_unitary(pq_ctx* ctx, int32_t m, int32_t ncell, const int32_t* modes, const double* angles,
                    pq_c128* U, int64_t ldu, void* stream);
int pq_mesh_unitary_vjp(pq_ctx* ctx, int32_t m, int32_t ncell, const int32_t* modes, const double* angles,
                        const pq_c128* gU, int64_t ldg, double* gangles, void* stream);

/*
 * Sampling loss of a batch of output patterns (Eq. BS_prob):
 *   loss = -(1/batch) sum_p ( log |perm_p|^2 - log_norm_p ),
 * log_norm_p = log(prod S_p! prod T_p!) (device, may be NULL for zeros), so
 * that loss is the mean negative log-probability.  Fixed-order double-double
 * sum.  pq_neg_log_prob_vjp writes gperm_p = dloss/dperm_p in the same
 * convention as above, scaled by *gloss (device scalar, NULL for 1):
 * gperm_p = -(2/batch) gloss / conj(perm_p).
 */
int pq_neg_log_prob(pq_ctx* ctx, int32_t batch, const pq_c128* perm, const double* log_norm, double* loss,
                    void* stream);
int pq_neg_log_prob_vjp(pq_ctx* ctx, int32_t batch, const pq_c128* perm, const double* gloss, pq_c128* gperm,
                        void* stream);

/*
 * Sweep-kernel timing.  While enabled, every Gray-code sweep launch on ctx is
 * bracketed by HIP events recorded on the launch stream.  pq_profile_read
 * waits for the recorded events, returns the number of sweep launches and
 * their summed duration in milliseconds since the last read (or enable), and
 * clears the record.  Disabled by default; enabling costs two event records
 * per launch.
 */
int pq_profile_enable(pq_ctx* ctx, int on);
int pq_profile_read(pq_ctx* ctx, int64_t* launches, double* total_ms);

/*
 * Planning description (no GPU work; usable without a device).  Fills the
 * fields below for the problem (S, T) exactly as pq_perm would plan it.
 */
typedef struct {
    int32_t status;        /* PQ_OK, or the error pq_perm would return */
    int32_t n;             /* photons */
    int32_t trivial;       /* 1: sums differ (value 0), 2: n == 0 (value 1), else 0 */
    int32_t transposed;    /* 1: the Gray code runs over the input side S */
    int32_t rows, cols;    /* compact sizes (iterated side, power side) */
    int32_t fixed_row;     /* index (into the iterated modes, ascending) of the fixed group */
    int32_t lane_digits;   /* digits mapped onto the 64 lanes of a wavefront */
    int32_t lane_states;   /* product of their radices (<= 64) */
    int32_t time_digits;   /* digits swept in time */
    int32_t inner_digits;  /* time digits driven by the per-step table */
    int32_t inner_states;  /* product of the inner radices */
    int32_t binary;        /* 1: every digit binary and every power 1 */
    uint64_t terms;        /* Gray-code terms N = mu_f prod_{i != f} (mu_i + 1) */
    uint64_t time_states;  /* terms / lane_states (rounded up for padding lanes) */
    double log2_norm;      /* log2 of 1 / sqrt(prod S! prod T!) */
} pq_plan_info;

int pq_plan_describe(int32_t m, const int32_t* S, const int32_t* T, pq_plan_info* out);

/*
 * Reflected mixed-radix Gray code helper (host; exposed for tests).
 * Digits are listed least-significant first with radices radix[0..d-1] >= 1.
 * Writes the Gray digits of rank `rank` into digits[0..d-1].  Returns
 * PQ_EINVAL for bad arguments or rank >= prod radix.
 */
int pq_gray_unrank(int32_t d, const int32_t* radix, uint64_t rank, int32_t* digits);

#ifdef __cplusplus
}
#endif

#endif /* PQ_H */
