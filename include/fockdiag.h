/*
 * fockdiag.h -- C ABI of the MI355X (gfx950) library for the selective
 * Fock-amplitude recurrence of noisy Gaussian states (De Prins, Yao, Apte,
 * Miatto, "A Quadratic Speedup in the Optimization of Noisy Quantum Optical
 * Circuits", Quantum 2023).
 *
 * What is computed (Sec. 2.1 Eq. recrel, Sec. 3.1 probability p(n), Sec. 3.2):
 * for an M-mode state with Bargmann triple (A, b, c) -- A complex symmetric
 * 2M x 2M, b in C^2M, c in C -- the Fock amplitudes are the scaled Taylor
 * coefficients rho_k = d^k F(0)/sqrt(k!) of F(z) = c exp(1/2 z^T A z + b^T z).
 * For a set D of detected modes and U of undetected modes the library returns
 *
 *     rho[k_U..., l_U..., n_D...] = < k_U, n_D | rho | l_U, n_D >,
 *
 * i.e. every ket/bra block of the undetected modes and only the diagonal of
 * the detected modes, at O(M^2 prod_U C^2 prod_D C) cost (Algorithm 1 for
 * U empty, Algorithm 2 otherwise; Sec. 4 complexity).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Complex numbers are interleaved (re, im): complex128 = two doubles,
 *    complex64 = two floats, selected by the plan's dtype.
 *  - A is 2M x 2M, row-major, in BLOCK order [ket_1..ket_M, bra_1..bra_M]
 *    (the paper's block formulas, Sec. 2.1 Eqs. A_rho/b_rho, read ket-first:
 *    the returned amplitudes satisfy rho[k, l] = <k|rho|l>); b has length 2M
 *    in the same order; c is one complex scalar.  The library uses
 *    1/2 (A + A^T): the recurrence is route-independent only for symmetric A.
 *  - rho is C-contiguous with shape [C_u for u in U (kets)] + [C_u for u in U
 *    (bras)] + [C_j for j in D], U and D each in increasing mode order.
 *    With U empty it is the table of detection probabilities p(n).
 *  - All data pointers (A, b, c, rho, workspace, saved, gradients) are DEVICE
 *    pointers owned by the caller.  No call frees caller memory.  A plan owns
 *    its own small device tables, released by fd_plan_destroy.
 *  - Every call is asynchronous on the given stream.  Argument errors are
 *    detected on the host, return a status and set fd_last_error(); nothing
 *    is launched then.  Non-finite inputs or outputs detected on the device
 *    set the plan's device status word, read by fd_device_status().
 *  - A plan may be used by one host thread at a time; calls on one plan that
 *    overlap on different streams race on its device status word only.
 */
#ifndef FOCKDIAG_H
#define FOCKDIAG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FD_OK = 0,
  FD_ERR_INVALID_ARG = 1,   /* bad shape, mask, pointer or size             */
  FD_ERR_UNSUPPORTED = 2,   /* outside the compiled limits (see below)      */
  FD_ERR_WORKSPACE = 3,     /* workspace or saved buffer too small          */
  FD_ERR_OOM = 4,           /* the plan could not allocate its tables       */
  FD_ERR_HIP = 5,           /* a HIP runtime call failed                    */
  FD_ERR_NONFINITE = 6      /* device saw NaN/Inf (fd_device_status only)   */
} fd_status;

typedef enum { FD_C128 = 0, FD_C64 = 1 } fd_dtype;

/* Plan flags: how the displacement vector b is treated.
 * FD_B_AUTO    the forward call copies b to the host (one synchronising
 *              2M-element read) and takes the b = 0 schedule when b is
 *              exactly zero (Sec. 2.4: odd-weight amplitudes then vanish and
 *              pivots need not be read);
 * FD_B_ZERO    the caller promises b == 0 (the b = 0 schedule, no host read);
 *              a non-zero b is then reported through fd_device_status;
 * FD_B_GENERAL always the general schedule (no host read). */
enum { FD_B_AUTO = 0u, FD_B_ZERO = 1u, FD_B_GENERAL = 2u };

/* Compiled limits: M <= 16 modes, at most 8 detected modes with cutoff >= 2,
 * at most 3 undetected modes with cutoff >= 2, every cutoff in [1, 64],
 * prod over detected cutoffs < 2^31 (<= 2^22 when a mode is undetected: the
 * plan keeps a 96-byte record per detected lattice point), one level of the
 * detected lattice times the undetected block <= 2^28 amplitudes,
 * undetected block B = prod C_u^2 <= 65536.  A node's block rows are staged
 * in LDS (160 KiB per workgroup) where they fit; otherwise, per kernel, they
 * stream from HBM (the forward and reverse block units read the rows where
 * they lie and keep their computed rows in per-workgroup slots of the
 * workspace, the block fills work on the block in HBM), which
 * fd_plan_workspace accounts for.  The forward mode (fock_diag_jvp) does not
 * stream: its LDS rows hold values and tangents, and blocks beyond them give
 * FD_ERR_UNSUPPORTED there.  Modes with cutoff 1 carry no photons and are
 * dropped internally. */

typedef struct fd_plan_s* fd_plan;

/* fd_plan_create -- validate a problem shape and build its schedule tables
 * on the host (the level structure of Algorithms 1/2: the families
 * diag + offset of Sec. 3.1.4 / App. B.2 and their per-level sizes).
 *   M              number of modes, 1..16
 *   cutoffs        host array of M Fock cutoffs C_j (>= 1); detected modes
 *                  return n_j < C_j, undetected modes k, l < C_j
 *   detected_mask  bit j set = mode j carries a PNR detector
 *   dt             FD_C128 or FD_C64 for every complex buffer of this plan
 *   flags          FD_B_AUTO / FD_B_ZERO / FD_B_GENERAL
 *   out            receives the plan (host handle)
 * No device memory is touched here; device tables are created on first use. */
fd_status fd_plan_create(int M, const int* cutoffs, uint32_t detected_mask, fd_dtype dt,
                         uint32_t flags, fd_plan* out);
fd_status fd_plan_destroy(fd_plan p);

/* fd_plan_workspace -- byte sizes of the caller-owned device buffers.
 *   with_vjp = 0: *fwd_bytes = workspace of fock_diag_fwd with saved == NULL
 *                 (intermediates kept in a two-level ring, Sec. 3.1.4 buffer
 *                 strategy), *saved_bytes = 0.
 *   with_vjp = 1: *saved_bytes = size of the `saved` buffer that keeps every
 *                 intermediate amplitude for the reverse sweep, *fwd_bytes =
 *                 workspace of both fock_diag_fwd (with saved) and
 *                 fock_diag_vjp (with saved).  fock_diag_vjp with saved ==
 *                 NULL needs fwd_bytes + saved_bytes of workspace. */
fd_status fd_plan_workspace(fd_plan p, int with_vjp, size_t* fwd_bytes, size_t* saved_bytes);

/* fd_plan_set_checkpoint -- memory of the reverse sweep.  Sec. 2.5's
 * derivatives need, in reverse level order, the forward values of the two
 * levels a pivot reads; by default the saved buffer keeps every level of
 * every intermediate family.  With every = s >= 1 it keeps only F0 (every
 * level: it is the output) and, for each segment of s levels, the families
 * of the level just below it (the state the forward needs to restart there,
 * Sec. 3.1.4's two-level buffer); fock_diag_vjp then recomputes each
 * segment's intermediates from its checkpoint into a segment buffer of s + 1
 * levels in the workspace, walking the segments from the top.  Memory falls
 * from all levels to about L / s + s levels of intermediates (L levels;
 * s ~ sqrt(L) is the least); the forward work is done twice.  Results are
 * bitwise those of the store-all sweep (same kernels on the same values).
 * every = 0 restores store-all.  fd_plan_workspace(with_vjp = 1) reports the
 * sizes for the current setting; a saved buffer filled under one setting
 * must be used under the same one.  Drops the plan's captured graphs. */
fd_status fd_plan_set_checkpoint(fd_plan p, int every);

/* fd_plan_set_write_counters -- debug mode for the exactly-once writes of the
 * buffer strategy (Sec. 3.1.4; the stored counts of App. B.3).  counters: a
 * device array of n unsigned ints, caller-owned and caller-zeroed, n >= the
 * saved buffer's size in elements (saved_bytes / 16 for complex128, / 8 for
 * complex64).  While set, every fock_diag_fwd call WITH a saved buffer adds 1
 * to counters[k] for each amplitude its kernels write at element k of
 * `saved` (Eq. recrel writes: the undetected block fill and every level; the
 * seed G_0 = c is set by the prep and not counted).  A correct schedule leaves
 * every count at 0 or 1, and their sum equals fd_plan_query(FD_Q_TARGETS).
 * Calls without a saved buffer, the reverse sweep, the batched and
 * static-scratch calls and the forward mode count nothing.  counters = NULL
 * (n = 0) switches the mode off.  Costs a global atomic per write: for tests,
 * not for timing.  Errors: FD_ERR_INVALID_ARG (NULL plan, n too small, n != 0
 * with NULL), FD_ERR_UNSUPPORTED (a checkpointed plan: its saved buffer does
 * not hold every amplitude).  Drops the plan's captured graphs. */
fd_status fd_plan_set_write_counters(fd_plan p, unsigned int* counters, size_t n);

/* fd_plan_query -- integer facts about the plan (host only, for tests and
 * reports).  `what`: see FD_Q_* below. */
enum {
  FD_Q_OUT_ELEMS = 0,      /* elements of rho                                   */
  FD_Q_LEVELS = 1,         /* photon-number levels swept (sum_D (C_j - 1) + 1)  */
  FD_Q_PIVOTS = 2,         /* pivots of Algorithm 1 over the detected modes     */
  FD_Q_STORED_NODES = 3,   /* written amplitudes (nodes) per App. B.3 types     */
  FD_Q_TARGETS = 4,        /* computed amplitudes incl. U blocks (per call)     */
  FD_Q_READ_TERMS = 5,     /* A-terms summed over all computed amplitudes       */
  FD_Q_BLOCK = 6,          /* entries per node (prod_U C_u^2, 1 if U empty)     */
  FD_Q_NODES_F0 = 7,       /* detected diagonal nodes prod_D C_j                */
  FD_Q_NODES_F1 = 8,       /* type-1 offset nodes                               */
  FD_Q_NODES_F2 = 9,       /* type-2 offset nodes                               */
  FD_Q_NODES_F1010 = 10,   /* type-1010 offset nodes                            */
  FD_Q_NODES_F1001 = 11,   /* type-1001 offset nodes                            */
  FD_Q_B_SCHEDULE = 12     /* 1 if the plan will use the b = 0 schedule         */
};
fd_status fd_plan_query(fd_plan p, int what, int64_t* out);

/* fock_diag_fwd -- rho[k_U, l_U, n_D] (Algorithm 1 or 2, Sec. 3).
 *   A, b, c    device inputs as described above
 *   rho        device output, fd_plan_query(FD_Q_OUT_ELEMS) complex elements
 *   workspace  device scratch of at least ws_bytes >= fd_plan_workspace(...)
 *   saved      NULL, or a device buffer of saved_bytes that receives every
 *              intermediate amplitude for fock_diag_vjp
 *   stream     HIP stream; all work is enqueued on it. */
fd_status fock_diag_fwd(fd_plan p, const void* A, const void* b, const void* c, void* rho,
                        void* workspace, size_t ws_bytes, void* saved, size_t saved_bytes,
                        hipStream_t stream);

/* fock_diag_vjp -- reverse-mode derivative of fock_diag_fwd (Sec. 2.5,
 * Eqs. dL_dB and dL_dA, taken in reverse instead of the paper's forward
 * mode).  With g = drho (same layout as rho), the outputs are
 *     dA = sum_k g_k conj(d rho_k / d A),  db = sum_k g_k conj(d rho_k / d b),
 *     dc = sum_k g_k conj(d rho_k / d c),
 * A being used through 1/2 (A + A^T), so dA is symmetric; block order.
 *   saved     the buffer filled by fock_diag_fwd with the same (A, b, c), or
 *             NULL to recompute the forward inside the workspace
 *   drho      device cotangent, same shape and dtype as rho
 *   dA/db/dc  device outputs (2M x 2M, 2M, 1 complex elements)
 * The reduction over amplitudes is done in a fixed order: results are
 * bitwise reproducible for a given plan and device. */
fd_status fock_diag_vjp(fd_plan p, const void* A, const void* b, const void* c,
                        const void* saved, size_t saved_bytes, const void* drho,
                        void* dA, void* db, void* dc, void* workspace, size_t ws_bytes,
                        hipStream_t stream);

/* fock_diag_fwd_static -- fock_diag_fwd without a caller workspace and
 * without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The sweep's intermediates go to a library-owned static device
 * array of 64 MiB (one per device, held from module load until the process
 * ends); its address is resolved on the first call on each device
 * (hipGetSymbolAddress, no allocation: make that first call outside a graph
 * capture).  Same arguments and result as fock_diag_fwd with saved == NULL.
 *   - Errors (host side, nothing launched): FD_ERR_WORKSPACE if the sweep
 *     needs more than 64 MiB (fd_plan_workspace with with_vjp = 0 reports
 *     the need), FD_ERR_INVALID_ARG for NULL or misaligned pointers and for a
 *     plan whose device tables do not exist yet on the current device (make
 *     one fock_diag_fwd / detection_probs / fock_diag_vjp / fock_diag_jvp
 *     call with the plan there first).
 *   - b is never read on the host: the b = 0 schedule is taken only for
 *     plans created with FD_B_ZERO; FD_B_AUTO plans take the general
 *     schedule (same amplitudes).  No graph replay and no per-kernel timing.
 *   - Every call on one device shares that device's array, which keeps the
 *     last call's contents (the sweep writes every entry before reading it):
 *     calls that overlap in time on one device race and give wrong results;
 *     serialise them (one stream, or events). */
fd_status fock_diag_fwd_static(fd_plan p, const void* A, const void* b, const void* c, void* rho,
                               hipStream_t stream);

/* Forward mode (Sec. 2.5, the tangent recurrences summed along one
 * direction): rho and its directional derivative
 *     drho = sum_ij dA_ij d rho / d A_ij + sum_i db_i d rho / d b_i + dc d rho / d c
 * for any box plan (Algorithm 1, or Algorithm 2 with undetected modes: the
 * tangent is carried through the undetected-block fill and the block units)
 * and for total-cutoff plans (fd_plan_create_total; rho and drho then in
 * level order).  A is used through 1/2 (A + A^T), and so is dA.  Every kept
 * amplitude carries its tangent through the same reads and writes, so the
 * sweep reads and writes twice the forward's bytes.
 *   dA, db, dc  device direction (2M x 2M, 2M, 1 complex elements, block order)
 *   rho, drho   device outputs, FD_Q_OUT_ELEMS complex elements each
 *   workspace   256-byte aligned device scratch of at least
 *               fd_plan_jvp_workspace bytes (values, then tangents)
 * Returns FD_ERR_UNSUPPORTED for plans created with FD_B_ZERO (a non-zero db
 * reaches the odd levels, which that schedule skips) and for undetected
 * blocks whose values and tangents exceed the LDS staging (the block fill:
 * 2B elements; the block units: twice the forward's rows).  With fd_plan_use_graphs the sweep is captured once per
 * set of pointers and replayed, as for fock_diag_fwd. */
fd_status fd_plan_jvp_workspace(fd_plan p, size_t* bytes);
fd_status fock_diag_jvp(fd_plan p, const void* A, const void* b, const void* c, const void* dA,
                        const void* db, const void* dc, void* rho, void* drho, void* workspace,
                        size_t ws_bytes, hipStream_t stream);

/* detection_probs -- p(n) = rho_{n1 n1 ... nM nM} for every n < cutoffs
 * (Sec. 3.1, Algorithm 1): fock_diag_fwd for a plan whose detected_mask
 * covers every mode.  probs has prod_j C_j complex elements (imaginary parts
 * are rounding noise for physical states). */
fd_status detection_probs(fd_plan p, const void* A, const void* b, const void* c, void* probs,
                          void* workspace, size_t ws_bytes, hipStream_t stream);

/* Batched forward over n independent circuits, each with its own plan and
 * buffers (arrays of n host-side entries holding device pointers), in one
 * persistent sweep launch.  All pivots of one weight are independent
 * (Sec. 2.2) and circuits are independent of each other: step S of every
 * circuit is swept together, by a cooperative grid that fills the device and
 * takes (circuit, step, tile) work items from a per-step queue, with a grid
 * barrier between steps.  Launches: prep (+ undetected block fill), the
 * sweep, the output permutation.  A circuit whose levels average at least
 * 2048 wavefront-sized units fills the device by itself and runs its own
 * level launches first (as fock_diag_fwd), and so does a circuit the sweep
 * cannot stage (three undetected modes, or rows beyond its LDS); the
 * persistent sweep takes the rest.
 *   plans      n plans of one dtype, created on the current device
 *   workspace  per circuit, >= fd_plan_workspace(plan, 0) bytes, 256-byte
 *              aligned; the n workspaces must not overlap (FD_ERR_INVALID_ARG)
 *   rho        per circuit, as for fock_diag_fwd
 * Results equal fock_diag_fwd's bit for bit.  The library keeps the work-item
 * table, per-circuit descriptors and the sweep's control words of the last 8
 * (plan set, pointer set) combinations in device memory (freed with the
 * plans); two batched calls with the same plans and pointers must not overlap
 * in time.  A device without cooperative launches gives FD_ERR_UNSUPPORTED.  A
 * barrier wait that exceeds its bound (a few seconds) is reported by
 * fd_device_status of the first plan as FD_ERR_HIP. */
fd_status fock_diag_fwd_batch(int n, const fd_plan* plans, const void* const* A,
                              const void* const* b, const void* const* c, void* const* rho,
                              void* const* workspace, const size_t* ws_bytes, hipStream_t stream);

/* Batched reverse sweep: fock_diag_vjp for n circuits (arrays of n entries as
 * in fock_diag_fwd_batch; saved may be NULL, or hold NULL entries, to
 * recompute those circuits' forward values in their workspaces).  A reverse
 * sweep keeps every forward intermediate of its circuit (9.9 GB for a
 * 6-mode circuit with a 30-photon undetected mode and 8-photon detected
 * modes) and fills the device on its own, so the circuits run one after
 * another on `stream`; unlike the forward batch, circuits may share one
 * workspace (the calls are stream-ordered).  Results equal fock_diag_vjp's
 * bit for bit.  Stops at the first failing circuit and returns its status. */
fd_status fock_diag_vjp_batch(int n, const fd_plan* plans, const void* const* A, const void* const* b,
                              const void* const* c, const void* const* saved, const size_t* saved_bytes,
                              const void* const* drho, void* const* dA, void* const* db, void* const* dc,
                              void* const* workspace, const size_t* ws_bytes, hipStream_t stream);

/* Scheduling knobs of fock_diag_fwd_batch (process-wide; a schedule built
 * under other knobs is rebuilt on next use):
 *   min_block_units, min_point_units, items_per_wave
 *              every step of a circuit is cut into items of units /
 *              (items_per_wave x resident wavefronts) units, at least
 *              min_block_units (lattice point, row chunk) units (Algorithm 2)
 *              or min_point_units lattice points (Algorithm 1);
 *   fill_waves a circuit whose levels average at least fill_waves
 *              wavefront-sized units runs its own level launches instead of
 *              joining the persistent sweep;
 *   use_graph  1: the first call with a given (plan set, pointer set) is
 *              captured into a HIP graph on a private stream (nothing runs
 *              during capture) and later calls with the same plans, pointers
 *              and knobs replay it on the caller's stream (buffer contents
 *              may change between calls); the last 8 graphs are kept and
 *              freed with their plans.  fd_batch_get_tuning reads -1 if the
 *              runtime refused a capture (a cooperative launch, say): calls
 *              then run their launches directly.  Graphs are not used while
 *              a plan of the batch records kernel times.
 * Defaults {2, 64, 4, 2048, 0}; the package's autotuner picks them per batch
 * signature by timing.  Values below 1 (use_graph: other than 0 or 1) give
 * FD_ERR_INVALID_ARG. */
typedef struct {
  int32_t min_block_units;
  int32_t min_point_units;
  int32_t items_per_wave;
  int32_t fill_waves;
  int32_t use_graph;
} fd_batch_tuning;
fd_status fd_batch_set_tuning(const fd_batch_tuning* t);
fd_status fd_batch_get_tuning(fd_batch_tuning* t);

/* Graph replay (for callers that reuse their buffers): with enable != 0, the
 * first fock_diag_fwd / fock_diag_vjp call with a given set of pointers is
 * captured once into a HIP graph (on a private capture stream, nothing runs
 * during capture) and every call with the same pointers launches the
 * instantiated graph on the caller's stream: one launch instead of one per
 * photon-number level.  Contents of the buffers may change between calls.
 * At most 8 graphs are kept per plan (least recently used dropped); disabling
 * drops them.  Ignored while per-kernel timing is enabled. */
fd_status fd_plan_use_graphs(fd_plan p, int enable);

/* Per-kernel timing for reports: with bit k of kind_mask set, every launch of
 * kernel kind k made through this plan is bracketed by two HIP events on its
 * stream (fd_plan_timing also drops earlier records).  fd_plan_kernel_times
 * waits for the recorded events and returns the number of launches and their
 * summed duration in milliseconds, then drops the records.  Kinds:
 * 0 input prep, 1 undetected-block fill, 2 forward level sweep, 3 output
 * permutation, 4 cotangent permutation, 5 reverse level sweep, 6 reverse of
 * the undetected-block fill, 7 gradient reduction, 8 accumulator clear,
 * 9 batched prep, 10 batched persistent sweep, 11 batched output permutation
 * (batched kinds are recorded on the first plan of the batch). */
enum { FD_K_PREP = 0, FD_K_UFILL = 1, FD_K_FWD_LEVEL = 2, FD_K_OUT_PERM = 3, FD_K_PERM_IN = 4,
       FD_K_VJP_LEVEL = 5, FD_K_UFILL_VJP = 6, FD_K_VJP_FINAL = 7, FD_K_ZERO = 8,
       FD_K_BATCH_PREP = 9, FD_K_BATCH_SWEEP = 10, FD_K_BATCH_OUT = 11 };
fd_status fd_plan_timing(fd_plan p, uint32_t kind_mask);
fd_status fd_plan_kernel_times(fd_plan p, int kind, int64_t* launches, double* total_ms);

/* Message of the last host-side error on the calling thread ("" if none). */
const char* fd_last_error(void);

/* Reads and clears the plan's device status word (synchronises `stream`):
 * FD_OK, or FD_ERR_NONFINITE if a non-finite input or output was seen, or
 * FD_ERR_INVALID_ARG if a plan made with FD_B_ZERO received a non-zero b, or
 * FD_ERR_HIP if a batched sweep gave up waiting at a step barrier. */
fd_status fd_device_status(fd_plan p, hipStream_t stream);

/* ---- Total photon cutoff and probability-sum stopping -----------------
 * fd_plan_create_total -- a plan with every mode detected whose lattice is
 * cut by the total photon number (the global cutoff condition of Sec. 2.3,
 * Eq. global_boundary_conditions, with N_max = total_cutoff + 1): the points
 * n with n_j < C_j and |n| <= total_cutoff, i.e. the levels of Algorithm 1
 * up to total_cutoff, whose level sets are simplices.  fock_diag_fwd / detection_probs
 * on such a plan return p(n) in level order: level S = 0, 1, ... at
 * fd_plan_level_offsets[S], inside a level the points in lexicographic order
 * with the first mode slowest; FD_Q_OUT_ELEMS entries.  Per-mode cutoffs
 * still apply (pass total_cutoff + 1 for none).  Limits as fd_plan_create
 * except that the box product may exceed 2^31 (the points below the cutoff
 * may not).  fock_diag_vjp takes the cotangent in the same level order (after
 * fock_diag_fwd with `saved`); the batched forward returns
 * FD_ERR_UNSUPPORTED for these plans. */
fd_status fd_plan_create_total(int M, const int* cutoffs, int total_cutoff, fd_dtype dt, uint32_t flags,
                               fd_plan* out);

/* Host copy of the level offsets of a plan with every mode detected: offsets
 * has FD_Q_LEVELS + 1 entries (n must be at least that); level S holds the
 * points offsets[S] .. offsets[S+1]-1 of the level-ordered output of a
 * total-cutoff plan (and of the internal node order of any all-detected
 * plan). */
fd_status fd_plan_level_offsets(fd_plan p, int64_t* offsets, int n);

/* detection_probs_until -- detection_probs with probability-sum stopping
 * (the second cutoff condition of Sec. 2.3: stop once the probabilities of
 * the outcomes computed so far sum close enough to one): levels are swept in
 * blocks of 4; after
 * each block the masses sum_{|n| = S} p(n) are read back (this call
 * synchronises `stream` once per block) and the sweep ends at the first
 * level S* with sum_{S <= S*} mass(S) >= 1 - eps.  probs holds p(n) for
 * |n| <= S* and zero above; *levels_done = S* + 1 (FD_Q_LEVELS if the sum
 * stays below 1 - eps), *mass = the sum over the returned levels (host
 * pointers).  eps in [0, 1); plan with every mode detected and at least one
 * cutoff >= 2; workspace as for fock_diag_fwd without saved. */
fd_status detection_probs_until(fd_plan p, const void* A, const void* b, const void* c, void* probs, double eps,
                                int* levels_done, double* mass, void* workspace, size_t ws_bytes,
                                hipStream_t stream);

/* ---- Pure states: the state vector ------------------------------------
 * The Fock amplitudes psi[n] = <n|psi>, 0 <= n_j < C_j, of a pure Gaussian
 * state given by its Bargmann triple (A: M x M complex symmetric, b: M, c):
 * the generating-function recurrence of Sec. 2.1 with D = M indices (one per
 * mode), psi[n] = (b_i psi[n - 1_i] + sum_l sqrt(n_l - [l = i]) A_il
 * psi[n - 1_i - 1_l]) / sqrt(n_i) with i the first mode where n_i > 0, swept
 * level by level in the total photon number |n| (the pure-state case of
 * Sec. 2.2 and the conditional pure states of Sec. 3.2: a state vector's
 * conditional amplitudes are slices of psi).  With b = 0 every amplitude of
 * odd |n| vanishes (Sec. 2.4) and only even levels are computed.
 * Limits: at most 8 modes with cutoff >= 2 (modes with cutoff 1 carry no
 * photons and are dropped), every cutoff in [1, 64], prod C_j < 2^31, one
 * level <= 2^28 amplitudes. */
typedef struct fd_state_plan_s* fd_state_plan;

/* flags: FD_B_ZERO (b == 0 promised: odd levels are not computed, a non-zero
 * b is reported through fd_state_device_status), FD_B_GENERAL, or FD_B_AUTO
 * (each call reads the M entries of b on the host and takes the b = 0 sweep
 * when they are all exactly zero).  No device memory is touched here. */
fd_status fd_state_plan_create(int M, const int* cutoffs, fd_dtype dt, uint32_t flags, fd_state_plan* out);
fd_status fd_state_plan_destroy(fd_state_plan p);
/* Workspace bytes for fock_state_fwd (the amplitudes in level order plus A
 * and b of the kept modes); 256-byte aligned device memory. */
fd_status fd_state_plan_workspace(fd_state_plan p, size_t* bytes);

/* fock_state_fwd -- psi of the triple, stream-ordered on `stream`.
 *   A          device, M x M, row-major, complex of the plan's dtype
 *   b          device, M entries;  c  device, 1 entry
 *   psi        device output, prod_j C_j entries in C order over modes
 *              0..M-1 (the last mode fastest); written completely
 *   workspace  device, >= fd_state_plan_workspace bytes, 256-byte aligned;
 *              may be reused once the call has completed on the stream
 * Errors: FD_ERR_INVALID_ARG (NULL or misaligned pointer, plan made on
 * another device), FD_ERR_WORKSPACE, FD_ERR_HIP; non-finite inputs or
 * outputs and a non-zero b under FD_B_ZERO are reported by
 * fd_state_device_status. */
fd_status fock_state_fwd(fd_state_plan p, const void* A, const void* b, const void* c, void* psi,
                         void* workspace, size_t ws_bytes, hipStream_t stream);

/* fock_state_vjp -- reverse mode of fock_state_fwd: with g = dL/dpsi^* the
 * cotangent of psi (Sec. 2.5, Eqs. dL_dB and dL_dA: the returned values are
 * sum_k g_k conj(d psi_k / d x)), writes dA (M x M, symmetric: A enters as
 * its symmetric part (A + A^T)/2), db (M) and dc (1).  The local gradients
 * are the closed-form solutions of the tangent recurrences of Sec. 2.5:
 * d psi_k/d b_i = sqrt(k_i) psi_{k-1_i}, d psi_k/d A_il = 1/2 sqrt(k_i (k_l -
 * [i = l])) psi_{k-1_i-1_l}, d psi_k/d c = psi_k / c, so the cotangents are
 * dot products of g with shifted copies of psi over the box (entries of modes
 * with cutoff 1 are zero).  Deterministic (fixed reduction order).
 *   psi        device, the output of fock_state_fwd for the same (A, b, c)
 *   dpsi       device, g in psi's layout
 *   c          device, the c of the forward call (dc = sum g conj(psi) / conj(c))
 *   workspace  device, >= fd_state_plan_vjp_workspace bytes, 256-byte aligned
 * Errors as fock_state_fwd. */
fd_status fd_state_plan_vjp_workspace(fd_state_plan p, size_t* bytes);
fd_status fock_state_vjp(fd_state_plan p, const void* c, const void* psi, const void* dpsi, void* dA, void* db,
                         void* dc, void* workspace, size_t ws_bytes, hipStream_t stream);

/* fock_state_jvp -- forward mode of fock_state_fwd: the tangent dpsi of psi
 * along a direction (dA: M x M, db: M, dc: 1) of the triple, from the same
 * closed forms (the tangent recurrences of Sec. 2.5 solved: dpsi_k = dc/c
 * psi_k + sum_i db_i sqrt(k_i) psi_{k-1_i} + sum_{i,l} dA_il 1/2
 * sqrt(k_i (k_l - [i = l])) psi_{k-1_i-1_l}; A enters as its symmetric part,
 * so only the symmetric part of dA matters).  One pass over the box, no
 * workspace; psi and c as for fock_state_vjp, dpsi in psi's layout.  With
 * fock_state_vjp it satisfies <g, J t> = <J^H g, t>.  Errors as
 * fock_state_fwd. */
fd_status fock_state_jvp(fd_state_plan p, const void* c, const void* psi, const void* dA, const void* db,
                         const void* dc, void* dpsi, hipStream_t stream);

/* As fd_device_status, for a state plan. */
fd_status fd_state_device_status(fd_state_plan p, hipStream_t stream);
/* As fd_plan_timing / fd_plan_kernel_times; kinds FD_K_PREP (A, b, c
 * staging), FD_K_FWD_LEVEL (one launch per computed level), FD_K_OUT_PERM,
 * FD_K_VJP_LEVEL (the cotangent dot products of fock_state_vjp, all their
 * launches as one record), FD_K_VJP_FINAL, and FD_K_FWD_LEVEL for the one
 * launch of fock_state_jvp. */
fd_status fd_state_plan_timing(fd_state_plan p, uint32_t kind_mask);
fd_status fd_state_plan_kernel_times(fd_state_plan p, int kind, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* FOCKDIAG_H */
