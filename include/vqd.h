/*
 * vqd.h -- C ABI of the MI355X (gfx950) density-matrix emulation library.
 *
 * The library applies gates and Kraus channels to an N-qubit density matrix
 * held in GPU memory and reads results out of it.  It is the data-parallel
 * core of the noisy-device emulation described in "The Virtual Quantum Device
 * (VQD)" (Gustiani, Jones, Benjamin): Sec. 2 chooses the density-matrix
 * representation with general Kraus operators; Sec. 3 defines the channels.
 *
 * Conventions shared by every call
 * --------------------------------
 * State layout.  rho is stored VECTORISED as 4^n complex128 values
 *   amp[r + 2^n c] = rho[r][c]       (interleaved re, im; FP64)
 * so qubit q of the register is vector bit q (row) and vector bit q + n
 * (column).  Because vec(U rho U^dagger) = (conj(U) (x) U) vec(rho), a gate U
 * on qubit q acts as U on bit q and conj(U) on bit q + n.
 *
 * Matrices.  All matrices are host pointers to row-major complex arrays of
 * interleaved (re, im) doubles, read during the call (the caller may free
 * them on return).  For a k-qubit op on targets t[0..k-1] the matrix index
 * is sum_j b(t[j]) 2^j: t[0] is the least significant bit.  A superoperator
 * acts on the 2k vector bits (t, t + n) with local index
 *   sum_j b(t[j]) 2^j  +  2^k sum_j b(t[j] + n) 2^j,
 * i.e. row bits first.  Built from Kraus operators K_j it is
 *   S = sum_j conj(K_j) (x) K_j     (S[(r',c'),(r,c)] = sum_j K_j[r'][r] conj(K_j[c'][c])).
 * Trace preservation is never checked: trace-decreasing (CPTN) maps such as
 * the leakage maps of Sec. 6 are legal.
 *
 * Memory.  The caller owns the device buffer of the state (for example a
 * torch tensor); the library never frees it, and a handle must not outlive
 * it.  The library owns small internal buffers (operation descriptors,
 * reduction partials), freed by the matching destroy call.
 *
 * Streams.  Apply and init calls are asynchronous on the handle's HIP stream.
 * vqd_calc_* calls synchronise that stream and write host outputs; their
 * vqd_calc_*_dev forms are asynchronous, write device outputs and allocate
 * nothing, so that init, a program and its read-outs can be captured in one
 * HIP graph.
 *
 * Errors.  Every call returns 0 (VQD_OK) or a negative code; the message of
 * the last failure on the calling thread is returned by vqd_last_error().  No
 * exception crosses the ABI.  On an error nothing has been enqueued.
 */
#ifndef VQD_H
#define VQD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VQD_OK        0
#define VQD_E_ARG    (-1)   /* bad qubit index, duplicate targets, null pointer, non-finite entry */
#define VQD_E_SIZE   (-2)   /* n out of range, buffer too small, k too large */
#define VQD_E_NOMEM  (-3)   /* an internal allocation failed */
#define VQD_E_HIP    (-4)   /* a HIP runtime call failed */
#define VQD_E_STATE  (-5)   /* call out of order (e.g. running an uncompiled program) */

#define VQD_MAX_QUBITS 16   /* 4^16 amplitudes = 64 GiB of complex128 */

typedef struct vqd_dm vqd_dm;
typedef struct vqd_prog vqd_prog;

/* Message of the last failed call on this thread ("" if none). */
const char *vqd_last_error(void);

/* Library version string. */
const char *vqd_version(void);

/* ------------------------------------------------------------------ state */

/* Wrap a caller-owned device buffer of `bytes` bytes holding 4^n complex128
 * amplitudes (n in [1, 16]) and a hipStream_t (NULL = default stream).
 * VQD_E_SIZE if bytes < 16 * 4^n.  The buffer is not modified. */
int vqd_dm_wrap(void *dev_amps, int n, size_t bytes, void *hip_stream, vqd_dm **out);

/* Release the handle and its internal buffers (not the wrapped buffer).
 * Synchronises the stream first.  NULL is accepted. */
int vqd_dm_destroy(vqd_dm *dm);

/* Change the stream later calls are enqueued on. */
int vqd_dm_set_stream(vqd_dm *dm, void *hip_stream);

/* |0..0><0..0|: one write pass over the buffer (Sec. 2 initial register). */
int vqd_dm_init_zero(vqd_dm *dm);

/* |b><b| for a computational basis state b < 2^n. */
int vqd_dm_init_basis(vqd_dm *dm, uint64_t b);

/* Product of single-qubit diagonal states (x)_j (p0[j]|0><0| + (1-p0[j])|1><1|),
 * the thermal initial state of the superconducting model (eq. thermalstate,
 * Sec. 8).  p0[j] is the ground-state population of qubit j (host array of n). */
int vqd_dm_init_product_diag(vqd_dm *dm, const double *p0);

/* Copy the 4^n amplitudes to / from a host array of 2 * 4^n doubles in the
 * vectorised order.  Synchronous.  Used as checkpoint and by tests. */
int vqd_dm_copy_to_host(const vqd_dm *dm, double *host);
int vqd_dm_copy_from_host(vqd_dm *dm, const double *host);

/* --------------------------------------------------------------- apply ops */

/* rho <- U rho U^dagger for a 2x2 U (8 doubles) on qubit q: U on vector bit q,
 * conj(U) on bit q + n, in one pass (Sec. 2; gates of Secs. 4-8). */
int vqd_apply_unitary1(vqd_dm *dm, int q, const double *u);

/* Same for a 4x4 U (32 doubles) on (q0, q1), q0 the low bit of U's index. */
int vqd_apply_unitary2(vqd_dm *dm, int q0, int q1, const double *u);

/* rho <- S(rho) for a single-qubit channel given as its 4x4 superoperator
 * (32 doubles) on the vector bits (q, q + n) -- e.g. the channels of eqs.
 * depol1, deph1, damp, gdamp, bf, depht2, ampt1 (Sec. 3). */
int vqd_apply_superop1(vqd_dm *dm, int q, const double *s);

/* Two-qubit channel as a 16x16 superoperator (512 doubles) on
 * (q0, q1, q0 + n, q1 + n) -- eqs. depol2, deph2, bf2, czleak and the
 * silicon parity-decay map (Secs. 3, 6, 7). */
int vqd_apply_superop2(vqd_dm *dm, int q0, int q1, const double *s);

/* A fused k-qubit block.  kind VQD_BLOCK_UNITARY: m is a 2^k x 2^k matrix U,
 * applied as U on the row bits and conj(U) on the column bits, k in [1, 4].
 * kind VQD_BLOCK_SUPEROP: m is a 4^k x 4^k superoperator, k in [1, 2].
 * Fusing a run of gates and channels on the same qubits into one block is
 * exact: the block is the product of the ops' superoperators (for channels,
 * the paper's own composition E(p,q) = deph o depol of eq. stderr, Sec. 3.2). */
#define VQD_BLOCK_UNITARY 0
#define VQD_BLOCK_SUPEROP 1
int vqd_apply_fused(vqd_dm *dm, int k, const int *targets, int kind, const double *m);

/* An element-wise (diagonal) superoperator on k <= 2 qubits: amp[i] is
 * multiplied by d[idx(i)], idx the local superoperator index of i (4^k
 * complex factors, 2 * 4^k doubles).  Covers the diagonal gates and channels
 * (Rz, CZ, CPh, ZZ crosstalk eq. weak_dephasing_zz, dephasing eq. deph1/2). */
int vqd_apply_diagonal(vqd_dm *dm, int k, const int *targets, const double *d);

/* ----------------------------------------------------- op programs (fusion) */

/* Named ops, parameters in the order listed (angles in radians, times in the
 * same unit as T1/T2). */
enum vqd_kind {
    VQD_K_RX = 1,       /* theta: exp(-i theta X / 2)                         */
    VQD_K_RY,           /* theta: exp(-i theta Y / 2)                         */
    VQD_K_RZ,           /* theta: exp(-i theta Z / 2)                         */
    VQD_K_H,            /* Hadamard                                           */
    VQD_K_X, VQD_K_Y, VQD_K_Z,
    VQD_K_SU2,          /* g0..g3: a0 I - i(a1 X + a2 Y + a3 Z), a = g/|g|    */
    VQD_K_CZ,           /* diag(1,1,1,-1)                                     */
    VQD_K_CPHASE,       /* theta: diag(1,1,1,e^{i theta})                     */
    VQD_K_XX,           /* theta: exp(-i theta/2 X(x)X)                       */
    VQD_K_ZZ,           /* alpha: exp(-i alpha Z(x)Z)  (eq. weak_dephasing_zz)*/
    VQD_K_DEPOL1,       /* p   (eq. depol1)                                   */
    VQD_K_DEPOL2,       /* p   (eq. depol2)                                   */
    VQD_K_DEPH1,        /* p   (eq. deph1)                                    */
    VQD_K_DEPH2,        /* p   (eq. deph2)                                    */
    VQD_K_AMP,          /* p   (eq. damp)                                     */
    VQD_K_GAMP,         /* p, gamma (eq. gdamp)                               */
    VQD_K_BITFLIP1,     /* b   (eq. bf)                                       */
    VQD_K_BITFLIP2,     /* b   (eq. bf2)                                      */
    VQD_K_AMP_T1,       /* dt, T1: amp(1 - exp(-dt/T1))          (eq. ampt1)  */
    VQD_K_DEPH_T2,      /* dt, T2: deph((1 - exp(-dt/T2)) / 2)   (eq. depht2) */
    VQD_K_DEPH_T2S,     /* dt, T2*: deph((1 - exp(-(dt/T2*)^2)) / 2) (eq. depht2s) */
    VQD_K_DEPOL_T1,     /* dt, T1: depol1(3/4 (1 - exp(-dt/T1)))  (eq. depolt1) */
    VQD_K_GAMP_T1,      /* p, dt, T1: gamp(p, 1 - exp(-dt/T1)), T1 relaxation
                           towards p|0><0| + (1-p)|1><1|      (eq. gdamp)     */
    VQD_K_RABI,         /* Omega, phi, Delta, t: the driven two-level unitary
                           U(phi, Delta, t) of Rabi frequency Omega (eq. u)   */
    VQD_K_OFFRES,       /* Omega, Delta, t: the drive a bystander qubit detuned
                           by Delta receives while a neighbour is driven at
                           Rabi frequency Omega for t (eq. off_resonant)      */
    VQD_K_CRZ,          /* alpha: |0><0| (x) I + |1><1| (x) Rz(alpha), control
                           targets[0] (eq. weak_dephasing)                    */
    VQD_K_PARITY_DECAY, /* no parameters: the decay |0 1> -> |1 0> (ket |a b>,
                           a on targets[0]) that accompanies the silicon parity
                           read-out, Kraus set {|00><00|, |11><11|, |10><10|,
                           |10><01|} (Sec. 7, eq. projmeas)                   */
    VQD_K_COUNT
};

/* Number of qubits and parameters of a named kind (-1 for an unknown kind). */
int vqd_kind_arity(int kind, int *n_qubits, int *n_params);

/* Build the matrix of a named gate (2^k x 2^k, interleaved complex) or the
 * superoperator of a named gate or channel (4^k x 4^k).  `out` must hold
 * 2 * 4^k (matrix) or 2 * 16^k (superop) doubles. */
int vqd_kind_matrix(int kind, const double *params, double *out);
int vqd_kind_superop(int kind, const double *params, double *out);

/* Error parameters from reported gate fidelities (App. B).  Entanglement
 * fidelity of depolarising p_depol followed by dephasing p_deph on an
 * nq-qubit gate (nq = 1: eq. fe1, 1 - p - q + 4/3 p q; nq = 2: 1 - p - q +
 * 16/15 p q).  vqd_fidelity_to_errors splits a reported average fidelity
 * fbar (converted by eq. fidelities_relation, F_e = ((d+1) fbar - 1)/d) into
 * p_depol = x eps and p_deph = (1 - x) eps, x in [0, 1] the depolarising
 * share, eps the smaller root in [0, 1]; VQD_E_ARG if there is none.
 * vqd_angle_scaled_error: eps |theta| / pi (App. C, rotation-angle scaling).
 * vqd_zz_crosstalk_strength: the static ZZ coupling of two transmons (Sec.
 * 8), beta = J^2 (1/(delta_ct - alpha_t) - 1/(delta_ct + alpha_c)) from the
 * coupling strength J, the frequency difference delta_ct = f_c - f_t and
 * the anharmonicities alpha_c, alpha_t, all in one frequency unit; the
 * result is in that unit.  VQD_E_ARG for a non-finite input or a zero
 * denominator. */
int vqd_entanglement_fidelity(int nq, double p_depol, double p_deph, double *fe);
int vqd_fidelity_to_errors(int nq, double fbar, double x, double *p_depol, double *p_deph);
double vqd_angle_scaled_error(double eps, double theta);
int vqd_zz_crosstalk_strength(double J, double delta_ct, double alpha_c, double alpha_t, double *beta);

/* Superoperator of a Kraus set: nk matrices of 2^k x 2^k, k in [1, 2]. */
int vqd_kraus_to_superop(int k, int nk, const double *kraus, double *out);

/* An op program: an ordered list of ops on an n-qubit register that the
 * library plans into fused passes.  A pass streams the state through HBM
 * once: a tile of 2^L amplitudes (L <= 13) is staged in registers and LDS and
 * every op of the pass is applied in-tile before the tile is written back.
 * The planner groups ops whose qubits fit one tile, fuses consecutive ops on
 * the same qubits into one block where that costs fewer flops, and applies
 * diagonal ops element-wise wherever their dependencies allow. */
int vqd_prog_create(int n, vqd_prog **out);
int vqd_prog_destroy(vqd_prog *p);
int vqd_prog_add_named(vqd_prog *p, int kind, const int *targets, const double *params);
/* count named ops at once: kinds[i], targets[4*i .. 4*i+arity), params[4*i ..]. */
int vqd_prog_add_named_many(vqd_prog *p, int count, const int *kinds, const int *targets,
                            const double *params);
int vqd_prog_add_unitary(vqd_prog *p, int k, const int *targets, const double *u);
int vqd_prog_add_superop(vqd_prog *p, int k, const int *targets, const double *s);
int vqd_prog_add_kraus(vqd_prog *p, int k, const int *targets, int nk, const double *kraus);

/* Planner options.  max_ops_per_pass = 1 disables fusion (one op per pass);
 * tile_bits in [4, 13] (a tile of 2^tile_bits amplitudes is one workgroup of
 * 2^(tile_bits-4) threads, staged through 16 * 2^tile_bits bytes of LDS);
 * min_contig_bits: low vector bits every tile keeps for coalesced access
 * (0..tile_bits). */
typedef struct vqd_plan_opts {
    int tile_bits;          /* default 13 */
    int min_contig_bits;    /* default 3  */
    int max_ops_per_pass;   /* default 0 = unlimited */
    int fuse_blocks;        /* default 1: multiply runs of ops into one block when cheaper */
    int pad_coalesce;       /* default 1: in passes with little FP64 work, add an op-free
                               first/last phase when the first/last register bits would
                               make HBM access strided */
    int hermitian;          /* default 0.  1: the caller's state is Hermitian (a density
                               matrix, Sec. 2); if every op of the program also maps
                               Hermitian matrices to Hermitian ones (every Kraus map and
                               unitary does), each pass computes only the tiles whose row
                               part of the index is at most its column part and writes the
                               conjugate transpose of each to its mirror image: about half
                               the work.  The tiles are then whole qubits (tile_bits is
                               rounded down to even) and always hold qubits
                               0..min(min_contig_bits, 3)-1 (fewer if the widest gate
                               would not fit), whose row and column bits give the
                               loads and stores their contiguous runs.  Between the
                               passes of a run only the computed half is current; the
                               last pass restores the whole matrix.  Otherwise the
                               program is planned as with 0.  Batches default to 1
                               (every instance starts from |0..0><0..0|). */
    int relayout;           /* default 0.  1 (Hermitian-mode programs only): between two
                               passes the state is stored under a relabelling of the
                               qubits that puts qubits shared by both passes' tiles
                               at the lowest positions, so that the loads and stores
                               of both passes move longer contiguous runs.  A pass
                               that changes the labelling writes into a second
                               state-sized buffer, which the density-matrix handle
                               allocates on the first run of such a program and
                               keeps until it is destroyed (16 * 4^n bytes; not
                               under stream capture).  The program always ends in
                               the caller's buffer under the original labelling.
                               Batches ignore it. */
} vqd_plan_opts;
void vqd_plan_opts_default(vqd_plan_opts *o);

/* Plan the program and upload its descriptors to the current device.
 * opts may be NULL (defaults).  May be called again to re-plan. */
int vqd_prog_compile(vqd_prog *p, const vqd_plan_opts *opts);

/* Plan the program on the host only (no device memory touched). */
int vqd_prog_plan(vqd_prog *p, const vqd_plan_opts *opts);

/* Export the planned descriptors for inspection by tools and tests.  Layout:
 * 12 uint32 header {magic 0x56514450, version 1, n_passes, n_phases,
 * n_kernel_ops, n_mats, sizeof pass, sizeof phase, sizeof op, n, tile
 * bits, 0} followed by the pass, phase and op records and n_mats complex
 * doubles.  The record layouts are internal to this library version.
 * With buf NULL or cap too small only *needed is written (and 0 returned
 * when buf is NULL; VQD_E_SIZE otherwise). */
int vqd_prog_export(const vqd_prog *p, void *buf, size_t cap, size_t *needed);

/* Enqueue all passes of a compiled program on dm's stream (dm->n == p->n). */
int vqd_prog_run(vqd_prog *p, vqd_dm *dm);

typedef struct vqd_prog_info {
    int n;
    int n_ops;              /* ops added                                   */
    int n_passes;           /* HBM passes after planning                   */
    int n_phases;           /* register phases over all passes             */
    int n_kernel_ops;       /* ops applied in-tile after block fusion      */
    double fma_per_amp;     /* planned FP64 FMAs per computed amplitude, all passes */
    int hermitian;          /* 1 if planned in Hermitian mode              */
    double tile_fraction;   /* share of the 4^n amplitudes each pass computes (1, or
                               (N+1)/(2N) in Hermitian mode with N = 2^(n - tile qubits)) */
    int relabelled;         /* 1 if the passes store the state between them under
                               qubit relabellings (vqd_plan_opts.relayout)          */
    int layout_changes;     /* passes that store into the second state buffer (even) */
} vqd_prog_info;
int vqd_prog_info_get(const vqd_prog *p, vqd_prog_info *out);

/* ----------------------------------------------------------------- batched */

/* A batch of independent density matrices of uneven size (n in [2, 16]),
 * each with its own op program, run by ONE persistent kernel launch.  Each
 * workgroup takes the next instance from a largest-first queue, sets it to
 * |0..0><0..0|, applies all of its planned passes tile by tile (tiles of at
 * most 2^12 amplitudes), and writes <Z_i>, i < n, of the final state.  This is
 * the many-small-density-matrix use of the emulator: the same circuit family
 * evaluated under many device variants (Sec. 4: repeated runs across
 * parameter choices; Sec. 8: parameter sweeps).
 *
 * Memory: the caller owns the arena (device memory holding every final
 * state; instance i's 4^n complex128 amplitudes start at the byte offset
 * vqd_batch_offsets() reports, 256-byte aligned) and the output buffer
 * (device doubles, n per instance).  The library owns the plan image, the
 * queue and its counter.  Calls that run must not overlap on one batch. */
typedef struct vqd_batch vqd_batch;

typedef struct vqd_batch_info {
    int n_instances;
    long long total_passes;   /* passes over all instances      */
    size_t arena_bytes;       /* arena size vqd_batch_run needs  */
    size_t n_outputs;         /* sum of the instances' n         */
    unsigned grid_items;      /* queue length                    */
    double fp64_fma;          /* FP64 FMAs one run executes: each instance's
                                 planned FMAs per computed amplitude times its
                                 computed amplitudes, summed               */
    double pass_bytes;        /* algorithmic HBM bytes of one run: per
                                 instance the initial state written (16 B per
                                 amplitude), every computed amplitude read and
                                 written once per pass (32 B), the last
                                 pass's mirror images and the diagonal read
                                 for <Z_i>, summed                          */
} vqd_batch_info;

int vqd_batch_create(vqd_batch **out);
int vqd_batch_destroy(vqd_batch *b);

/* Append a copy of program p's ops as a new instance (its index in *index). */
int vqd_batch_add(vqd_batch *b, const vqd_prog *p, int *index);

/* Plan options for every instance with n qubits (tile_bits in [4, 12]).
 * The defaults are tile_bits min(12, 2n), min_contig_bits 1, hermitian 1;
 * vqd_batch_plan_opts reports the options in use (set, autotuned or
 * default). */
int vqd_batch_set_opts(vqd_batch *b, int n, const vqd_plan_opts *opts);
int vqd_batch_plan_opts(const vqd_batch *b, int n, vqd_plan_opts *opts);

/* Plan all instances (host threads), lay out arena and outputs, upload the
 * plan image to the current device.  Reports the sizes the run needs. */
int vqd_batch_compile(vqd_batch *b, size_t *arena_bytes, size_t *n_outputs);

/* Where instance `index` lives in the arena and in the outputs. */
int vqd_batch_offsets(const vqd_batch *b, int index, size_t *arena_offset_bytes, size_t *out_offset);

/* Parametric templates: many instances of one circuit structure that differ
 * only in their parameters (rotation angles, noise rates), as in a sweep over
 * ansatz angles and device noise (Sec. 2 and 3: one noisy ansatz evaluated for
 * many parameter and noise settings).  The structure is planned once, with
 * generic parameters; each instance gets only its own coefficient block.
 *
 * vqd_batch_add_template: `count` ops of named kinds (enum vqd_kind) on
 * `targets` (4 ints per op, the first arity(kind) used) of an n-qubit state
 * (2 <= n <= 16).  Writes its id to *template_id.  Nothing is planned yet.
 *
 * vqd_batch_add_instances: `count` instances of template `template_id`;
 * params holds count x n_ops x 4 doubles (host, copied; per op the first
 * arity(kind) parameters are used, the rest ignored).  Instance indices (for
 * vqd_batch_offsets) count every vqd_batch_add and every template instance in
 * the order added; the first of these `count` is written to *first_index.
 * All or nothing: a non-finite parameter adds none.  Each instance starts
 * from |0..0><0..0| and yields its <Z_i> like any other.
 *
 * vqd_batch_compile then checks every instance against the planned form:
 * parameters under which a coefficient that the generic plan found zero (or
 * real) is not, fail with VQD_E_ARG naming the instance. */
int vqd_batch_add_template(vqd_batch *b, int n, int count, const int *kinds, const int *targets,
                           int *template_id);
int vqd_batch_add_instances(vqd_batch *b, int template_id, int count, const double *params, int *first_index);

/* Plan a template on the host (as vqd_batch_compile does, without a GPU) and
 * serialise it in the layout of vqd_prog_export, with the coefficients for
 * `params` (n_ops x 4 doubles; NULL keeps the generic planning parameters).
 * buf == NULL: only *needed is set. */
int vqd_template_export(int n, int count, const int *kinds, const int *targets, const double *params,
                        const vqd_plan_opts *opts, void *buf, size_t cap, size_t *needed);

/* Enqueue the batched run on hip_stream.  use_graph != 0 captures the launch
 * (queue reset kernel + persistent kernel) into a HIP graph on first use and
 * replays it (on a library stream ordered after and before hip_stream by
 * events) while arena and out stay the same. */
int vqd_batch_run(vqd_batch *b, void *arena, size_t arena_bytes, double *out, void *hip_stream,
                  int use_graph);

/* Autotuner: for every qubit count in the batch, time candidate tile shapes
 * (tile bits, contiguous low bits) on up to max_per_n instances of that
 * count using the caller's arena and outputs, keep the fastest, and record
 * it in the JSON file cache_path (read first; entries found there are used
 * without timing).  Synchronous.  The batch must be compiled again after. */
int vqd_batch_autotune(vqd_batch *b, void *arena, size_t arena_bytes, double *out, void *hip_stream,
                       const char *cache_path, int max_per_n);

int vqd_batch_info_get(const vqd_batch *b, vqd_batch_info *out);

/* ---------------------------------------------------------------- read-out */

/* Tr rho (complex). */
int vqd_calc_trace(const vqd_dm *dm, double *re, double *im);

/* Tr rho^2 = sum_i |amp_i|^2 (Hermitian rho). */
int vqd_calc_purity(const vqd_dm *dm, double *out);

/* p_r = Re rho[r][r], r < 2^n; not clamped or renormalised (host array 2^n). */
int vqd_calc_probs(const vqd_dm *dm, double *out);

/* <Z_i> = sum_r (-1)^{r_i} p_r for i < n (host array n). */
int vqd_calc_expec_z(const vqd_dm *dm, double *out);

/* <Z_i Z_j> for npairs pairs given as 2*npairs qubit indices. */
int vqd_calc_expec_zz(const vqd_dm *dm, const int *pairs, int npairs, double *out);

/* Tr(P rho) for the Pauli string P = (x)_q sigma_{codes[q]}, codes[q] in
 * {0=I, 1=X, 2=Y, 3=Z} (Sec. 2: expectation values of Pauli strings). */
int vqd_calc_expec_pauli(const vqd_dm *dm, const uint8_t *codes, double *re, double *im);

/* Device-output read-outs (Sec. 2: expectation values and density-matrix
 * elements read from the state).  The same quantities, reduced in the same
 * fixed order as the calls above (so the values are bit-identical to
 * theirs), written to caller-owned DEVICE memory: out of vqd_calc_trace_dev
 * holds 2 doubles (re, im), of _purity_dev 1, of _probs_dev 2^n, of
 * _expec_z_dev n, of _expec_zz_dev npairs, of _expec_pauli_dev 2 (re, im).
 * vqd_calc_expec_zz_dev reads its pairs from DEVICE memory (2*npairs ints);
 * the Pauli codes stay a host array (read during the call).
 * Asynchronous on the handle's stream: the outputs are valid once that
 * stream has reached the call.  No allocation, no synchronisation and no
 * host copy: the partial sums go to a scratch buffer that vqd_dm_wrap
 * allocates once per handle, so these calls may be captured into a HIP graph
 * together with init and program calls.  Calls on one handle share that
 * scratch and are ordered by its stream.  Errors: VQD_E_ARG (null pointer,
 * bad pair count, Pauli code > 3); nothing is enqueued on an error. */
int vqd_calc_trace_dev(const vqd_dm *dm, double *out);
int vqd_calc_purity_dev(const vqd_dm *dm, double *out);
int vqd_calc_probs_dev(const vqd_dm *dm, double *out);
int vqd_calc_expec_z_dev(const vqd_dm *dm, double *out);
int vqd_calc_expec_zz_dev(const vqd_dm *dm, const int *pairs, int npairs, double *out);
int vqd_calc_expec_pauli_dev(const vqd_dm *dm, const uint8_t *codes, double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc), which
 * therefore cannot wrap a handle: <Z_i> of the state in dev_amps (4^n
 * complex128, layout as for vqd_dm_wrap, n in [1, VQD_MAX_QUBITS]) written
 * to the DEVICE array out[n] on hip_stream, asynchronously, with the same
 * kernels and summation order as vqd_calc_expec_z_dev (bit-identical
 * values).  Allocates nothing: the partial sums go to a static device
 * scratch of 256 * (2 + VQD_MAX_QUBITS) doubles (36 KiB) that every GPU the
 * library runs on holds until the process ends.  All calls on one GPU share
 * that scratch: calls that overlap in time on one GPU (different streams or
 * threads without ordering) race and may return wrong values.  Errors:
 * VQD_E_ARG (null pointer), VQD_E_SIZE (n out of range), VQD_E_HIP. */
int vqd_calc_expec_z_noalloc(const void *dev_amps, int n, void *hip_stream, double *out);

/* ------------------------------------------------------------- surrogate */

/* Virtual-device noise insertion (Sec. 2: a device specification maps an
 * ideal circuit to the channels a noisy device realises; Secs. 3.4, 3.5 and
 * 8: crosstalk, passive T1/T2 decay, thermal relaxation, read-out).  A
 * device holds, per named gate kind, a duration and active noise
 * (depolarising p_depol then dephasing p_deph on the gate's qubits after
 * the gate; one- or two-qubit forms by the gate's size), per-qubit T1 and T2
 * (<= 0 disables), crosstalk edges with a ZZ phase alpha (eq.
 * weak_dephasing_zz), static ZZ couplings, and read-out noise.
 *
 * vqd_device_insert_noise schedules the ideal gates (named gate kinds, 4
 * targets and 4 parameters per gate as for vqd_prog_add_named_many) as soon
 * as possible into parallel batches (a gate joins the batch after the last
 * one that uses any of its qubits; a batch lasts as long as its slowest
 * gate) and emits, per batch: its gates in input order, each followed by its
 * active noise; ZZ(alpha) on every crosstalk edge whose qubits are both
 * idle, if the batch holds a two-qubit gate; ZZ(beta_e dt) on every static
 * coupling e whose pair carries no two-qubit gate of the batch, dt the
 * batch's duration; then for every qubit in ascending order its T1 decay and
 * its T2 decay for the time dt it is idle in the batch.  Operations with no
 * effect are left out.  Output arrays hold cap ops (kinds, 4 targets and 4
 * parameters each, as for named_many); with all three NULL only *out_count
 * is set.  Unspecified gate kinds take no time and add no noise.  Host only.
 *
 * vqd_device_set_angle_scaling: for a parameterised gate kind (and its
 * per-target specifications), multiply its
 * active noise probabilities (scale_noise) and/or its duration
 * (scale_duration) by |theta| / pi, theta the gate's first parameter (App.
 * C); a scaled probability above 1 makes insert_noise fail with VQD_E_ARG.
 * vqd_device_set_thermal: per-qubit ground population p0 of the thermal
 * state (eq. thermalstate; default 1); with p0 < 1 amplitude-damping T1
 * decay becomes gamp_t1(p0, dt, T1), relaxation towards that state (eq.
 * gdamp).  vqd_device_set_passive_forms: the T1 decay kind (VQD_K_AMP_T1,
 * the default, or VQD_K_DEPOL_T1, eq. depolt1) and the T2 decay kind
 * (VQD_K_DEPH_T2, the default, or VQD_K_DEPH_T2S, eq. depht2s).
 * vqd_device_set_static_zz: couplings beta[e] (radians of ZZ phase, as in
 * exp(-i a Z(x)Z), per unit time) on the pairs edges[2e], edges[2e+1].
 * vqd_device_set_off_resonant: off-resonant driving (Sec. 3.3; the silicon
 * device of Sec. 7).  rabi[q] >= 0 and freq[q] are qubit q's Rabi frequency
 * and its own frequency, both angular (radians per unit time); rabi = NULL
 * turns the model off.  A one-qubit gate of duration t > 0 on a qubit q with
 * rabi[q] > 0 drives q, and every qubit j that no gate of the batch targets
 * receives VQD_K_OFFRES(rabi[q], freq[j] - freq[q], t) (eq. off_resonant).
 * These ops follow the batch's gates and their active noise, by driving
 * gate in input order and then ascending j, and precede crosstalk and
 * passive decay.  VQD_E_ARG for a negative or non-finite rabi[q] or a
 * non-finite freq[q].
 * vqd_device_set_serial: serial != 0 runs every gate in a batch of its own,
 * in input order (Sec. 7), instead of the as-soon-as-possible batches.
 * vqd_device_set_exchange_crosstalk: residual exchange on the edges
 * (edges[2e], edges[2e+1]), as the conditional Z rotation of eq.
 * weak_dephasing (VQD_K_CRZ, control edges[2e]) on edges whose two qubits
 * no gate of the batch targets (Sec. 7).  While a two-qubit gate on edge i
 * runs, edge j != i receives crz(on[i * n_edges + j] * theta / pi), theta
 * the gate's first parameter (pi for a kind without parameters); a batch
 * with no two-qubit gate gives edge j crz(off[j]).  Zero values emit
 * nothing; these ops follow the off-resonant ones.  n_edges = 0 turns the
 * model off.  VQD_E_ARG for a bad or repeated edge or a non-finite value.
 *
 * vqd_device_set_parity_readout / vqd_device_parity_readout_noise: the
 * silicon parity read-out of a pair (Sec. 7, eq. projmeas): the two-qubit
 * bit flip bitflip2(b) (eq. bf2) on either side of the parity projection
 * (eq. m), which is accompanied by VQD_K_PARITY_DECAY, while every other
 * qubit idles for t_meas.  parity_readout_noise emits stage 0 (before the
 * projection): bitflip2(b) on (q0, q1), T1 and T2 decay for t_meas on every
 * other qubit in ascending order, then PARITY_DECAY on (q0, q1); stage 1
 * (after it): bitflip2(b).  Zero b or t_meas emit nothing.  VQD_E_ARG for
 * b outside [0, 0.75], a negative or non-finite t_meas, or bad qubits.
 * vqd_device_set_readout_form: VQD_K_DEPOL1 (the default, the model below)
 * or VQD_K_BITFLIP1, the trapped-ion read-out of Sec. 4: a symmetric bit
 * flip bitflip1(eps[q]) (eq. bf) on each listed qubit before the
 * projection, nothing after it, and T1 and T2 decay for t_meas on the
 * unlisted qubits.  VQD_E_ARG for another kind.
 * vqd_device_set_readout / vqd_device_readout_noise: the read-out model of
 * Sec. 8, T1 decay for the measurement time t_meas, then depolarising
 * noise eps[q], then the projective measurement, then depolarising noise
 * eps[q] again.  readout_noise emits, for the listed qubits in list order,
 * stage 0 (before the measurement): T1 decay for t_meas and depol1(eps[q]),
 * then T1 and T2 decay for t_meas on every unlisted qubit in ascending
 * order; stage 1 (after): depol1(eps[q]).  Output arrays as for
 * insert_noise.  VQD_E_ARG for a duplicate or out-of-range qubit. */
typedef struct vqd_device vqd_device;
int vqd_device_create(int n, vqd_device **out);      /* 1 <= n <= 64 */
int vqd_device_destroy(vqd_device *d);
int vqd_device_set_gate(vqd_device *d, int kind, double duration, double p_depol, double p_deph);
/* The specification of one gate kind on one set of targets (nq = the kind's
 * qubit count; the order of the targets does not matter), overriding the
 * kind's own for gates on exactly these qubits: per-qubit rotation
 * fidelities and per-pair two-qubit gates (App. C).  The kind's angle
 * scaling applies to it as well. */
int vqd_device_set_gate_on(vqd_device *d, int kind, int nq, const int *targets, double duration, double p_depol,
                           double p_deph);
int vqd_device_set_angle_scaling(vqd_device *d, int kind, int scale_noise, int scale_duration);
int vqd_device_set_passive(vqd_device *d, const double *T1, const double *T2);   /* n each */
int vqd_device_set_thermal(vqd_device *d, const double *p0);                     /* n */
int vqd_device_set_passive_forms(vqd_device *d, int t1_kind, int t2_kind);
int vqd_device_set_crosstalk(vqd_device *d, int n_edges, const int *edges, double alpha);
int vqd_device_set_static_zz(vqd_device *d, int n_edges, const int *edges, const double *beta);
int vqd_device_set_off_resonant(vqd_device *d, const double *rabi, const double *freq);  /* n each */
int vqd_device_set_serial(vqd_device *d, int serial);
int vqd_device_set_exchange_crosstalk(vqd_device *d, int n_edges, const int *edges, const double *on,
                                      const double *off);    /* on: n_edges^2 (row: active edge), off: n_edges */
int vqd_device_set_readout(vqd_device *d, double t_meas, const double *eps);     /* eps: n */
int vqd_device_set_parity_readout(vqd_device *d, double t_meas, double b);
int vqd_device_set_readout_form(vqd_device *d, int kind);
int vqd_device_parity_readout_noise(const vqd_device *d, int q0, int q1, int stage, int cap, int *out_count,
                                    int *out_kinds, int *out_targets, double *out_params);
int vqd_device_readout_noise(const vqd_device *d, int nq, const int *qubits, int stage, int cap,
                             int *out_count, int *out_kinds, int *out_targets, double *out_params);

/* Device presets: the parameter tables of the paper's virtual devices (App.
 * C) as device specifications; times in microseconds.
 *
 * VQD_PRESET_SUPERCONDUCTING (Sec. 8, table conf:scq), 6 qubits: ideal
 * gates, 0.05 us for one-qubit gates other than Rz and Z (no time), 0.5 us
 * for two-qubit gates; per-qubit T1 relaxation towards the thermal state
 * and T2 dephasing; static ZZ coupling 2 pi beta per microsecond on the 7
 * coupled pairs, beta from vqd_zz_crosstalk_strength with the tabulated
 * couplings, qubit frequencies (control minus target, the pair's lower
 * qubit the control) and anharmonicities in MHz; read-out: 5 us and
 * eps = 1 - the read-out fidelity.  p0 receives 1 - the excited
 * initialisation probabilities (for vqd_dm_init_product_diag).
 *
 * VQD_PRESET_TRAPPED_ION (Sec. 4, table conf:trapped_ions), 8 qubits (two
 * nodes of four ions): Rx, Ry with depolarising noise of average fidelity
 * 0.99999 (vqd_fidelity_to_errors, x = 1), 0.05 us per pi, noise and time
 * scaled by |theta| / pi; H, X, Y as pi rotations; CZ of fidelity 0.999 split
 * 0.1 : 0.9, 5 us; T1 amplitude damping and Gaussian T2* dephasing
 * (3e9 us, 1e6 us); read-out: bit flips of probability 0.001 (the
 * VQD_K_BITFLIP1 form), 50 us.  p0 receives the initialisation fidelity
 * 0.9999.
 *
 * VQD_PRESET_SILICON (Sec. 7, table conf:silicon), 6 qubits in a line,
 * serial: Rx, Ry (and H, X, Y as pi rotations) with per-qubit pure
 * dephasing from the tabulated fidelities (x = 0), 0.1 us per pi, Rx and Ry
 * scaled by |theta| / pi, driving the other qubits off resonance (Rabi
 * frequency 2 pi 5 MHz, qubit frequencies 2 pi x the table's); CZ and CPhase
 * (scaled by |theta| / pi) on the pairs (q, q+1) with two-qubit dephasing
 * from the per-pair fidelities and 1 / (2 x the pair's gate frequency);
 * exchange crosstalk with the tabulated on-matrix and off-values on those
 * pairs; depolarising T1 decay (1e4 us) and per-qubit T2 dephasing; the
 * parity read-out with b = 1 - 0.99 and 10 us.  p0 receives 1.
 *
 * vqd_device_preset creates *out (destroy with vqd_device_destroy); p0 is
 * NULL or holds vqd_device_preset_qubits(preset) doubles.  VQD_E_ARG for an
 * unknown preset. */
enum vqd_preset { VQD_PRESET_SUPERCONDUCTING = 1, VQD_PRESET_TRAPPED_ION = 2, VQD_PRESET_SILICON = 3 };
int vqd_device_preset(int preset, vqd_device **out, double *p0);
int vqd_device_preset_qubits(int preset, int *n);
int vqd_device_insert_noise(const vqd_device *d, int count, const int *kinds, const int *targets,
                            const double *params, int cap, int *out_count, int *out_kinds,
                            int *out_targets, double *out_params);

/* Measurement (the read-out of the devices of Secs. 4-6; the parity
 * measurement of eq. (m); the simulated shots of Sec. 6).
 *
 * vqd_measure_z: projective measurement of qubit q in the computational
 * basis.  The outcome weights are w_m = Re Tr(P_m rho), P_m = |m><m| on q;
 * with the caller's uniform u in [0, 1) the outcome is 0 if w_0 > u (w_0 +
 * w_1), else 1 (the draw rule of the trajectory calls).  rho becomes
 * P_m rho P_m / w_m in place.  *outcome gets m, *weight (may be NULL) w_m.
 * Synchronises the handle's stream (the weights come back to the host), then
 * enqueues the collapse.  VQD_E_STATE if both weights are <= 0.
 *
 * vqd_measure_parity: eq. (m) on (q0, q1): outcome 0 for the odd-parity
 * projector |01><01| + |10><10|, 1 for the even one; otherwise as above.
 *
 * vqd_sample: `shots` basis states from the diagonal probabilities
 * p_x = max(0, Re rho[x][x]): for shot s the smallest x whose running sum
 * p_0 + ... + p_x (formed left to right) exceeds uniforms[s] W, W the sum
 * of all p_x; the last x with p_x > 0 if rounding leaves none.  uniforms
 * ([shots] doubles in [0, 1)) and out ([shots] uint32, bit q = qubit q) are
 * caller-owned device arrays; asynchronous on the handle's stream. */
int vqd_measure_z(vqd_dm *dm, int q, double u, int *outcome, double *weight);
int vqd_measure_parity(vqd_dm *dm, int q0, int q1, double u, int *outcome, double *weight);
int vqd_sample(vqd_dm *dm, const double *uniforms, long long shots, uint32_t *out);

/* Monte Carlo trajectories on state vectors: the paper's alternative to the
 * density matrix (Sec. 2, where QuESTlink replaces each channel by one
 * operator drawn from its Kraus map and averages expected values over many
 * sampled state vectors).  Memory per sample is 2^n amplitudes instead of 4^n.
 *
 * A trajectory program holds n qubits (1 <= n <= 13) and an ordered list of
 * unitary gates and channels.  Each trajectory starts in |0...0> and, in op
 * order, applies every gate as psi -> U psi and every channel {K_i} by
 * drawing one operator: with the trajectory's next uniform variate u in
 * [0, 1) and weights w_i = ||K_i psi||^2, the drawn index is the smallest i
 * whose running sum w_0 + ... + w_i (left to right) exceeds u W, W the sum
 * of all weights (the last positive weight if rounding leaves none), and the
 * state becomes K_i psi / sqrt(w_i).  For a mixed-unitary channel (every
 * K_i^dagger K_i = q_i I, as for the depolarising, dephasing and bit-flip
 * maps of Sec. 3) the weights are the constants q_i.  The same uniform
 * always gives the same draw, so runs are reproducible and comparable
 * sample by sample; a draw can differ between two implementations only
 * when u lies within rounding of an interval boundary.
 *
 * The whole state of a trajectory stays on the chip (registers and LDS of
 * one workgroup); only the outputs go to memory.  Gates must be unitary
 * (|U^dagger U - I| <= 1e-10, else VQD_E_ARG); channels may be any Kraus set
 * of 1 to 16 operators on 1 or 2 qubits, trace preserving or not. */
typedef struct vqd_traj vqd_traj;

typedef struct vqd_traj_info {
    int n;
    int n_ops;            /* gates and channels added */
    int n_channels;       /* uniforms one trajectory consumes */
    int n_phases;         /* register layouts of the plan */
    int n_kernel_ops;     /* ops after fusion */
    int n_mixed;          /* channels drawn from constant weights */
    int n_general;        /* channels whose weights come from the state */
    double fma_per_amp;   /* planned FP64 FMA per amplitude per trajectory */
} vqd_traj_info;

int vqd_traj_create(int n, vqd_traj **out);
int vqd_traj_destroy(vqd_traj *t);
/* Same kinds, targets and parameters as vqd_prog_add_named (gates and
 * channels of Sec. 3); named_many takes 4 targets and 4 parameters per op
 * and adds all or nothing. */
int vqd_traj_add_named(vqd_traj *t, int kind, const int *targets, const double *params);
int vqd_traj_add_named_many(vqd_traj *t, int count, const int *kinds, const int *targets,
                            const double *params);
/* Host matrices as for vqd_prog_add_unitary / vqd_prog_add_kraus (row-major
 * interleaved complex; k in [1, 4] for gates, [1, 2] for Kraus maps of
 * nk in [1, 16] operators). */
int vqd_traj_add_unitary(vqd_traj *t, int k, const int *targets, const double *u);
int vqd_traj_add_kraus(vqd_traj *t, int k, const int *targets, int nk, const double *kraus);

/* Plan the program and copy its descriptors to the current device (which
 * later runs must use).  Ops added afterwards need another compile. */
int vqd_traj_compile(vqd_traj *t);
int vqd_traj_info_get(const vqd_traj *t, vqd_traj_info *out);

/* Host-only planning (no device) and a copy of the planned descriptors:
 * ten uint32 (magic 0x54445156, version 1, n, n_eff = max(n, 4), channels,
 * phases, ops, pool entries, sizeof(TPhase), sizeof(TOp)), then the phases,
 * the ops and the coefficient pool (complex doubles); layouts as in the
 * library's internal header.  With buf = NULL only *needed is set. */
int vqd_traj_plan(vqd_traj *t);
int vqd_traj_export(const vqd_traj *t, void *buf, size_t cap, size_t *needed);

/* Run `count` trajectories, asynchronously on hip_stream.  Device arrays:
 *   uniforms   [count][n_channels] doubles in [0, 1), trajectory-major
 *              (may be NULL when the program has no channel);
 *   z_out      [count][n]   <Z_q> = sum_x |psi_x|^2 (1 - 2 x_q) of each final state;
 *   norm_out   [count]      sum_x |psi_x|^2 (may be NULL);
 *   state_out  [count][2^n] final states, interleaved complex (may be NULL).
 * All are caller-owned.  count = 0 does nothing. */
int vqd_traj_run(vqd_traj *t, const double *uniforms, long long count, double *z_out, double *norm_out,
                 double *state_out, void *hip_stream);

/* Mean over the rows of x ([count][m] device doubles) and its standard error
 * sqrt(sum (x - mean)^2 / (count - 1)) / sqrt(count) (infinity for count = 1),
 * into device arrays mean[m], sem[m]; asynchronous on hip_stream. */
int vqd_traj_stats(const double *x, long long count, int m, double *mean, double *sem, void *hip_stream);

/* Learned surrogate of the emulator: an ensemble of `members` MLPs mapping
 * 24 scaled inputs (8 device parameters and 16 angles of a hardware-efficient
 * ansatz, Sec. 2 and 3; the network itself is not in the paper) to the 10
 * read-outs <Z_i>.  Each member: 24 -> 256 -> 256 -> 256 -> 10, GELU after
 * each hidden layer (GELU(z) = z Phi(z)), linear output; loss = mean squared
 * error over the batch and the 10 outputs; Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected).
 *
 * Number formats: FP32 master weights and Adam moments.  Every matrix product
 * takes bfloat16 operands (round to nearest even) and accumulates in FP32;
 * rounded are the input, the weights, the hidden activations after GELU and
 * the back-propagated pre-activation gradients (which feed the weight, bias
 * and input gradients alike).  Biases and pre-activations stay FP32.
 *
 * Parameter vector of a member (VQD_MLP_N_PARAMS floats): row-major
 * W1[256][24], b1[256], W2[256][256], b2, W3[256][256], b3, W4[10][256],
 * b4[10]; host arrays hold `members` such vectors back to back.
 *
 * Memory: the handle owns its parameters, Adam state and the training
 * workspace (sized for max_batch) on the device current at creation; inputs
 * and outputs of train/predict calls are caller-owned device arrays (x:
 * [B][24] float, y: [B][10] float, idx: optional [B] int row indices into x
 * and y, mean: [B][10], spread: [B], member_out: optional [members][B][10]).
 * Calls on one handle must not overlap. */
typedef struct vqd_mlp vqd_mlp;

#define VQD_MLP_N_PARAMS 140554
enum { VQD_MLP_PARAMS = 0, VQD_MLP_ADAM_M = 1, VQD_MLP_ADAM_V = 2, VQD_MLP_GRAD = 3 };

int vqd_mlp_create(int members, int max_batch, vqd_mlp **out);   /* 1 <= members <= 8 */
int vqd_mlp_destroy(vqd_mlp *h);
int vqd_mlp_n_params(void);

/* Host copies in and out (members x VQD_MLP_N_PARAMS floats).  set: PARAMS,
 * ADAM_M or ADAM_V (setting PARAMS refreshes the bf16 copies); get: also
 * GRAD, the gradient of the last grad/train call.  Both synchronise. */
int vqd_mlp_set_state(vqd_mlp *h, int which, const float *host);
int vqd_mlp_get_state(const vqd_mlp *h, int which, float *host);
int vqd_mlp_set_step(vqd_mlp *h, long long step);   /* Adam step count t */
long long vqd_mlp_get_step(const vqd_mlp *h);

/* Loss (per member, device float[members], may be NULL) and gradient of
 * every member on the same batch of B <= max_batch samples. */
int vqd_mlp_grad(vqd_mlp *h, const float *x, const float *y, const int *idx, int B, float *loss_out,
                 void *hip_stream);

/* vqd_mlp_grad then one Adam step with learning rate lr (t incremented). */
int vqd_mlp_train_step(vqd_mlp *h, const float *x, const float *y, const int *idx, int B, float lr,
                       float *loss_out, void *hip_stream);

/* Ensemble inference on B samples (any B >= 0): mean over members and
 * spread = max over the 10 outputs of the population standard deviation
 * across members.  A caller falls back to the emulator where spread exceeds
 * its threshold. */
int vqd_mlp_predict(const vqd_mlp *h, const float *x, int B, float *mean, float *spread, float *member_out,
                    void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* VQD_H */
