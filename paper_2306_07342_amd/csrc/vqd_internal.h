// Internal definitions of the vqd library: descriptor structs shared by the
// host planner and the gfx950 kernels, handle structs, error helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/vqd.h"

namespace vqd {

using cd = std::complex<double>;

// ----------------------------------------------------------------- errors --
void set_error(const std::string &msg);
void clear_error();
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

// Argument helpers of the C ABI.
std::vector<cd> read_complex(const double *p, size_t count);
bool all_finite(const double *p, size_t count);
int check_targets(int n, int k, const int *t);

#define VQD_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

// ------------------------------------------------------- kernel descriptors --
// A pass streams every amplitude through HBM once.  The 2n vector bits are
// split into L "tile" bits (local index 0..2^L-1, kept inside one workgroup)
// and 2n-L "group" bits (one workgroup per tile).  A pass runs a sequence of
// register phases: in a phase each thread holds 16 amplitudes whose local
// indices differ in 4 "register" bits; the other L-4 local bits come from
// the thread id.  Between phases the tile is exchanged through LDS.

constexpr int kMaxTileBits = 13;
constexpr int kMaxThreadBits = kMaxTileBits - 4;
constexpr int kRegBits = 4;
constexpr int kSlots = 16;
constexpr uint32_t kPhantomPos = 30;   // global position of a bit beyond 2n (only n = 1 has any)
constexpr uint32_t kNotLocal = 0xffu;  // KOp::lpos of a group (non-tile) bit

enum KOpKind : uint32_t {
    KOP_MAT = 1,      // dense matrix on the register bits `opmask`, stored column-major
    KOP_XOR = 2,      // flip-pattern matrix on `opmask`: y[i] = sum_x W[x][i] a[i ^ flip(x)],
                      // flip(x) flipping the row and column bit of the same qubits
    KOP_DIAG = 3,     // 16 element-wise factors indexed by the register slot
    KOP_DIAG_RT = 4,  // element-wise factors from an LDS table indexed by global bits
    KOP_PTM = 5,      // a trace-preserving map on the two register bits `opmask` (the row
                      // and column bit of one qubit) that takes Hermitian blocks to
                      // Hermitian blocks, applied through its real Pauli transfer matrix R:
                      // the 2x2 block B of each slot group (B[u][v] at local index u + 2v)
                      // goes to its Pauli components a_P = Tr(P B), a' = R a, and back.
                      // Coefficients: rows X, Y, Z of R / 2 over the columns (I, X, Y, Z),
                      // 12 reals packed two per entry (row I is (1, 0, 0, 0))
};

// KOP_DIAG_RT index modes: which register slot bits feed the table index.
enum RtMode : uint32_t {
    RT_NONE = 0,      // index = gathered global bits (same factor for all 16 slots)
    RT_PAIR_A = 1,    // index = b(slot 0) + 2 b(slot 2) + 4 * gathered bits
    RT_PAIR_B = 2,    // index = b(slot 1) + 2 b(slot 3) + 4 * gathered bits
    RT_GENERIC = 3,   // every index bit gathered from the slot's own global index
};

struct alignas(16) KOp {
    uint32_t kind;
    uint32_t opmask;    // KOP_MAT / KOP_XOR: register bits acted on (ascending)
    uint32_t mat;       // offset of the coefficients in the pool (complex entries; real-only
                        // coefficients are packed two per entry); KOP_DIAG_RT: offset inside
                        // the pass's LDS-staged table block
    uint32_t real;      // all coefficients are real
    uint32_t mode;      // KOP_DIAG_RT: RtMode
    uint32_t nbits;     // KOP_DIAG_RT: number of gathered index bits
    uint32_t gpos[4];   // KOP_DIAG_RT: their global bit positions (gathered bit j -> index bit j)
    uint32_t lpos[4];   // KOP_DIAG_RT: local tile bit of gathered bit j, or kNotLocal for a
                        // group bit (uniform over the workgroup's tile)
    uint32_t pad[2];
};

// LDS index swizzle of the pass kernels: xor the low 4 bits of a local index
// (16 elements of 16 bytes: one pass of 16 lanes of a 128-bit LDS access
// over the banks) with its bits 4-7 and 8-11, so that strided register phases
// spread over the banks.  Xor-linear: the swizzle of (thread bits | slot
// bits) is the xor of the two parts' swizzles.
__host__ __device__ inline uint32_t lds_swizzle(uint32_t l)
{
    return l ^ (((l >> 4) ^ (l >> 8)) & 15u);
}

// Row bit q <-> column bit q + n: the transpose of an index bit position in
// the vectorised layout.
__host__ __device__ inline uint32_t mirror_pos(uint32_t g, uint32_t n) { return g < n ? g + n : g - n; }

struct alignas(16) KPhase {
    uint32_t op_begin, op_end;
    uint32_t reg_local[4];
    uint32_t reg_gpos[4];
    uint32_t thr_local[kMaxThreadBits];
    uint32_t thr_gpos[kMaxThreadBits];
    // Per register slot e (filled by finish_slot_tables from the fields
    // above, so the kernels read them instead of recomputing them):
    uint32_t lds_slot[kSlots];   // byte offset part in LDS: swizzle(local bits of e) * 16
    uint32_t g_slot[kSlots];     // global index part: OR of 1 << reg_gpos[b] over the bits b of e
    uint32_t gm_slot[kSlots];    // the same with every position mirrored (row <-> column bit)
    // Physical position of the transpose partner (the other bit of the same
    // qubit) of each reg_gpos / thr_gpos entry, in the layout those positions
    // are in: n away in the vectorised layout, the neighbouring bit in an
    // interleaved one (unused thread entries 0)
    uint32_t reg_mpos[4];
    uint32_t thr_mpos[kMaxThreadBits];
};

struct alignas(16) KPass {
    uint32_t L;               // tile bits (threads = 2^(L-4))
    uint32_t n_group_bits;
    uint32_t phase_begin, phase_end;
    uint32_t phantom;         // some tile bit lies beyond 2n (tiny registers)
    uint32_t xcd_swizzle;     // remap workgroup ids so tiles sharing cache lines share an XCD
    uint32_t rt_mat;          // start (complex entries) of this pass's runtime-diagonal tables
    uint32_t rt_count;        // their total size; staged in LDS after the tile
    uint64_t n_tiles;
    uint32_t group_gpos[32];
    uint32_t herm;            // Hermitian mode (kHerm* flags): group_gpos holds m row bits,
                              // then their m column bits; the n_tiles = N(N+1)/2 tiles
                              // (N = 2^m) are the group pairs i <= j
    // kHermHalfIn: the previous pass's group pair (i, j) of the amplitude in
    // register slot e of this pass's first phase takes the bits hi_slot[e]
    // into i and hj_slot[e] into j (the thread and tile parts are added by
    // the kernel); filled by finish_slot_tables
    uint32_t hi_slot[kSlots];
    uint32_t hj_slot[kSlots];
    // Relabelled plans: the state between two passes is stored under a
    // permutation of the qubits (the physical row bit of qubit q at position
    // lambda(q), its column bit at lambda(q) + n).  group_gpos and the first
    // phase's positions are in the layout this pass loads; out_gpos and the
    // last phase's positions in the layout it stores (equal to group_gpos
    // when the layout stays)
    uint32_t out_gpos[32];
    uint32_t swap_out;        // stores into the other state buffer (the layout changes)
};
constexpr uint32_t kHermPass = 1u;     // computes the tiles i <= j only
constexpr uint32_t kHermMirror = 2u;   // also stores each i < j tile's conjugate transpose
                                       // to its mirror (the program's last pass)
constexpr uint32_t kHermHalfIn = 4u;   // the previous pass stored only its tiles i <= j:
                                       // an amplitude whose group pair in that pass had
                                       // i > j is loaded from its transpose, conjugated
// Bits 4-5 of KPass::herm: c, the number of group qubits below qubit 3 (they
// split 128-byte lines between tiles).  Tiles are launched in blocks of 4^c
// (i = I 2^c + a, j = J 2^c + b over a, b < 2^c, blocks I <= J), a block's
// members 8 launch indices apart so that they run on one XCD together; in a
// block with I = J the members with a > b are computed but not stored.
constexpr uint32_t kHermLineShift = 4u;
// Bits 8-11: the block stride s = min(8, number of blocks), the launch-index
// distance between a block's members (no padding when there are few blocks).
constexpr uint32_t kHermStrideShift = 8u;

// Device-side image of a planned program.
struct DevProgram {
    void *buf = nullptr;      // one allocation holding everything below
    size_t bytes = 0;
    KPass *passes = nullptr;
    KPhase *phases = nullptr;
    KOp *ops = nullptr;
    double2 *mats = nullptr;
};

// Host-side planned program.
// How the coefficients of one kernel op were made from the logical ops, so
// that they can be recomputed for other parameter values of the same op
// kinds (parametric batch templates) without planning again.
// One diagonal op's share of a runtime-diagonal table: which of its index
// bits come from register slots (row_j, col_j in the pair modes) and which are
// gathered (rtj, at union positions upos of the merged op's index).
struct RtPart {
    int src = -1;
    int nb = 0;
    int g[4] = {0, 0, 0, 0};      // global position of each op index bit
    uint32_t mode = 0;
    int row_j = -1, col_j = -1;
    std::vector<int> rtj, upos;
};
constexpr int kMaxRtBits = 4;     // gathered bits of one runtime-diagonal op

struct Recipe {
    bool rt = false;
    std::vector<int> src;       // logical ops multiplied into the block, application order
    int reg_gpos[4] = {0, 0, 0, 0};
    uint32_t kind = 0, mask = 0;
    bool real = false;
    uint32_t mode = 0;          // runtime diagonal: index mode and bit mapping
    int rt_union = 0;           // runtime diagonal: gathered bits and the ops multiplied in
    std::vector<RtPart> rt_parts;
    size_t mat_off = 0;         // where the coefficients live in HostPlan::mats
};

struct HostPlan {
    std::vector<KPass> passes;
    std::vector<KPhase> phases;
    std::vector<KOp> ops;
    std::vector<cd> mats;
    std::vector<Recipe> recipes;    // one per kernel op when recorded
    double fma_per_amp = 0;
    bool alt_buffer = false;        // some pass stores into a second state buffer
    bool relabelled = false;        // positions set for per-pass layouts (mirror tables included)
    bool hermitian = false;         // planned in Hermitian mode
    double tile_fraction = 1.0;     // share of the amplitudes the passes compute
};

// ------------------------------------------------------------- logical ops --
struct LOp {
    int k = 0;                    // number of qubits
    int q[4] = {0, 0, 0, 0};      // targets, q[0] = least significant
    bool diag = false;            // element-wise superoperator (factors in D)
    bool wide_unitary = false;    // k >= 3 unitary applied as U on rows, conj(U) on columns
    std::vector<cd> S;            // superoperator 4^k x 4^k (k <= 2), local index order
    std::vector<cd> D;            // diagonal factors 4^k (diag ops)
    std::vector<cd> U;            // 2^k x 2^k (wide unitaries)
};

// Build a logical op from a superoperator; detects diagonal structure.
LOp make_superop_op(int k, const int *targets, const cd *S);
// The same, written into an existing op (its vectors keep their capacity).
void fill_superop_op(LOp &op, int k, const int *targets, const cd *S);
LOp make_unitary_op(int k, const int *targets, const cd *U);

// Planner entry point.  Returns VQD_OK or an error code (message set).
struct PlanOpts {
    int tile_bits = 13;
    int min_contig_bits = 3;
    int max_ops_per_pass = 0;
    bool fuse_blocks = true;
    bool pad_coalesce = true;
    bool record_recipes = false;    // fill HostPlan::recipes
    bool keep_identity = false;     // do not drop ops that are exactly the identity
    bool merge_rt = true;           // tabulate runs of runtime diagonals together
    int rt_budget = 0;              // runtime-diagonal table entries a pass may stage in
                                    // LDS (0: what 160 KiB leaves beside the tile)
    bool hermitian = false;         // compute half the tiles of a Hermitian state when every
                                    // op preserves Hermiticity (HostPlan::hermitian says if)
    bool relayout = false;          // Hermitian plans: store the state between passes under
                                    // qubit relabellings that make tile I/O contiguous
};
int plan_program(int n, const std::vector<LOp> &ops, const PlanOpts &opt, HostPlan &out);
// Fill the per-slot tables of every phase and pass of a plan (KPhase::lds_slot,
// g_slot, gm_slot; KPass::hi_slot, hj_slot) from their bit assignments.
void finish_slot_tables(int n, HostPlan &plan);
// Recompute a recorded plan's coefficients for new logical ops of the same
// structure (same kinds and targets).  mats gets the plan's layout.
int recompute_mats(int n, const HostPlan &plan, const std::vector<LOp> &ops, std::vector<cd> &mats);
// Table of a (merged) runtime-diagonal op, layout as in RtMode.
void rt_table(uint32_t mode, int ubits, const std::vector<RtPart> &parts, const std::vector<LOp> &ops,
              std::vector<cd> &table);
// Serialise a plan (layout of vqd_prog_export).
int export_plan(const HostPlan &plan, int n, int tile_bits, void *buf, size_t cap, size_t *needed);
// Parametric templates: validate, plan with canonical parameters, and compute
// one instance's coefficient block (`lops` is per-call scratch).
int check_template(int n, int count, const int *kinds, const int *targets);
int plan_template(int n, const std::vector<int> &kinds, const std::vector<int> &targets, PlanOpts o,
                  HostPlan &plan);
int template_mats(int n, const std::vector<int> &kinds, const std::vector<int> &targets, const HostPlan &plan,
                  const double *params, std::vector<LOp> &lops, std::vector<cd> &mats);
PlanOpts to_plan_opts(const vqd_plan_opts &o);

// Upload a plan into a device program (re-using its buffer when large enough).
int upload_plan(const HostPlan &plan, DevProgram &dev, hipStream_t stream);
void free_dev_program(DevProgram &dev);

// --------------------------------------------------------- trajectories --
// Monte Carlo state-vector trajectories.  One trajectory of n_eff = max(n, 4)
// qubits is held by 2^(n_eff-4) threads with 16 register slots each: in every
// phase four qubits are the register bits and the others the thread bits; the
// state moves between phases through LDS.  A workgroup holds several
// trajectories when n_eff < 12.
constexpr int kTrajMaxQubits = 13;
constexpr int kTrajMaxThreadBits = kTrajMaxQubits - 4;
constexpr int kTrajMaxKraus = 16;

enum TOpKind : uint32_t {
    TOP_MAT = 1,      // dense matrix on register bits `mask` (column-major; real ones packed)
    TOP_DTHR = 2,     // diagonal gate on thread qubits only: 2^nd factors, index bit j = bit dq[j]
                      // of the amplitude index (one factor per thread)
    TOP_MIX = 3,      // mixed-unitary channel: nk (running sum of weights, weight), then nk unitaries
    TOP_KRAUS = 4,    // general channel: nk Gram matrices K^dagger K (row-major), then nk
                      // Kraus matrices (column-major)
    TOP_DREG = 5,     // diagonal gate on register qubits only: 16 factors, one per register slot
    TOP_DMIX = 6,     // two-qubit diagonal gate, one register qubit (bit `mask`) and one thread
                      // qubit dq[0]: factors (thread bit, register bit) = 00, 01, 10, 11
    TOP_DRM = 7,      // a TOP_DREG and a TOP_DMIX in a row, as one op: 16 slot factors, then
                      // the four TOP_DMIX factors (register bit `mask`, thread qubit dq[0])
    TOP_DMIX2 = 8,    // two TOP_DMIX in a row, as one op: the first's four factors (register
                      // bit `mask`, thread qubit dq[0]), then the second's (register bit
                      // `dmask`, thread qubit dq[1])
    TOP_MATS = 9,     // nd (2 to 4) one-qubit TOP_MATs in a row, as one op: matrix j acts on
                      // register bit (dmask >> 2j) & 3, its 2x2 complex coefficients
                      // (column-major) at 4j
};

struct alignas(16) TOp {
    uint32_t kind;
    uint32_t mask;    // TOP_MAT / TOP_MIX / TOP_KRAUS: register bits acted on
    uint32_t mat;     // offset of the coefficients in the pool (complex entries)
    uint32_t real;    // TOP_MAT: real coefficients, packed two per entry
    uint32_t nk;      // TOP_MIX / TOP_KRAUS: number of operators
    uint32_t chan;    // TOP_MIX / TOP_KRAUS: channel index (column of the uniforms)
    uint32_t nd;      // TOP_DTHR: number of qubits (1 or 2)
    uint32_t dmask;   // TOP_MIX / TOP_KRAUS: bit i set if operator i is diagonal
    uint32_t dq[2];   // TOP_DTHR / TOP_DMIX: thread qubits, dq[0] the low bit of the factor index
    uint32_t rmask;   // TOP_MIX / TOP_KRAUS: bit i set if operator i is diagonal and real
    uint32_t gdiag;   // TOP_KRAUS: every K_i^dagger K_i is diagonal (only rho_T's diagonal is needed)
    // One-qubit channels with two operators whose draw needs only a few
    // numbers carry them here (inl = 1), so the kernel reads them with the
    // descriptor instead of in dependent loads from the pool (which still
    // holds the full form):
    //  * TOP_MIX, both operators diagonal and real: cf = {running sum 0,
    //    running sum 1, operator 0's two diagonal entries, operator 1's};
    //  * TOP_KRAUS with diagonal Gram matrices and a diagonal real K_0:
    //    cf = {G_0's two diagonal entries, G_1's, K_0's}.
    // Diagonal entries in register order (register bit value 0, then 1).
    // inl = 2: another mixed-unitary channel whose operator 0 is stored as
    // exactly the identity: cf = {running sum 0, the total}, enough to see
    // that operator 0 is drawn (the common case).
    uint32_t inl;
    // On the first op of a run of inl = 1 channels in one phase (at most
    // kTrajGroupMax ops, at most kTrajGroupKraus of them damping, at least
    // two, trace preserving within 1e-15; the mixed-unitary ones with
    // diagonal entries of magnitude 1 within 1e-15): the run's length.  Trajectories of whole waves draw the run with
    // one reduction; 0 elsewhere.
    uint32_t grp;
    uint32_t pad_[2];
    double cf[6];
};
constexpr uint32_t kTrajGroupMax = 8;
constexpr uint32_t kTrajGroupKraus = 4;

struct alignas(16) TPhase {
    uint32_t op_begin, op_end;
    uint32_t reg_q[4];                      // qubit of register bit b
    uint32_t thr_q[kTrajMaxThreadBits];     // qubit of thread bit i (zero-filled past n_eff - 4)
    uint32_t flags;                         // kTPhaseReduces
    uint32_t lds_slot[kSlots];              // swizzled LDS index part of register slot e
};
// The phase holds a general channel, whose weights are a reduction over the
// whole state (a workgroup barrier when a trajectory spans several waves).
constexpr uint32_t kTPhaseReduces = 1u;

int launch_traj(const TPhase *phases, uint32_t n_phases, const TOp *ops, const double2 *pool, int n,
                int n_eff, uint32_t n_ch, const double *U, uint64_t T, double *z_out, double *norm_out,
                double *state_out, hipStream_t stream);
int launch_traj_stats(const double *x, uint64_t T, int m, double *mean, double *sem, hipStream_t stream);

// ----------------------------------------------------------- measurement --
enum MeasKind : uint32_t { MEAS_Z = 0, MEAS_PARITY = 1 };
int launch_project(double2 *amps, int n, int kind, int q0, int q1, int m, double scale, hipStream_t stream);
// scratch: 2^(n+1) + 1 doubles of device memory
int launch_sample(const double2 *amps, int n, double *scratch, const double *U, uint64_t shots, uint32_t *out,
                  hipStream_t stream);

// ------------------------------------------------------------- batched --
// One density matrix of a batch (queue order).
struct alignas(16) BatchItem {
    uint64_t arena_off;       // first amplitude of the instance in the arena
    uint64_t mat_base;        // added to every coefficient offset of its passes
    uint32_t n;
    uint32_t pass_begin, pass_end;
    uint32_t out_off;         // first of its n <Z_i> outputs
};

struct BatchDev {
    DevProgram prog;          // all instances' passes, phases, ops, coefficients
    BatchItem *items = nullptr;
    uint32_t *counter = nullptr;
    void *buf = nullptr;      // allocation holding items and counter
    uint32_t n_items = 0;
    uint32_t max_rt = 0;      // largest runtime-diagonal table block of any pass
};

// ------------------------------------------------------------- launches --
// One pass: loads from amps_in, stores to amps_out (the same buffer unless
// the pass changes the layout).
int launch_pass(double2 *amps_in, double2 *amps_out, const DevProgram &dev, const KPass &pass, uint32_t pass_idx,
                hipStream_t stream);
int launch_init(double2 *amps, int n, int mode, uint64_t b, const double *p0, hipStream_t stream);
int launch_batch(double2 *arena, const BatchDev &bd, double *out, hipStream_t stream);

struct ReduceScratch {
    double *dev = nullptr;      // partials + results
    size_t cap = 0;             // doubles
    double *host = nullptr;     // pinned host staging
    size_t host_cap = 0;
};
int ensure_scratch(ReduceScratch &s, size_t dev_doubles, size_t host_doubles);
void free_scratch(ReduceScratch &s);

int reduce_purity(const double2 *amps, int n, ReduceScratch &s, hipStream_t st, double *out);
int reduce_diag(const double2 *amps, int n, ReduceScratch &s, hipStream_t st, double *trace2,
                double *z, double *probs);
int reduce_zz(const double2 *amps, int n, const int *pairs, int npairs, ReduceScratch &s,
              hipStream_t st, double *out);
int reduce_pauli(const double2 *amps, int n, uint64_t xmask, uint64_t zmask, int ny,
                 ReduceScratch &s, hipStream_t st, double *re, double *im);
// Device-output forms: no allocation, no synchronisation, no host copy.  `s`
// holds readout_scratch_doubles(n) doubles of device memory.
size_t readout_scratch_doubles(int n);
int reduce_purity_dev(const double2 *amps, int n, const ReduceScratch &s, hipStream_t st, double *out);
int reduce_diag_dev(const double2 *amps, int n, const ReduceScratch &s, hipStream_t st, double *tr, double *z,
                    double *probs);
int reduce_zz_dev(const double2 *amps, int n, const int *pairs, int npairs, const ReduceScratch &s,
                  hipStream_t st, double *out);
int reduce_pauli_dev(const double2 *amps, int n, uint64_t xmask, uint64_t zmask, int ny, const ReduceScratch &s,
                     hipStream_t st, double *out);
// <Z_i> into device memory with the library's static device scratch: no
// handle, no allocation.
int expec_z_noalloc(const double2 *amps, int n, hipStream_t st, double *out);

// ------------------------------------------------------------- builders --
int kind_arity(int kind, int *nq, int *np);
// Parameters used to plan a parametric template: generic values for which no
// matrix entry of the kind vanishes or turns real by accident.
void canonical_params(int kind, double *p);
int kind_matrix(int kind, const double *params, std::vector<cd> &U, int &k);
int kind_superop(int kind, const double *params, std::vector<cd> &S, int &k);
// Kraus set of a named channel (each a 2^k x 2^k row-major matrix).
int kind_kraus(int kind, const double *params, std::vector<std::vector<cd>> &Ks, int &k);
bool kind_is_channel(int kind);
void kraus_to_superop(int k, int nk, const cd *K, std::vector<cd> &S);
void unitary_to_superop(int k, const cd *U, std::vector<cd> &S);

}  // namespace vqd

// ------------------------------------------------------------- handles --
struct vqd_dm {
    double2 *amps = nullptr;
    double2 *alt = nullptr;         // second state buffer of relabelled plans (owned; on demand)
    int n = 0;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    vqd::DevProgram imm;            // descriptors of immediate (single-op) calls
    vqd::ReduceScratch red;         // synchronous read-outs (grows on demand)
    vqd::ReduceScratch gred;        // device-output read-outs: fixed size, allocated by the wrap
};

struct vqd_prog {
    int n = 0;
    std::vector<vqd::LOp> ops;
    vqd::HostPlan plan;
    vqd::DevProgram dev;
    bool compiled = false;
    int device = -1;
    int n_kernel_ops = 0;
    int tile_bits = 13;
};
