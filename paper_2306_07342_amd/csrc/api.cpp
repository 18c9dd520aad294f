// C ABI of the vqd library (declarations and contract in include/vqd.h).
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "vqd_internal.h"

namespace vqd {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
int fail(int code, const std::string &msg)
{
    set_error(msg);
    return code;
}
int hip_fail(hipError_t e, const char *what)
{
    return fail(VQD_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

std::vector<cd> read_complex(const double *p, size_t count)
{
    std::vector<cd> v(count);
    for (size_t i = 0; i < count; ++i) v[i] = cd(p[2 * i], p[2 * i + 1]);
    return v;
}

bool all_finite(const double *p, size_t count)
{
    for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int check_targets(int n, int k, const int *t)
{
    if (!t) return fail(VQD_E_ARG, "null targets");
    for (int j = 0; j < k; ++j) {
        if (t[j] < 0 || t[j] >= n)
            return fail(VQD_E_ARG, "qubit index " + std::to_string(t[j]) + " outside [0, " +
                                       std::to_string(n) + ")");
        for (int i = 0; i < j; ++i)
            if (t[i] == t[j]) return fail(VQD_E_ARG, "duplicate target " + std::to_string(t[j]));
    }
    return VQD_OK;
}

namespace {

int check_dm(const vqd_dm *dm)
{
    if (!dm || !dm->amps) return fail(VQD_E_ARG, "null density-matrix handle");
    return VQD_OK;
}

// Plan and run a single op as one pass on the handle's immediate program.
int run_single(vqd_dm *dm, const LOp &op)
{
    std::vector<LOp> ops{op};
    HostPlan plan;
    PlanOpts opt;
    int rc = plan_program(dm->n, ops, opt, plan);
    if (rc) return rc;
    rc = upload_plan(plan, dm->imm, dm->stream);
    if (rc) return rc;
    for (size_t i = 0; i < plan.passes.size(); ++i) {
        rc = launch_pass(dm->amps, dm->amps, dm->imm, plan.passes[i], (uint32_t)i, dm->stream);
        if (rc) return rc;
    }
    return VQD_OK;
}

}  // namespace

PlanOpts to_plan_opts(const vqd_plan_opts &o)
{
    PlanOpts po;
    po.tile_bits = o.tile_bits;
    po.min_contig_bits = o.min_contig_bits;
    po.max_ops_per_pass = o.max_ops_per_pass;
    po.fuse_blocks = o.fuse_blocks != 0;
    po.pad_coalesce = o.pad_coalesce != 0;
    po.hermitian = o.hermitian != 0;
    po.relayout = o.relayout != 0;
    return po;
}

int export_plan(const HostPlan &pl, int n, int tile_bits, void *buf, size_t cap, size_t *needed)
{
    const size_t hdr = 12 * sizeof(uint32_t);
    const size_t total = hdr + pl.passes.size() * sizeof(KPass) + pl.phases.size() * sizeof(KPhase) +
                         pl.ops.size() * sizeof(KOp) + pl.mats.size() * 2 * sizeof(double);
    *needed = total;
    if (!buf) return VQD_OK;
    if (cap < total) return fail(VQD_E_SIZE, "export buffer too small");
    uint32_t h[12] = {0x56514450u, 1u, (uint32_t)pl.passes.size(), (uint32_t)pl.phases.size(),
                      (uint32_t)pl.ops.size(), (uint32_t)pl.mats.size(), (uint32_t)sizeof(KPass),
                      (uint32_t)sizeof(KPhase), (uint32_t)sizeof(KOp), (uint32_t)n,
                      (uint32_t)tile_bits, 0u};
    char *o = static_cast<char *>(buf);
    std::memcpy(o, h, hdr);
    o += hdr;
    std::memcpy(o, pl.passes.data(), pl.passes.size() * sizeof(KPass));
    o += pl.passes.size() * sizeof(KPass);
    std::memcpy(o, pl.phases.data(), pl.phases.size() * sizeof(KPhase));
    o += pl.phases.size() * sizeof(KPhase);
    std::memcpy(o, pl.ops.data(), pl.ops.size() * sizeof(KOp));
    o += pl.ops.size() * sizeof(KOp);
    for (const cd &z : pl.mats) {
        const double v[2] = {z.real(), z.imag()};
        std::memcpy(o, v, sizeof v);
        o += sizeof v;
    }
    return VQD_OK;
}

}  // namespace vqd

using namespace vqd;

extern "C" {

const char *vqd_last_error(void) { return g_last_error.c_str(); }

const char *vqd_version(void) { return "vqd-gfx950 0.1"; }

int vqd_dm_wrap(void *dev_amps, int n, size_t bytes, void *hip_stream, vqd_dm **out)
{
    clear_error();
    if (!out) return fail(VQD_E_ARG, "null output pointer");
    *out = nullptr;
    if (!dev_amps) return fail(VQD_E_ARG, "null device buffer");
    if (n < 1 || n > VQD_MAX_QUBITS)
        return fail(VQD_E_SIZE, "n must be in [1, " + std::to_string(VQD_MAX_QUBITS) + "]");
    const size_t need = size_t(16) << (2 * n);
    if (bytes < need)
        return fail(VQD_E_SIZE, "buffer of " + std::to_string(bytes) + " bytes; 4^n complex128 need " +
                                    std::to_string(need));
    vqd_dm *dm = new (std::nothrow) vqd_dm();
    if (!dm) return fail(VQD_E_NOMEM, "handle allocation failed");
    dm->amps = static_cast<double2 *>(dev_amps);
    dm->n = n;
    dm->bytes = bytes;
    dm->stream = static_cast<hipStream_t>(hip_stream);
    (void)hipGetDevice(&dm->device);
    // the device-output read-outs never allocate (they may be captured in a
    // graph): their scratch is sized for this n here, once (on a host with
    // no GPU there is nothing to allocate, and those calls report that)
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
        if (int rc = ensure_scratch(dm->gred, readout_scratch_doubles(n), 0)) {
            delete dm;
            return rc;
        }
    }
    *out = dm;
    return VQD_OK;
}

int vqd_dm_destroy(vqd_dm *dm)
{
    clear_error();
    if (!dm) return VQD_OK;
    (void)hipStreamSynchronize(dm->stream);
    free_dev_program(dm->imm);
    free_scratch(dm->red);
    free_scratch(dm->gred);
    if (dm->alt) (void)hipFree(dm->alt);
    delete dm;
    return VQD_OK;
}

int vqd_dm_set_stream(vqd_dm *dm, void *hip_stream)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (hipStreamSynchronize(dm->stream) != hipSuccess) return fail(VQD_E_HIP, "stream sync failed");
    dm->stream = static_cast<hipStream_t>(hip_stream);
    return VQD_OK;
}

int vqd_dm_init_zero(vqd_dm *dm)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    return launch_init(dm->amps, dm->n, 0, 0, nullptr, dm->stream);
}

int vqd_dm_init_basis(vqd_dm *dm, uint64_t b)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (b >= (1ull << dm->n)) return fail(VQD_E_ARG, "basis state outside [0, 2^n)");
    return launch_init(dm->amps, dm->n, 0, b + (b << dm->n), nullptr, dm->stream);
}

int vqd_dm_init_product_diag(vqd_dm *dm, const double *p0)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (!p0) return fail(VQD_E_ARG, "null p0");
    if (!all_finite(p0, dm->n)) return fail(VQD_E_ARG, "non-finite p0");
    return launch_init(dm->amps, dm->n, 1, 0, p0, dm->stream);
}

int vqd_dm_copy_to_host(const vqd_dm *dm, double *host)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (!host) return fail(VQD_E_ARG, "null host buffer");
    VQD_HIP(hipMemcpyAsync(host, dm->amps, size_t(16) << (2 * dm->n), hipMemcpyDeviceToHost, dm->stream));
    VQD_HIP(hipStreamSynchronize(dm->stream));
    return VQD_OK;
}

int vqd_dm_copy_from_host(vqd_dm *dm, const double *host)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (!host) return fail(VQD_E_ARG, "null host buffer");
    VQD_HIP(hipMemcpyAsync(dm->amps, host, size_t(16) << (2 * dm->n), hipMemcpyHostToDevice, dm->stream));
    VQD_HIP(hipStreamSynchronize(dm->stream));
    return VQD_OK;
}

static int apply_superop_k(vqd_dm *dm, int k, const int *t, const double *s)
{
    if (int rc = check_dm(dm)) return rc;
    if (int rc = check_targets(dm->n, k, t)) return rc;
    if (!s) return fail(VQD_E_ARG, "null matrix");
    const size_t cnt = size_t(1) << (4 * k);
    if (!all_finite(s, 2 * cnt)) return fail(VQD_E_ARG, "non-finite matrix entry");
    std::vector<cd> S = read_complex(s, cnt);
    return run_single(dm, make_superop_op(k, t, S.data()));
}

static int apply_unitary_k(vqd_dm *dm, int k, const int *t, const double *u)
{
    if (int rc = check_dm(dm)) return rc;
    if (int rc = check_targets(dm->n, k, t)) return rc;
    if (!u) return fail(VQD_E_ARG, "null matrix");
    const size_t cnt = size_t(1) << (2 * k);
    if (!all_finite(u, 2 * cnt)) return fail(VQD_E_ARG, "non-finite matrix entry");
    std::vector<cd> U = read_complex(u, cnt);
    return run_single(dm, make_unitary_op(k, t, U.data()));
}

int vqd_apply_unitary1(vqd_dm *dm, int q, const double *u)
{
    clear_error();
    return apply_unitary_k(dm, 1, &q, u);
}

int vqd_apply_unitary2(vqd_dm *dm, int q0, int q1, const double *u)
{
    clear_error();
    const int t[2] = {q0, q1};
    return apply_unitary_k(dm, 2, t, u);
}

int vqd_apply_superop1(vqd_dm *dm, int q, const double *s)
{
    clear_error();
    return apply_superop_k(dm, 1, &q, s);
}

int vqd_apply_superop2(vqd_dm *dm, int q0, int q1, const double *s)
{
    clear_error();
    const int t[2] = {q0, q1};
    return apply_superop_k(dm, 2, t, s);
}

int vqd_apply_fused(vqd_dm *dm, int k, const int *targets, int kind, const double *m)
{
    clear_error();
    if (kind == VQD_BLOCK_UNITARY) {
        if (k < 1 || k > 4) return fail(VQD_E_SIZE, "fused unitary block needs k in [1, 4]");
        return apply_unitary_k(dm, k, targets, m);
    }
    if (kind == VQD_BLOCK_SUPEROP) {
        if (k < 1 || k > 2) return fail(VQD_E_SIZE, "fused superoperator block needs k in [1, 2]");
        return apply_superop_k(dm, k, targets, m);
    }
    return fail(VQD_E_ARG, "unknown block kind");
}

int vqd_apply_diagonal(vqd_dm *dm, int k, const int *targets, const double *d)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (k < 1 || k > 2) return fail(VQD_E_SIZE, "diagonal op needs k in [1, 2]");
    if (int rc = check_targets(dm->n, k, targets)) return rc;
    if (!d) return fail(VQD_E_ARG, "null factors");
    const size_t cnt = size_t(1) << (2 * k);
    if (!all_finite(d, 2 * cnt)) return fail(VQD_E_ARG, "non-finite factor");
    LOp op;
    op.k = k;
    for (int j = 0; j < k; ++j) op.q[j] = targets[j];
    op.diag = true;
    op.D = read_complex(d, cnt);
    return run_single(dm, op);
}

// ------------------------------------------------------------- programs --

int vqd_kind_arity(int kind, int *n_qubits, int *n_params)
{
    return kind_arity(kind, n_qubits, n_params);
}

int vqd_kind_matrix(int kind, const double *params, double *out)
{
    clear_error();
    if (!out) return fail(VQD_E_ARG, "null output");
    int np = 0;
    if (kind_arity(kind, nullptr, &np) != 0) return fail(VQD_E_ARG, "unknown kind");
    if (np > 0 && !params) return fail(VQD_E_ARG, "null params");
    std::vector<cd> U;
    int k = 0;
    if (int rc = kind_matrix(kind, params, U, k)) return rc;
    for (size_t i = 0; i < U.size(); ++i) {
        out[2 * i] = U[i].real();
        out[2 * i + 1] = U[i].imag();
    }
    return VQD_OK;
}

int vqd_kind_superop(int kind, const double *params, double *out)
{
    clear_error();
    if (!out) return fail(VQD_E_ARG, "null output");
    int np = 0;
    if (kind_arity(kind, nullptr, &np) != 0) return fail(VQD_E_ARG, "unknown kind");
    if (np > 0 && !params) return fail(VQD_E_ARG, "null params");
    std::vector<cd> S;
    int k = 0;
    if (int rc = kind_superop(kind, params, S, k)) return rc;
    for (size_t i = 0; i < S.size(); ++i) {
        out[2 * i] = S[i].real();
        out[2 * i + 1] = S[i].imag();
    }
    return VQD_OK;
}

int vqd_kraus_to_superop(int k, int nk, const double *kraus, double *out)
{
    clear_error();
    if (k < 1 || k > 2) return fail(VQD_E_SIZE, "Kraus maps need k in [1, 2]");
    if (nk < 1 || !kraus || !out) return fail(VQD_E_ARG, "bad Kraus arguments");
    const size_t cnt = size_t(nk) << (2 * k);
    if (!all_finite(kraus, 2 * cnt)) return fail(VQD_E_ARG, "non-finite Kraus entry");
    std::vector<cd> K = read_complex(kraus, cnt), S;
    kraus_to_superop(k, nk, K.data(), S);
    for (size_t i = 0; i < S.size(); ++i) {
        out[2 * i] = S[i].real();
        out[2 * i + 1] = S[i].imag();
    }
    return VQD_OK;
}

void vqd_plan_opts_default(vqd_plan_opts *o)
{
    if (!o) return;
    o->tile_bits = 13;
    o->min_contig_bits = 3;
    o->max_ops_per_pass = 0;
    o->fuse_blocks = 1;
    o->pad_coalesce = 1;
    o->hermitian = 0;
    o->relayout = 0;
}

int vqd_prog_create(int n, vqd_prog **out)
{
    clear_error();
    if (!out) return fail(VQD_E_ARG, "null output pointer");
    *out = nullptr;
    if (n < 1 || n > VQD_MAX_QUBITS) return fail(VQD_E_SIZE, "n must be in [1, 16]");
    vqd_prog *p = new (std::nothrow) vqd_prog();
    if (!p) return fail(VQD_E_NOMEM, "program allocation failed");
    p->n = n;
    *out = p;
    return VQD_OK;
}

int vqd_prog_destroy(vqd_prog *p)
{
    clear_error();
    if (!p) return VQD_OK;
    (void)hipDeviceSynchronize();
    free_dev_program(p->dev);
    delete p;
    return VQD_OK;
}

static int prog_push(vqd_prog *p, LOp &&op)
{
    p->ops.push_back(std::move(op));
    p->compiled = false;
    return VQD_OK;
}

int vqd_prog_add_named(vqd_prog *p, int kind, const int *targets, const double *params)
{
    clear_error();
    if (!p) return fail(VQD_E_ARG, "null program");
    int nq = 0, np = 0;
    if (kind_arity(kind, &nq, &np) != 0) return fail(VQD_E_ARG, "unknown kind " + std::to_string(kind));
    if (int rc = check_targets(p->n, nq, targets)) return rc;
    if (np > 0 && !params) return fail(VQD_E_ARG, "null params");
    std::vector<cd> S;
    int k = 0;
    if (int rc = kind_superop(kind, params, S, k)) return rc;
    return prog_push(p, make_superop_op(k, targets, S.data()));
}

int vqd_prog_add_named_many(vqd_prog *p, int count, const int *kinds, const int *targets,
                            const double *params)
{
    clear_error();
    if (!p) return fail(VQD_E_ARG, "null program");
    if (count < 0 || (count > 0 && (!kinds || !targets || !params))) return fail(VQD_E_ARG, "bad arrays");
    const size_t before = p->ops.size();
    for (int i = 0; i < count; ++i) {
        const int rc = vqd_prog_add_named(p, kinds[i], targets + 4 * (size_t)i, params + 4 * (size_t)i);
        if (rc) {
            p->ops.resize(before);      // all or nothing
            return fail(rc, "op " + std::to_string(i) + ": " + vqd_last_error());
        }
    }
    return VQD_OK;
}

int vqd_prog_add_unitary(vqd_prog *p, int k, const int *targets, const double *u)
{
    clear_error();
    if (!p) return fail(VQD_E_ARG, "null program");
    if (k < 1 || k > 4) return fail(VQD_E_SIZE, "unitary needs k in [1, 4]");
    if (int rc = check_targets(p->n, k, targets)) return rc;
    if (!u) return fail(VQD_E_ARG, "null matrix");
    const size_t cnt = size_t(1) << (2 * k);
    if (!all_finite(u, 2 * cnt)) return fail(VQD_E_ARG, "non-finite matrix entry");
    std::vector<cd> U = read_complex(u, cnt);
    return prog_push(p, make_unitary_op(k, targets, U.data()));
}

int vqd_prog_add_superop(vqd_prog *p, int k, const int *targets, const double *s)
{
    clear_error();
    if (!p) return fail(VQD_E_ARG, "null program");
    if (k < 1 || k > 2) return fail(VQD_E_SIZE, "superoperator needs k in [1, 2]");
    if (int rc = check_targets(p->n, k, targets)) return rc;
    if (!s) return fail(VQD_E_ARG, "null matrix");
    const size_t cnt = size_t(1) << (4 * k);
    if (!all_finite(s, 2 * cnt)) return fail(VQD_E_ARG, "non-finite matrix entry");
    std::vector<cd> S = read_complex(s, cnt);
    return prog_push(p, make_superop_op(k, targets, S.data()));
}

int vqd_prog_add_kraus(vqd_prog *p, int k, const int *targets, int nk, const double *kraus)
{
    clear_error();
    if (!p) return fail(VQD_E_ARG, "null program");
    if (k < 1 || k > 2) return fail(VQD_E_SIZE, "Kraus map needs k in [1, 2]");
    if (int rc = check_targets(p->n, k, targets)) return rc;
    if (nk < 1 || !kraus) return fail(VQD_E_ARG, "bad Kraus arguments");
    const size_t cnt = size_t(nk) << (2 * k);
    if (!all_finite(kraus, 2 * cnt)) return fail(VQD_E_ARG, "non-finite Kraus entry");
    std::vector<cd> K = read_complex(kraus, cnt), S;
    kraus_to_superop(k, nk, K.data(), S);
    return prog_push(p, make_superop_op(k, targets, S.data()));
}


int vqd_prog_plan(vqd_prog *p, const vqd_plan_opts *opts)
{
    clear_error();
    if (!p) return fail(VQD_E_ARG, "null program");
    vqd_plan_opts o;
    vqd_plan_opts_default(&o);
    if (opts) o = *opts;
    p->compiled = false;
    p->tile_bits = o.tile_bits;
    return plan_program(p->n, p->ops, to_plan_opts(o), p->plan);
}

int vqd_prog_export(const vqd_prog *p, void *buf, size_t cap, size_t *needed)
{
    clear_error();
    if (!p || !needed) return fail(VQD_E_ARG, "null argument");
    return export_plan(p->plan, p->n, p->tile_bits, buf, cap, needed);
}


int vqd_prog_compile(vqd_prog *p, const vqd_plan_opts *opts)
{
    clear_error();
    if (!p) return fail(VQD_E_ARG, "null program");
    if (int rc = vqd_prog_plan(p, opts)) return rc;
    if (p->plan.passes.empty()) {
        p->compiled = true;
        return VQD_OK;
    }
    if (int rc = upload_plan(p->plan, p->dev, nullptr)) return rc;
    (void)hipGetDevice(&p->device);
    p->n_kernel_ops = (int)p->plan.ops.size();
    p->compiled = true;
    return VQD_OK;
}

int vqd_prog_run(vqd_prog *p, vqd_dm *dm)
{
    clear_error();
    if (!p) return fail(VQD_E_ARG, "null program");
    if (int rc = check_dm(dm)) return rc;
    if (!p->compiled) return fail(VQD_E_STATE, "program not compiled");
    if (p->n != dm->n) return fail(VQD_E_ARG, "program and state have different qubit counts");
    if (!p->plan.passes.empty() && p->device != dm->device)
        return fail(VQD_E_ARG, "program compiled for another device");
    if (p->plan.alt_buffer && !dm->alt) {
        // the second state buffer of a relabelled plan, kept by the handle
        const size_t need = size_t(16) << (2 * dm->n);
        if (hipMalloc(&dm->alt, need) != hipSuccess) {
            dm->alt = nullptr;
            return fail(VQD_E_NOMEM, "second state buffer allocation failed");
        }
    }
    // a pass that changes the layout stores into the other buffer; the
    // planner makes their number even, so the state ends where it started
    double2 *cur = dm->amps;
    for (size_t i = 0; i < p->plan.passes.size(); ++i) {
        double2 *out = p->plan.passes[i].swap_out ? (cur == dm->amps ? dm->alt : dm->amps) : cur;
        if (int rc = launch_pass(cur, out, p->dev, p->plan.passes[i], (uint32_t)i, dm->stream)) return rc;
        cur = out;
    }
    if (cur != dm->amps) return fail(VQD_E_STATE, "relabelled plan ended in the second buffer");
    return VQD_OK;
}

int vqd_prog_info_get(const vqd_prog *p, vqd_prog_info *out)
{
    clear_error();
    if (!p || !out) return fail(VQD_E_ARG, "null argument");
    out->n = p->n;
    out->n_ops = (int)p->ops.size();
    out->n_passes = (int)p->plan.passes.size();
    out->n_phases = (int)p->plan.phases.size();
    out->n_kernel_ops = (int)p->plan.ops.size();
    out->fma_per_amp = p->plan.fma_per_amp;
    out->hermitian = p->plan.hermitian ? 1 : 0;
    out->tile_fraction = p->plan.tile_fraction;
    out->relabelled = p->plan.relabelled ? 1 : 0;
    out->layout_changes = 0;
    for (const KPass &P : p->plan.passes) out->layout_changes += P.swap_out ? 1 : 0;
    return VQD_OK;
}

// ------------------------------------------------------------- read-out --

int vqd_calc_trace(const vqd_dm *dm, double *re, double *im)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (!re || !im) return fail(VQD_E_ARG, "null output");
    double t[2];
    auto *m = const_cast<vqd_dm *>(dm);
    if (int rc = reduce_diag(m->amps, m->n, m->red, m->stream, t, nullptr, nullptr)) return rc;
    *re = t[0];
    *im = t[1];
    return VQD_OK;
}

int vqd_calc_purity(const vqd_dm *dm, double *out)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (!out) return fail(VQD_E_ARG, "null output");
    auto *m = const_cast<vqd_dm *>(dm);
    return reduce_purity(m->amps, m->n, m->red, m->stream, out);
}

int vqd_calc_probs(const vqd_dm *dm, double *out)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (!out) return fail(VQD_E_ARG, "null output");
    auto *m = const_cast<vqd_dm *>(dm);
    return reduce_diag(m->amps, m->n, m->red, m->stream, nullptr, nullptr, out);
}

int vqd_calc_expec_z(const vqd_dm *dm, double *out)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (!out) return fail(VQD_E_ARG, "null output");
    auto *m = const_cast<vqd_dm *>(dm);
    return reduce_diag(m->amps, m->n, m->red, m->stream, nullptr, out, nullptr);
}

int vqd_calc_expec_zz(const vqd_dm *dm, const int *pairs, int npairs, double *out)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (npairs < 0 || (npairs > 0 && (!pairs || !out))) return fail(VQD_E_ARG, "bad pair arguments");
    if (npairs == 0) return VQD_OK;
    for (int i = 0; i < npairs; ++i)
        if (int rc = check_targets(dm->n, 2, pairs + 2 * i)) return rc;
    auto *m = const_cast<vqd_dm *>(dm);
    return reduce_zz(m->amps, m->n, pairs, npairs, m->red, m->stream, out);
}

int vqd_calc_expec_pauli(const vqd_dm *dm, const uint8_t *codes, double *re, double *im)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (!codes || !re || !im) return fail(VQD_E_ARG, "null argument");
    uint64_t xm = 0, zm = 0;
    int ny = 0;
    for (int q = 0; q < dm->n; ++q) {
        const int c = codes[q];
        if (c > 3) return fail(VQD_E_ARG, "Pauli code must be 0..3");
        if (c == 1 || c == 2) xm |= 1ull << q;
        if (c == 2 || c == 3) zm |= 1ull << q;
        ny += (c == 2);
    }
    auto *m = const_cast<vqd_dm *>(dm);
    return reduce_pauli(m->amps, m->n, xm, zm, ny, m->red, m->stream, re, im);
}

// ------------------------------------------------- device-output read-outs --

int vqd_calc_trace_dev(const vqd_dm *dm, double *out)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (!out) return fail(VQD_E_ARG, "null output");
    return reduce_diag_dev(dm->amps, dm->n, dm->gred, dm->stream, out, nullptr, nullptr);
}

int vqd_calc_purity_dev(const vqd_dm *dm, double *out)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (!out) return fail(VQD_E_ARG, "null output");
    return reduce_purity_dev(dm->amps, dm->n, dm->gred, dm->stream, out);
}

int vqd_calc_probs_dev(const vqd_dm *dm, double *out)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (!out) return fail(VQD_E_ARG, "null output");
    return reduce_diag_dev(dm->amps, dm->n, dm->gred, dm->stream, nullptr, nullptr, out);
}

int vqd_calc_expec_z_dev(const vqd_dm *dm, double *out)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (!out) return fail(VQD_E_ARG, "null output");
    return reduce_diag_dev(dm->amps, dm->n, dm->gred, dm->stream, nullptr, out, nullptr);
}

int vqd_calc_expec_zz_dev(const vqd_dm *dm, const int *pairs, int npairs, double *out)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (npairs < 0 || (npairs > 0 && (!pairs || !out))) return fail(VQD_E_ARG, "bad pair arguments");
    if (npairs == 0) return VQD_OK;
    return reduce_zz_dev(dm->amps, dm->n, pairs, npairs, dm->gred, dm->stream, out);
}

int vqd_calc_expec_pauli_dev(const vqd_dm *dm, const uint8_t *codes, double *out)
{
    clear_error();
    if (int rc = check_dm(dm)) return rc;
    if (!codes || !out) return fail(VQD_E_ARG, "null argument");
    uint64_t xm = 0, zm = 0;
    int ny = 0;
    for (int q = 0; q < dm->n; ++q) {
        const int c = codes[q];
        if (c > 3) return fail(VQD_E_ARG, "Pauli code must be 0..3");
        if (c == 1 || c == 2) xm |= 1ull << q;
        if (c == 2 || c == 3) zm |= 1ull << q;
        ny += (c == 2);
    }
    return reduce_pauli_dev(dm->amps, dm->n, xm, zm, ny, dm->gred, dm->stream, out);
}

int vqd_calc_expec_z_noalloc(const void *dev_amps, int n, void *hip_stream, double *out)
{
    clear_error();
    if (!dev_amps || !out) return fail(VQD_E_ARG, "null argument");
    if (n < 1 || n > VQD_MAX_QUBITS)
        return fail(VQD_E_SIZE, "n must be in [1, " + std::to_string(VQD_MAX_QUBITS) + "]");
    return expec_z_noalloc(static_cast<const double2 *>(dev_amps), n, static_cast<hipStream_t>(hip_stream), out);
}

}  // extern "C"
