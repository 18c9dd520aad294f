// Virtual-device noise insertion (declarations and contract in
// include/vqd.h): maps an ideal gate list to the noisy op stream of a device
// specification.  Gates are scheduled as soon as possible into parallel
// batches (a gate joins the batch after the last one that uses any of its
// qubits); a batch lasts as long as its slowest gate.  Each batch is
// emitted as its gates in input order, each followed by its active noise
// (depolarising, then dephasing; optionally scaled by the rotation angle,
// App. C), then ZZ crosstalk on the listed edges whose qubits are both idle
// (when the batch holds a two-qubit gate), then the static ZZ coupling of
// every coupled pair that carries no two-qubit gate (Sec. 8), then passive
// T1 and T2 decay for every qubit's idle time dt (Secs. 2, 3.4, 3.5, 8; eqs.
// ampt1, depolt1, gdamp, depht2, depht2s).  Read-out noise (Sec. 8: T1 decay
// for the measurement time and depolarising noise on either side of the
// projection) comes from its own call.
#include <algorithm>
#include <array>
#include <cmath>
#include <string>
#include <vector>

#include "vqd_internal.h"

namespace {

struct GateSpec {
    double duration = 0.0, p_depol = 0.0, p_deph = 0.0;
    bool scale_noise = false, scale_duration = false;     // by |theta| / pi
};

struct Op {
    int kind;
    int t[4];
    double p[4];
};

}  // namespace

struct vqd_device {
    int n = 0;
    GateSpec gate[VQD_K_COUNT];
    // per-target specifications: (kind, sorted targets) -> spec
    std::vector<std::pair<std::array<int, 5>, GateSpec>> gate_on;
    std::vector<double> T1, T2;
    std::vector<double> p0;                    // thermal ground populations
    int t1_kind = VQD_K_AMP_T1, t2_kind = VQD_K_DEPH_T2;
    std::vector<std::pair<int, int>> edges;
    double alpha = 0.0;
    std::vector<std::pair<int, int>> zz_edges;  // static coupling
    std::vector<double> zz_beta;
    double t_meas = 0.0;
    std::vector<double> eps;                   // read-out infidelities
    int readout_kind = VQD_K_DEPOL1;           // or VQD_K_BITFLIP1 (Sec. 4)
    std::vector<double> rabi, freq;            // off-resonant driving (empty: off)
    double par_t = 0.0, par_b = 0.0;           // parity read-out
    bool serial = false;                       // one gate per batch
    std::vector<std::pair<int, int>> xe_edges; // exchange crosstalk: edges,
    std::vector<double> xe_on, xe_off;         // on[i * m + j], off[j]
};

namespace {

using OpList = std::vector<Op>;

void emit(OpList &out, int kind, int a, int b, double p0, double p1 = 0.0, double p2 = 0.0)
{
    out.push_back(Op{kind, {a, b, 0, 0}, {p0, p1, p2, 0.0}});
}

// T1 decay of qubit q over a time dt: amplitude damping (towards the thermal
// state under a thermal population) or depolarising decay.
void t1_decay(const vqd_device *d, OpList &out, int q, double dt)
{
    if (!(d->T1[q] > 0.0) || !(dt > 0.0)) return;
    if (d->t1_kind == VQD_K_DEPOL_T1) emit(out, VQD_K_DEPOL_T1, q, 0, dt, d->T1[q]);
    else if (d->p0[q] < 1.0) emit(out, VQD_K_GAMP_T1, q, 0, d->p0[q], dt, d->T1[q]);
    else emit(out, VQD_K_AMP_T1, q, 0, dt, d->T1[q]);
}

void t2_decay(const vqd_device *d, OpList &out, int q, double dt)
{
    if (!(d->T2[q] > 0.0) || !(dt > 0.0)) return;
    emit(out, d->t2_kind, q, 0, dt, d->T2[q]);
}

int write_ops(const OpList &out, int cap, int *out_count, int *out_kinds, int *out_targets, double *out_params)
{
    *out_count = (int)out.size();
    if (!out_kinds && !out_targets && !out_params) return VQD_OK;      // size query
    if (!out_kinds || !out_targets || !out_params) return vqd::fail(VQD_E_ARG, "null output array");
    if (cap < (int)out.size()) return vqd::fail(VQD_E_SIZE, "output arrays too small");
    for (size_t i = 0; i < out.size(); ++i) {
        out_kinds[i] = out[i].kind;
        for (int j = 0; j < 4; ++j) {
            out_targets[4 * i + j] = out[i].t[j];
            out_params[4 * i + j] = out[i].p[j];
        }
    }
    return VQD_OK;
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

std::array<int, 5> target_key(int kind, int nq, const int *t)
{
    std::array<int, 5> k{kind, -1, -1, -1, -1};
    for (int j = 0; j < nq; ++j) k[1 + j] = t[j];
    std::sort(k.begin() + 1, k.begin() + 1 + nq);
    return k;
}

// The gate's specification: the one for its exact target set, else its kind's.
const GateSpec &spec_for(const vqd_device *d, int kind, int nq, const int *t)
{
    if (!d->gate_on.empty()) {
        const std::array<int, 5> k = target_key(kind, nq, t);
        for (const auto &e : d->gate_on)
            if (e.first == k) return e.second;
    }
    return d->gate[kind];
}

}  // namespace

using namespace vqd;

extern "C" {

int vqd_device_create(int n, vqd_device **out)
{
    clear_error();
    if (!out) return fail(VQD_E_ARG, "null output pointer");
    *out = nullptr;
    if (n < 1 || n > 64) return fail(VQD_E_SIZE, "device needs n in [1, 64]");
    vqd_device *d = new (std::nothrow) vqd_device;
    if (!d) return fail(VQD_E_NOMEM, "out of host memory");
    d->n = n;
    d->T1.assign(n, 0.0);
    d->T2.assign(n, 0.0);
    d->p0.assign(n, 1.0);
    d->eps.assign(n, 0.0);
    *out = d;
    return VQD_OK;
}

int vqd_device_destroy(vqd_device *d)
{
    clear_error();
    delete d;
    return VQD_OK;
}

int vqd_device_set_gate(vqd_device *d, int kind, double duration, double p_depol, double p_deph)
{
    clear_error();
    if (!d) return fail(VQD_E_ARG, "null device");
    int nq = 0;
    if (kind_arity(kind, &nq, nullptr) != 0 || kind_is_channel(kind))
        return fail(VQD_E_ARG, "not a gate kind: " + std::to_string(kind));
    if (!(duration >= 0.0) || !std::isfinite(duration)) return fail(VQD_E_ARG, "duration must be finite and >= 0");
    if (!(p_depol >= 0.0 && p_depol <= 1.0) || !(p_deph >= 0.0 && p_deph <= 1.0))
        return fail(VQD_E_ARG, "noise probabilities outside [0, 1]");
    d->gate[kind] = GateSpec{duration, p_depol, p_deph};
    return VQD_OK;
}

int vqd_device_set_passive(vqd_device *d, const double *T1, const double *T2)
{
    clear_error();
    if (!d || !T1 || !T2) return fail(VQD_E_ARG, "null argument");
    for (int q = 0; q < d->n; ++q)
        if (std::isnan(T1[q]) || std::isnan(T2[q])) return fail(VQD_E_ARG, "NaN coherence time");
    d->T1.assign(T1, T1 + d->n);
    d->T2.assign(T2, T2 + d->n);
    return VQD_OK;
}

int vqd_device_set_crosstalk(vqd_device *d, int n_edges, const int *edges, double alpha)
{
    clear_error();
    if (!d) return fail(VQD_E_ARG, "null device");
    if (n_edges < 0 || (n_edges > 0 && !edges)) return fail(VQD_E_ARG, "bad edge list");
    if (!std::isfinite(alpha)) return fail(VQD_E_ARG, "non-finite crosstalk phase");
    std::vector<std::pair<int, int>> e;
    for (int i = 0; i < n_edges; ++i) {
        if (int rc = check_targets(d->n, 2, edges + 2 * i)) return rc;
        e.emplace_back(edges[2 * i], edges[2 * i + 1]);
    }
    d->edges = std::move(e);
    d->alpha = alpha;
    return VQD_OK;
}

int vqd_device_set_gate_on(vqd_device *d, int kind, int nq, const int *targets, double duration, double p_depol,
                           double p_deph)
{
    clear_error();
    if (!d || !targets) return fail(VQD_E_ARG, "null argument");
    int k_nq = 0;
    if (kind_arity(kind, &k_nq, nullptr) != 0 || kind_is_channel(kind))
        return fail(VQD_E_ARG, "not a gate kind: " + std::to_string(kind));
    if (nq != k_nq) return fail(VQD_E_ARG, "target count does not match the gate kind");
    if (int rc = check_targets(d->n, nq, targets)) return rc;
    if (!(duration >= 0.0) || !std::isfinite(duration)) return fail(VQD_E_ARG, "duration must be finite and >= 0");
    if (!(p_depol >= 0.0 && p_depol <= 1.0) || !(p_deph >= 0.0 && p_deph <= 1.0))
        return fail(VQD_E_ARG, "noise probabilities outside [0, 1]");
    const std::array<int, 5> key = target_key(kind, nq, targets);
    GateSpec g{duration, p_depol, p_deph, d->gate[kind].scale_noise, d->gate[kind].scale_duration};
    for (auto &e : d->gate_on)
        if (e.first == key) {
            e.second = g;
            return VQD_OK;
        }
    d->gate_on.emplace_back(key, g);
    return VQD_OK;
}

int vqd_device_set_angle_scaling(vqd_device *d, int kind, int scale_noise, int scale_duration)
{
    clear_error();
    if (!d) return fail(VQD_E_ARG, "null device");
    int nq = 0, np = 0;
    if (kind_arity(kind, &nq, &np) != 0 || kind_is_channel(kind) || np < 1)
        return fail(VQD_E_ARG, "not a parameterised gate kind: " + std::to_string(kind));
    d->gate[kind].scale_noise = scale_noise != 0;
    d->gate[kind].scale_duration = scale_duration != 0;
    for (auto &e : d->gate_on)
        if (e.first[0] == kind) {
            e.second.scale_noise = scale_noise != 0;
            e.second.scale_duration = scale_duration != 0;
        }
    return VQD_OK;
}

int vqd_device_set_thermal(vqd_device *d, const double *p0)
{
    clear_error();
    if (!d || !p0) return fail(VQD_E_ARG, "null argument");
    for (int q = 0; q < d->n; ++q)
        if (!(p0[q] >= 0.0 && p0[q] <= 1.0)) return fail(VQD_E_ARG, "thermal population outside [0, 1]");
    d->p0.assign(p0, p0 + d->n);
    return VQD_OK;
}

int vqd_device_set_passive_forms(vqd_device *d, int t1_kind, int t2_kind)
{
    clear_error();
    if (!d) return fail(VQD_E_ARG, "null device");
    if (t1_kind != VQD_K_AMP_T1 && t1_kind != VQD_K_DEPOL_T1)
        return fail(VQD_E_ARG, "T1 decay must be VQD_K_AMP_T1 or VQD_K_DEPOL_T1");
    if (t2_kind != VQD_K_DEPH_T2 && t2_kind != VQD_K_DEPH_T2S)
        return fail(VQD_E_ARG, "T2 decay must be VQD_K_DEPH_T2 or VQD_K_DEPH_T2S");
    d->t1_kind = t1_kind;
    d->t2_kind = t2_kind;
    return VQD_OK;
}

int vqd_device_set_static_zz(vqd_device *d, int n_edges, const int *edges, const double *beta)
{
    clear_error();
    if (!d) return fail(VQD_E_ARG, "null device");
    if (n_edges < 0 || (n_edges > 0 && (!edges || !beta))) return fail(VQD_E_ARG, "bad edge list");
    std::vector<std::pair<int, int>> e;
    std::vector<double> b;
    for (int i = 0; i < n_edges; ++i) {
        if (int rc = check_targets(d->n, 2, edges + 2 * i)) return rc;
        if (!std::isfinite(beta[i])) return fail(VQD_E_ARG, "non-finite coupling");
        e.emplace_back(edges[2 * i], edges[2 * i + 1]);
        b.push_back(beta[i]);
    }
    d->zz_edges = std::move(e);
    d->zz_beta = std::move(b);
    return VQD_OK;
}

int vqd_device_set_off_resonant(vqd_device *d, const double *rabi, const double *freq)
{
    clear_error();
    if (!d) return fail(VQD_E_ARG, "null device");
    if (!rabi) {
        d->rabi.clear();
        d->freq.clear();
        return VQD_OK;
    }
    if (!freq) return fail(VQD_E_ARG, "null qubit frequencies");
    for (int q = 0; q < d->n; ++q) {
        if (!finite_nonneg(rabi[q])) return fail(VQD_E_ARG, "Rabi frequency negative or not finite");
        if (!std::isfinite(freq[q])) return fail(VQD_E_ARG, "qubit frequency not finite");
    }
    d->rabi.assign(rabi, rabi + d->n);
    d->freq.assign(freq, freq + d->n);
    return VQD_OK;
}

int vqd_device_set_parity_readout(vqd_device *d, double t_meas, double b)
{
    clear_error();
    if (!d) return fail(VQD_E_ARG, "null device");
    if (!finite_nonneg(t_meas)) return fail(VQD_E_ARG, "read-out time negative or not finite");
    if (!(b >= 0.0 && b <= 0.75)) return fail(VQD_E_ARG, "bit-flip probability outside [0, 0.75]");
    d->par_t = t_meas;
    d->par_b = b;
    return VQD_OK;
}

int vqd_device_parity_readout_noise(const vqd_device *d, int q0, int q1, int stage, int cap, int *out_count,
                                    int *out_kinds, int *out_targets, double *out_params)
{
    clear_error();
    if (!d || !out_count) return fail(VQD_E_ARG, "null argument");
    const int t[2] = {q0, q1};
    if (int rc = check_targets(d->n, 2, t)) return rc;
    if (stage != 0 && stage != 1) return fail(VQD_E_ARG, "stage must be 0 or 1");
    OpList out;
    if (d->par_b > 0.0) emit(out, VQD_K_BITFLIP2, q0, q1, d->par_b);
    if (stage == 0) {
        if (d->par_t > 0.0)
            for (int q = 0; q < d->n; ++q)
                if (q != q0 && q != q1) {
                    t1_decay(d, out, q, d->par_t);
                    t2_decay(d, out, q, d->par_t);
                }
        emit(out, VQD_K_PARITY_DECAY, q0, q1, 0.0);
    }
    return write_ops(out, cap, out_count, out_kinds, out_targets, out_params);
}

int vqd_device_set_readout_form(vqd_device *d, int kind)
{
    clear_error();
    if (!d) return fail(VQD_E_ARG, "null device");
    if (kind != VQD_K_DEPOL1 && kind != VQD_K_BITFLIP1)
        return fail(VQD_E_ARG, "read-out form must be VQD_K_DEPOL1 or VQD_K_BITFLIP1");
    d->readout_kind = kind;
    return VQD_OK;
}

int vqd_device_set_serial(vqd_device *d, int serial)
{
    clear_error();
    if (!d) return fail(VQD_E_ARG, "null device");
    d->serial = serial != 0;
    return VQD_OK;
}

int vqd_device_set_exchange_crosstalk(vqd_device *d, int n_edges, const int *edges, const double *on,
                                      const double *off)
{
    clear_error();
    if (!d) return fail(VQD_E_ARG, "null device");
    if (n_edges < 0 || (n_edges > 0 && (!edges || !on || !off))) return fail(VQD_E_ARG, "bad edge arrays");
    std::vector<std::pair<int, int>> e;
    for (int i = 0; i < n_edges; ++i) {
        if (int rc = check_targets(d->n, 2, edges + 2 * (size_t)i)) return rc;
        const std::pair<int, int> k(std::min(edges[2 * i], edges[2 * i + 1]),
                                    std::max(edges[2 * i], edges[2 * i + 1]));
        for (const auto &x : e)
            if (std::min(x.first, x.second) == k.first && std::max(x.first, x.second) == k.second)
                return fail(VQD_E_ARG, "repeated edge");
        e.emplace_back(edges[2 * i], edges[2 * i + 1]);
    }
    const size_t m = (size_t)n_edges;
    for (size_t i = 0; i < m * m; ++i)
        if (!std::isfinite(on[i])) return fail(VQD_E_ARG, "exchange crosstalk not finite");
    for (size_t i = 0; i < m; ++i)
        if (!std::isfinite(off[i])) return fail(VQD_E_ARG, "exchange crosstalk not finite");
    d->xe_edges = std::move(e);
    d->xe_on.assign(on, on + m * m);
    d->xe_off.assign(off, off + m);
    return VQD_OK;
}

int vqd_device_set_readout(vqd_device *d, double t_meas, const double *eps)
{
    clear_error();
    if (!d || !eps) return fail(VQD_E_ARG, "null argument");
    if (!finite_nonneg(t_meas)) return fail(VQD_E_ARG, "measurement time must be finite and >= 0");
    for (int q = 0; q < d->n; ++q)
        if (!(eps[q] >= 0.0 && eps[q] <= 1.0)) return fail(VQD_E_ARG, "read-out infidelity outside [0, 1]");
    d->t_meas = t_meas;
    d->eps.assign(eps, eps + d->n);
    return VQD_OK;
}

int vqd_device_readout_noise(const vqd_device *d, int nq, const int *qubits, int stage, int cap, int *out_count,
                             int *out_kinds, int *out_targets, double *out_params)
{
    clear_error();
    if (!d || !out_count) return fail(VQD_E_ARG, "null argument");
    if (stage != 0 && stage != 1) return fail(VQD_E_ARG, "stage must be 0 (before) or 1 (after)");
    if (nq < 0 || nq > d->n || (nq > 0 && !qubits)) return fail(VQD_E_ARG, "bad qubit list");
    std::vector<char> measured(d->n, 0);
    for (int i = 0; i < nq; ++i) {
        if (qubits[i] < 0 || qubits[i] >= d->n) return fail(VQD_E_ARG, "qubit out of range");
        if (measured[qubits[i]]) return fail(VQD_E_ARG, "duplicate qubit");
        measured[qubits[i]] = 1;
    }
    OpList out;
    const bool flips = d->readout_kind == VQD_K_BITFLIP1;
    for (int i = 0; i < nq; ++i) {
        const int q = qubits[i];
        if (flips) {
            if (stage == 0 && d->eps[q] > 0.0) emit(out, VQD_K_BITFLIP1, q, 0, d->eps[q]);
            continue;
        }
        if (stage == 0) t1_decay(d, out, q, d->t_meas);
        if (d->eps[q] > 0.0) emit(out, VQD_K_DEPOL1, q, 0, d->eps[q]);
    }
    if (stage == 0)
        for (int q = 0; q < d->n; ++q)
            if (!measured[q]) {
                t1_decay(d, out, q, d->t_meas);
                t2_decay(d, out, q, d->t_meas);
            }
    return write_ops(out, cap, out_count, out_kinds, out_targets, out_params);
}

int vqd_device_insert_noise(const vqd_device *d, int count, const int *kinds, const int *targets, const double *params,
                            int cap, int *out_count, int *out_kinds, int *out_targets, double *out_params)
{
    clear_error();
    if (!d || !out_count) return fail(VQD_E_ARG, "null argument");
    if (count < 0 || (count > 0 && (!kinds || !targets || !params))) return fail(VQD_E_ARG, "bad gate arrays");
    const int n = d->n;
    // validate, and schedule as soon as possible
    std::vector<int> last(n, -1), batch_of(count);
    int n_batches = 0;
    for (int i = 0; i < count; ++i) {
        int nq = 0, np = 0;
        if (kind_arity(kinds[i], &nq, &np) != 0 || kind_is_channel(kinds[i]))
            return fail(VQD_E_ARG, "gate " + std::to_string(i) + ": not a gate kind");
        if (int rc = check_targets(n, nq, targets + 4 * (size_t)i)) return rc;
        int b = d->serial ? i : 0;
        for (int j = 0; j < nq; ++j) b = std::max(b, last[targets[4 * (size_t)i + j]] + 1);
        for (int j = 0; j < nq; ++j) last[targets[4 * (size_t)i + j]] = b;
        batch_of[i] = b;
        n_batches = std::max(n_batches, b + 1);
    }
    std::vector<std::vector<int>> batches(n_batches);
    for (int i = 0; i < count; ++i) batches[batch_of[i]].push_back(i);

    OpList out;
    std::vector<double> busy(n);
    std::vector<char> active(n);
    std::vector<std::pair<int, int>> pairs;      // two-qubit gates of the batch
    std::vector<std::pair<int, double>> drives;  // driven one-qubit gates: (qubit, duration)
    std::vector<std::pair<int, double>> xon;     // two-qubit gates on crosstalk edges: (edge, theta)
    const int m = (int)d->xe_edges.size();
    for (const auto &batch : batches) {
        double dur = 0.0;
        bool two = false;
        std::fill(busy.begin(), busy.end(), 0.0);
        std::fill(active.begin(), active.end(), 0);
        pairs.clear();
        drives.clear();
        xon.clear();
        for (int i : batch) {
            int nq = 0;
            kind_arity(kinds[i], &nq, nullptr);
            const int *t = targets + 4 * (size_t)i;
            const GateSpec &g = spec_for(d, kinds[i], nq, t);
            const double *par = params + 4 * (size_t)i;
            const double s = std::fabs(par[0]) / 3.14159265358979323846;
            const double gd = g.scale_duration ? g.duration * s : g.duration;
            const double pd = g.scale_noise ? g.p_depol * s : g.p_depol;
            const double pq = g.scale_noise ? g.p_deph * s : g.p_deph;
            if (!(pd <= 1.0) || !(pq <= 1.0))
                return fail(VQD_E_ARG, "gate " + std::to_string(i) + ": angle-scaled noise probability above 1");
            dur = std::max(dur, gd);
            Op o{kinds[i], {0, 0, 0, 0}, {0.0, 0.0, 0.0, 0.0}};
            for (int j = 0; j < 4; ++j) {
                o.t[j] = t[j];
                o.p[j] = par[j];
            }
            out.push_back(o);
            if (pd > 0.0) emit(out, nq == 1 ? VQD_K_DEPOL1 : VQD_K_DEPOL2, t[0], nq > 1 ? t[1] : 0, pd);
            if (pq > 0.0) emit(out, nq == 1 ? VQD_K_DEPH1 : VQD_K_DEPH2, t[0], nq > 1 ? t[1] : 0, pq);
            two = two || nq == 2;
            if (nq == 2) {
                pairs.emplace_back(std::min(t[0], t[1]), std::max(t[0], t[1]));
                int np = 0;
                kind_arity(kinds[i], nullptr, &np);
                for (int e = 0; e < m; ++e) {
                    const auto &x = d->xe_edges[e];
                    if (std::min(x.first, x.second) == pairs.back().first &&
                        std::max(x.first, x.second) == pairs.back().second)
                        xon.emplace_back(e, np > 0 ? par[0] : 3.14159265358979323846);
                }
            }
            if (nq == 1 && gd > 0.0 && !d->rabi.empty() && d->rabi[t[0]] > 0.0) drives.emplace_back(t[0], gd);
            for (int j = 0; j < nq; ++j) {
                busy[t[j]] = gd;
                active[t[j]] = 1;
            }
        }
        // off-resonant driving of the batch's passive qubits (eq. off_resonant)
        for (const auto &dv : drives)
            for (int j = 0; j < n; ++j)
                if (!active[j])
                    emit(out, VQD_K_OFFRES, j, 0, d->rabi[dv.first], d->freq[j] - d->freq[dv.first], dv.second);
        // residual exchange on passive edges (eq. weak_dephasing)
        auto passive_edge = [&](int e) {
            return !active[d->xe_edges[e].first] && !active[d->xe_edges[e].second];
        };
        for (const auto &g : xon)
            for (int e = 0; e < m; ++e) {
                const double a = d->xe_on[(size_t)g.first * m + e] * g.second / 3.14159265358979323846;
                if (e != g.first && a != 0.0 && passive_edge(e))
                    emit(out, VQD_K_CRZ, d->xe_edges[e].first, d->xe_edges[e].second, a);
            }
        if (!two)
            for (int e = 0; e < m; ++e)
                if (d->xe_off[e] != 0.0 && passive_edge(e))
                    emit(out, VQD_K_CRZ, d->xe_edges[e].first, d->xe_edges[e].second, d->xe_off[e]);
        if (two && d->alpha != 0.0)
            for (const auto &e : d->edges)
                if (!active[e.first] && !active[e.second]) emit(out, VQD_K_ZZ, e.first, e.second, d->alpha);
        if (dur > 0.0)
            for (size_t k = 0; k < d->zz_edges.size(); ++k) {
                const auto &e = d->zz_edges[k];
                const std::pair<int, int> key(std::min(e.first, e.second), std::max(e.first, e.second));
                if (d->zz_beta[k] == 0.0 || std::find(pairs.begin(), pairs.end(), key) != pairs.end()) continue;
                emit(out, VQD_K_ZZ, e.first, e.second, d->zz_beta[k] * dur);
            }
        for (int q = 0; q < n; ++q) {
            const double idle = dur - busy[q];
            if (!(idle > 0.0)) continue;
            t1_decay(d, out, q, idle);
            t2_decay(d, out, q, idle);
        }
    }
    return write_ops(out, cap, out_count, out_kinds, out_targets, out_params);
}

}  // extern "C"
