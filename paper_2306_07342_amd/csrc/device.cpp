// Virtual-device noise insertion (declarations and contract in
// include/vqd.h): maps an ideal gate list to the noisy op stream of a device
// specification.  Gates are scheduled as soon as possible into parallel
// batches (a gate joins the batch after the last one that uses any of its
// qubits); a batch lasts as long as its slowest gate.  Each batch is
// emitted as its gates in input order, each followed by its active noise
// (depolarising, then dephasing), then ZZ crosstalk on the listed edges
// whose qubits are both idle (when the batch holds a two-qubit gate), then
// passive amp(1 - exp(-dt/T1)) and deph((1 - exp(-dt/T2))/2) for every
// qubit's idle time dt (Secs. 2, 3.4, 3.5; eqs. ampt1, depht2).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "vqd_internal.h"

namespace {

struct GateSpec {
    double duration = 0.0, p_depol = 0.0, p_deph = 0.0;
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
    std::vector<double> T1, T2;
    std::vector<std::pair<int, int>> edges;
    double alpha = 0.0;
};

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
        int b = 0;
        for (int j = 0; j < nq; ++j) b = std::max(b, last[targets[4 * (size_t)i + j]] + 1);
        for (int j = 0; j < nq; ++j) last[targets[4 * (size_t)i + j]] = b;
        batch_of[i] = b;
        n_batches = std::max(n_batches, b + 1);
    }
    std::vector<std::vector<int>> batches(n_batches);
    for (int i = 0; i < count; ++i) batches[batch_of[i]].push_back(i);

    std::vector<Op> out;
    auto emit = [&](int kind, int a, int b, double p0, double p1) {
        Op o{kind, {a, b, 0, 0}, {p0, p1, 0.0, 0.0}};
        out.push_back(o);
    };
    std::vector<double> busy(n);
    std::vector<char> active(n);
    for (const auto &batch : batches) {
        double dur = 0.0;
        bool two = false;
        std::fill(busy.begin(), busy.end(), 0.0);
        std::fill(active.begin(), active.end(), 0);
        for (int i : batch) {
            const GateSpec &g = d->gate[kinds[i]];
            dur = std::max(dur, g.duration);
            int nq = 0;
            kind_arity(kinds[i], &nq, nullptr);
            const int *t = targets + 4 * (size_t)i;
            Op o{kinds[i], {0, 0, 0, 0}, {0.0, 0.0, 0.0, 0.0}};
            for (int j = 0; j < 4; ++j) {
                o.t[j] = t[j];
                o.p[j] = params[4 * (size_t)i + j];
            }
            out.push_back(o);
            if (g.p_depol > 0.0) emit(nq == 1 ? VQD_K_DEPOL1 : VQD_K_DEPOL2, t[0], nq > 1 ? t[1] : 0, g.p_depol, 0.0);
            if (g.p_deph > 0.0) emit(nq == 1 ? VQD_K_DEPH1 : VQD_K_DEPH2, t[0], nq > 1 ? t[1] : 0, g.p_deph, 0.0);
            two = two || nq == 2;
            for (int j = 0; j < nq; ++j) {
                busy[t[j]] = g.duration;
                active[t[j]] = 1;
            }
        }
        if (two && d->alpha != 0.0)
            for (const auto &e : d->edges)
                if (!active[e.first] && !active[e.second]) emit(VQD_K_ZZ, e.first, e.second, d->alpha, 0.0);
        for (int q = 0; q < n; ++q) {
            const double idle = dur - busy[q];
            if (!(idle > 0.0)) continue;
            if (d->T1[q] > 0.0) emit(VQD_K_AMP_T1, q, 0, idle, d->T1[q]);
            if (d->T2[q] > 0.0) emit(VQD_K_DEPH_T2, q, 0, idle, d->T2[q]);
        }
    }
    *out_count = (int)out.size();
    if (!out_kinds && !out_targets && !out_params) return VQD_OK;      // size query
    if (!out_kinds || !out_targets || !out_params) return fail(VQD_E_ARG, "null output array");
    if (cap < (int)out.size()) return fail(VQD_E_SIZE, "output arrays too small");
    for (size_t i = 0; i < out.size(); ++i) {
        out_kinds[i] = out[i].kind;
        for (int j = 0; j < 4; ++j) {
            out_targets[4 * i + j] = out[i].t[j];
            out_params[4 * i + j] = out[i].p[j];
        }
    }
    return VQD_OK;
}

}  // extern "C"
