// Measurement on the density matrix (declarations and contract in
// include/vqd.h): projective Z and parity measurements with collapse, and
// shot sampling from the diagonal.
#include <cmath>
#include <string>

#include "vqd_internal.h"

using namespace vqd;

namespace {

// The draw rule of the library: outcome 0 if its weight exceeds u W, else 1
// (the second weight if the first is not positive and rounding leaves none).
int draw2(double w0, double w1, double u)
{
    const double W = w0 + w1;
    const double thr = u * W;
    if (w0 > thr) return 0;
    if (w0 + w1 > thr) return 1;
    return (w1 > 0.0) ? 1 : 0;
}

int finish(vqd_dm *dm, int kind, int q0, int q1, double w0, double w1, double u, int *outcome, double *weight)
{
    if (!(w0 > 0.0) && !(w1 > 0.0)) return fail(VQD_E_STATE, "the state has no weight on either outcome");
    const int m = draw2(w0, w1, u);
    const double w = m ? w1 : w0;
    if (int rc = launch_project(dm->amps, dm->n, kind, q0, q1, m, 1.0 / w, dm->stream)) return rc;
    *outcome = m;
    if (weight) *weight = w;
    return VQD_OK;
}

int check_u(double u)
{
    if (!(u >= 0.0 && u < 1.0)) return fail(VQD_E_ARG, "u must lie in [0, 1)");
    return VQD_OK;
}

}  // namespace

extern "C" {

int vqd_measure_z(vqd_dm *dm, int q, double u, int *outcome, double *weight)
{
    clear_error();
    if (!dm || !dm->amps) return fail(VQD_E_ARG, "null density-matrix handle");
    if (!outcome) return fail(VQD_E_ARG, "null outcome");
    if (int rc = check_targets(dm->n, 1, &q)) return rc;
    if (int rc = check_u(u)) return rc;
    double tr[2];
    std::vector<double> z(dm->n);
    if (int rc = reduce_diag(dm->amps, dm->n, dm->red, dm->stream, tr, z.data(), nullptr)) return rc;
    // weights of |0> and |1> on q from the trace and <Z_q>
    return finish(dm, MEAS_Z, q, q, 0.5 * (tr[0] + z[q]), 0.5 * (tr[0] - z[q]), u, outcome, weight);
}

int vqd_measure_parity(vqd_dm *dm, int q0, int q1, double u, int *outcome, double *weight)
{
    clear_error();
    if (!dm || !dm->amps) return fail(VQD_E_ARG, "null density-matrix handle");
    if (!outcome) return fail(VQD_E_ARG, "null outcome");
    const int t[2] = {q0, q1};
    if (int rc = check_targets(dm->n, 2, t)) return rc;
    if (int rc = check_u(u)) return rc;
    double tr[2], zz = 0.0;
    if (int rc = reduce_diag(dm->amps, dm->n, dm->red, dm->stream, tr, nullptr, nullptr)) return rc;
    if (int rc = reduce_zz(dm->amps, dm->n, t, 1, dm->red, dm->stream, &zz)) return rc;
    // outcome "0": odd parity, weight (tr - <ZZ>)/2; "1": even, (tr + <ZZ>)/2
    return finish(dm, MEAS_PARITY, q0, q1, 0.5 * (tr[0] - zz), 0.5 * (tr[0] + zz), u, outcome, weight);
}

int vqd_sample(vqd_dm *dm, const double *uniforms, long long shots, uint32_t *out)
{
    clear_error();
    if (!dm || !dm->amps) return fail(VQD_E_ARG, "null density-matrix handle");
    if (shots < 0) return fail(VQD_E_ARG, "negative shot count");
    if (shots > 0 && (!uniforms || !out)) return fail(VQD_E_ARG, "null uniforms or output");
    const size_t D = size_t(1) << dm->n;
    if (int rc = ensure_scratch(dm->red, 2 * D + 1, 0)) return rc;
    return launch_sample(dm->amps, dm->n, dm->red.dev, uniforms, (uint64_t)shots, out, dm->stream);
}

}  // extern "C"
