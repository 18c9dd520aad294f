// Device presets: the parameter tables of the paper's virtual devices (App.
// C) turned into device-layer specifications (declarations and contract in
// include/vqd.h).  Units as in App. C: microseconds and megahertz.
//
// Superconducting (Sec. 8, table conf:scq): six transmons.  Gates are ideal
// (the model's errors are all passive); Rx and Ry (and the other one-qubit
// rotations, which the device realises with them) take 0.05 us, Z rotations
// are frame changes and take no time, two-qubit gates (cross-resonance ZX,
// siZZle ZZ) take 0.5 us.  Passive noise: T1 relaxation towards the thermal
// state the qubits are initialised in (eqs. thermalstate, gdamp), T2
// dephasing (eq. depht2), and the static ZZ coupling of every capacitively
// coupled pair, beta = J^2 (1/(Delta - alpha_t) - 1/(Delta + alpha_c)) in
// MHz, applied as a phase of 2 pi beta per microsecond except while a
// two-qubit gate drives that pair.  Read-out: T1 decay for the 5 us
// measurement and depolarising noise of the read-out infidelity 1 - F on
// either side of the projection.
//
// Trapped ions (Sec. 4, table conf:trapped_ions): two nodes of four ions in
// one register (qubits 0-3 and 4-7).  Passive noise: T1 amplitude damping
// and Gaussian T2* dephasing (eq. depht2s).  x and y rotations: depolarising
// noise from the reported fidelity (App. B), scaled with the duration by
// |theta| / pi (App. C); a pi rotation takes 1 / (2 x Rabi frequency).  CZ:
// the reported fidelity split 0.1 : 0.9 into depolarising and dephasing
// noise, duration 1 / (2 x its gate frequency).  Read-out: a symmetric bit
// flip of the tabulated probability before the projection (eq. bf), 50 us
// during which the other ions idle.  Ion transport and remote entanglement
// are not part of the preset.
//
// Silicon (Sec. 7, table conf:silicon): six spin qubits in a line, gates run
// one at a time.  x and y rotations: pure dephasing from the per-qubit
// fidelity (error ratio 0:1), 1 / (2 x Rabi frequency) per pi, noise and
// duration scaled by |theta| / pi; they drive the other qubits off
// resonance (eq. off_resonant) with the 5 MHz Rabi frequency and the qubit
// frequencies of the table.  CZ (and CPhase, scaled by |theta| / pi) on the
// five neighbouring pairs: two-qubit dephasing from the per-pair fidelity,
// 1 / (2 x the pair's gate frequency).  Residual exchange on passive
// neighbouring pairs as conditional Z rotations (eq. weak_dephasing): the
// ExchangeRotOn matrix while a CZ or CPhase runs, ExchangeRotOff otherwise.
// Passive noise: depolarising T1 decay (eq. depolt1) and T2 dephasing.
// Parity read-out: bit flips with b = 1 - the read-out fidelity around the
// decaying parity projection, 10 us during which the other qubits idle.
#include <cmath>
#include <string>

#include "vqd_internal.h"

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

int superconducting(vqd_device **out, double *p0)
{
    constexpr int n = 6;
    const double T1[n] = {63, 93, 109, 115, 68, 125};
    const double T2[n] = {113, 149, 185, 161, 122, 200};
    const double excited[n] = {3.2e-2, 2.1e-2, 0.8e-2, 0.9e-2, 2.5e-2, 0.7e-2};
    const double freq[n] = {4.5e3, 4.9e3, 4.7e3, 5.1e3, 4.9e3, 5.3e3};
    const double anharm[n] = {296.7, 298.6, 297.4, 298.3, 297.2, 299.1};
    const double fid_read[n] = {0.9, 0.92, 0.96, 0.97, 0.93, 0.97};
    const int pairs[7][2] = {{0, 1}, {0, 2}, {1, 3}, {2, 3}, {2, 4}, {3, 5}, {4, 5}};
    const double J[7] = {4, 1.5, 1.5, 4, 1.5, 1.5, 4};
    const double t_meas = 5.0, t_1q = 0.05, t_2q = 0.5;

    vqd_device *d = nullptr;
    if (int rc = vqd_device_create(n, &d)) return rc;
    double ground[n], eps[n], beta[7];
    int edges[14];
    for (int q = 0; q < n; ++q) {
        ground[q] = 1.0 - excited[q];
        eps[q] = 1.0 - fid_read[q];
    }
    for (int e = 0; e < 7; ++e) {
        const int c = pairs[e][0], t = pairs[e][1];
        edges[2 * e] = c;
        edges[2 * e + 1] = t;
        double b = 0.0;
        if (int rc = vqd_zz_crosstalk_strength(J[e], freq[c] - freq[t], anharm[c], anharm[t], &b)) {
            vqd_device_destroy(d);
            return rc;
        }
        beta[e] = kTwoPi * b;
    }
    int rc = VQD_OK;
    for (int k : {VQD_K_RX, VQD_K_RY, VQD_K_H, VQD_K_X, VQD_K_Y, VQD_K_SU2})
        if (!rc) rc = vqd_device_set_gate(d, k, t_1q, 0.0, 0.0);
    for (int k : {VQD_K_CZ, VQD_K_CPHASE, VQD_K_XX, VQD_K_ZZ})
        if (!rc) rc = vqd_device_set_gate(d, k, t_2q, 0.0, 0.0);
    if (!rc) rc = vqd_device_set_passive(d, T1, T2);
    if (!rc) rc = vqd_device_set_thermal(d, ground);
    if (!rc) rc = vqd_device_set_static_zz(d, 7, edges, beta);
    if (!rc) rc = vqd_device_set_readout(d, t_meas, eps);
    if (rc) {
        vqd_device_destroy(d);
        return rc;
    }
    if (p0)
        for (int q = 0; q < n; ++q) p0[q] = ground[q];
    *out = d;
    return VQD_OK;
}

int trapped_ion(vqd_device **out, double *p0)
{
    constexpr int n = 8;
    const double T1 = 3e9, T2s = 10e5, fid_init = 0.9999;
    const double fid_xy = 0.99999, x_xy = 1.0, rabi = 10.0;
    const double fid_cz = 0.999, x_cz = 0.1, freq_cz = 0.1;
    const double t_read = 50.0, bf_read = 0.001;

    vqd_device *d = nullptr;
    if (int rc = vqd_device_create(n, &d)) return rc;
    double t1[n], t2[n];
    for (int q = 0; q < n; ++q) {
        t1[q] = T1;
        t2[q] = T2s;
    }
    double pd1 = 0, pq1 = 0, pd2 = 0, pq2 = 0;
    int rc = vqd_fidelity_to_errors(1, fid_xy, x_xy, &pd1, &pq1);
    if (!rc) rc = vqd_fidelity_to_errors(2, fid_cz, x_cz, &pd2, &pq2);
    const double t_pi = 1.0 / (2.0 * rabi), t_cz = 1.0 / (2.0 * freq_cz);
    for (int k : {VQD_K_RX, VQD_K_RY}) {
        if (!rc) rc = vqd_device_set_gate(d, k, t_pi, pd1, pq1);
        if (!rc) rc = vqd_device_set_angle_scaling(d, k, 1, 1);
    }
    for (int k : {VQD_K_H, VQD_K_X, VQD_K_Y})     // pi rotations
        if (!rc) rc = vqd_device_set_gate(d, k, t_pi, pd1, pq1);
    if (!rc) rc = vqd_device_set_gate(d, VQD_K_CZ, t_cz, pd2, pq2);
    if (!rc) rc = vqd_device_set_passive(d, t1, t2);
    if (!rc) rc = vqd_device_set_passive_forms(d, VQD_K_AMP_T1, VQD_K_DEPH_T2S);
    double eps[n];
    for (int q = 0; q < n; ++q) eps[q] = bf_read;
    if (!rc) rc = vqd_device_set_readout(d, t_read, eps);
    if (!rc) rc = vqd_device_set_readout_form(d, VQD_K_BITFLIP1);
    if (rc) {
        vqd_device_destroy(d);
        return rc;
    }
    if (p0)
        for (int q = 0; q < n; ++q) p0[q] = fid_init;
    *out = d;
    return VQD_OK;
}

int silicon(vqd_device **out, double *p0)
{
    constexpr int n = 6, np = n - 1;
    const double T1 = 1e4;
    const double T2[n] = {14, 21.1, 40.1, 37.2, 44.7, 26.7};
    const double qfreq[n] = {15.62e3, 15.88e3, 16.3e3, 16.1e3, 15.9e3, 15.69e3};
    const double rabi = 5.0;
    const double fid_xy[n] = {0.9977, 0.9987, 0.9996, 0.9988, 0.9991, 0.9989};
    const double freq_cz[np] = {12.1, 11.1, 6.6, 9.8, 5.4};
    const double fid_cz[np] = {0.937, 0.934, 0.929, 0.997, 0.979};
    const double rot_on[np * np] = {0, 0.023, 0.018, 0.03, 0.04,
                                    0.05, 0, 0.03, 0.03, 0.04,
                                    0.05, 0.03, 0, 0.07, 0.042,
                                    0.038, 0.03, 0.031, 0, 0.25,
                                    0.033, 0.03, 0.02, 0.03, 0};
    const double rot_off[np] = {0.039, 0.015, 0.03, 0.02, 0.028};
    const double fid_read = 0.99, t_read = 10.0;

    vqd_device *d = nullptr;
    if (int rc = vqd_device_create(n, &d)) return rc;
    double t1[n], w_rabi[n], w_q[n];
    int edges[2 * np];
    for (int q = 0; q < n; ++q) {
        t1[q] = T1;
        w_rabi[q] = kTwoPi * rabi;
        w_q[q] = kTwoPi * qfreq[q];
    }
    const double t_pi = 1.0 / (2.0 * rabi);
    int rc = VQD_OK;
    for (int q = 0; q < n && !rc; ++q) {
        double pd = 0, pq = 0;
        rc = vqd_fidelity_to_errors(1, fid_xy[q], 0.0, &pd, &pq);
        for (int k : {VQD_K_RX, VQD_K_RY, VQD_K_H, VQD_K_X, VQD_K_Y})
            if (!rc) rc = vqd_device_set_gate_on(d, k, 1, &q, t_pi, pd, pq);
    }
    for (int k : {VQD_K_RX, VQD_K_RY, VQD_K_CPHASE})
        if (!rc) rc = vqd_device_set_angle_scaling(d, k, 1, 1);
    for (int e = 0; e < np && !rc; ++e) {
        edges[2 * e] = e;
        edges[2 * e + 1] = e + 1;
        double pd = 0, pq = 0;
        rc = vqd_fidelity_to_errors(2, fid_cz[e], 0.0, &pd, &pq);
        for (int k : {VQD_K_CZ, VQD_K_CPHASE})
            if (!rc) rc = vqd_device_set_gate_on(d, k, 2, edges + 2 * e, 1.0 / (2.0 * freq_cz[e]), pd, pq);
    }
    if (!rc) rc = vqd_device_set_passive(d, t1, T2);
    if (!rc) rc = vqd_device_set_passive_forms(d, VQD_K_DEPOL_T1, VQD_K_DEPH_T2);
    if (!rc) rc = vqd_device_set_off_resonant(d, w_rabi, w_q);
    if (!rc) rc = vqd_device_set_exchange_crosstalk(d, np, edges, rot_on, rot_off);
    if (!rc) rc = vqd_device_set_serial(d, 1);
    if (!rc) rc = vqd_device_set_parity_readout(d, t_read, 1.0 - fid_read);
    if (rc) {
        vqd_device_destroy(d);
        return rc;
    }
    if (p0)
        for (int q = 0; q < n; ++q) p0[q] = 1.0;
    *out = d;
    return VQD_OK;
}

}  // namespace

using namespace vqd;

extern "C" {

int vqd_device_preset(int preset, vqd_device **out, double *p0)
{
    clear_error();
    if (!out) return fail(VQD_E_ARG, "null output pointer");
    *out = nullptr;
    int rc;
    switch (preset) {
    case VQD_PRESET_SUPERCONDUCTING: rc = superconducting(out, p0); break;
    case VQD_PRESET_TRAPPED_ION: rc = trapped_ion(out, p0); break;
    case VQD_PRESET_SILICON: rc = silicon(out, p0); break;
    default: return fail(VQD_E_ARG, "unknown preset " + std::to_string(preset));
    }
    return rc;
}

int vqd_device_preset_qubits(int preset, int *n)
{
    clear_error();
    if (!n) return fail(VQD_E_ARG, "null output pointer");
    switch (preset) {
    case VQD_PRESET_SUPERCONDUCTING: *n = 6; return VQD_OK;
    case VQD_PRESET_TRAPPED_ION: *n = 8; return VQD_OK;
    case VQD_PRESET_SILICON: *n = 6; return VQD_OK;
    default: return fail(VQD_E_ARG, "unknown preset " + std::to_string(preset));
    }
}

}  // extern "C"
