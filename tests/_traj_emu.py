"""CPU execution of exported trajectory plans (vqd_traj_export).

Test infrastructure: decodes the library's phase/op descriptors and runs
them on full state vectors with numpy, op by op, with the kernel's rules
(mixed-unitary channels drawn from their stored weights, general ones from
Tr(K^dagger K rho_T) of the reduced density matrix of the targets).  It
checks the host planner's encoding (register masks, bit orders, packing,
channel order) without a GPU; the register and LDS mechanics of the kernel
are left to the GPU tests.
"""
from __future__ import annotations

import math

import numpy as np

from oracle.trajectories import apply_matrix

MAGIC = 0x54445156
TOP_MAT, TOP_DTHR, TOP_MIX, TOP_KRAUS, TOP_DREG, TOP_DMIX, TOP_DRM, TOP_DMIX2, TOP_MATS = 1, 2, 3, 4, 5, 6, 7, 8, 9

PHASE = np.dtype([("ob", "<u4"), ("oe", "<u4"), ("reg", "<u4", 4), ("thr", "<u4", 9), ("flags", "<u4")])
PHASE_REDUCES = 1
OP = np.dtype([("kind", "<u4"), ("mask", "<u4"), ("mat", "<u4"), ("real", "<u4"), ("nk", "<u4"),
               ("chan", "<u4"), ("nd", "<u4"), ("dmask", "<u4"), ("dq", "<u4", 2), ("rmask", "<u4"),
               ("gdiag", "<u4"), ("inl", "<u4"), ("grp", "<u4"), ("pad", "<u4", 2), ("cf", "<f8", 6)])


def parse(blob: bytes) -> dict:
    h = np.frombuffer(blob, dtype="<u4", count=10)
    assert h[0] == MAGIC and h[1] == 1
    n, ne, nch, nph, nop, npool, szp, szo = (int(x) for x in h[2:10])
    assert szp >= PHASE.itemsize and szo == OP.itemsize
    off = 40
    # the phase records may carry fields past the ones read here (kernel tables)
    dph = np.dtype({"names": list(PHASE.names), "formats": [PHASE.fields[k][0] for k in PHASE.names],
                    "offsets": [PHASE.fields[k][1] for k in PHASE.names], "itemsize": szp})
    phases = np.frombuffer(blob, dtype=dph, count=nph, offset=off)
    off += nph * szp
    ops = np.frombuffer(blob, dtype=OP, count=nop, offset=off)
    off += nop * szo
    pool = np.frombuffer(blob, dtype="<f8", count=2 * npool, offset=off).view(np.complex128)
    return {"n": n, "n_eff": ne, "n_channels": nch, "phases": phases, "ops": ops, "pool": pool}


def _qubits(mask, reg):
    return [int(reg[b]) for b in range(4) if (int(mask) >> b) & 1]


def _colmajor(pool, off, d):
    return pool[off:off + d * d].reshape(d, d).T


def _mat(pool, op, d):
    off = int(op["mat"])
    if op["real"]:
        packed = pool[off:off + (d * d + 1) // 2]
        c = np.stack([packed.real, packed.imag], axis=1).reshape(-1)[:d * d].astype(complex)
        return c.reshape(d, d).T
    return _colmajor(pool, off, d)


def _reduced(psi, qs):
    n = int(psi.size).bit_length() - 1
    mask = sum(1 << q for q in qs)
    x = np.arange(psi.size)
    base = x[(x & mask) == 0]
    off = np.array([sum(((l >> j) & 1) << q for j, q in enumerate(qs)) for l in range(1 << len(qs))])
    A = psi[base[:, None] | off[None, :]]
    del n
    return A.T @ A.conj()


def _draw(w, u):
    W = 0.0
    for x in w:
        W += x
    thr = u * W
    cum = 0.0
    for i, x in enumerate(w):
        cum += x
        if cum > thr:
            return i
    return max(i for i, x in enumerate(w) if x > 0)


def _group(psi, members, reg, urow):
    """A marked run of inline one-qubit channels drawn the way trajectories
    of whole waves draw it: every damping member's weights from the run's
    input populations (times the no-jump Gram factors of the damping members
    before it), one product of diagonal factors, one normalisation.  The
    damping members are trace preserving, so member k's total weight is the
    previous running sum C_k.  Returns (state, members applied): when a
    damping member draws its jump only the members before it are applied
    (the kernel takes the rest one by one, from that member); (None, 0) when
    the first member jumps."""
    x = np.arange(psi.size)
    bits = [(x >> int(reg[int(m["mask"]).bit_length() - 1])) & 1 for m in members]
    q = np.abs(psi) ** 2
    C = [float(np.sum(q))]
    for m, b in zip(members, bits):
        if int(m["kind"]) == TOP_KRAUS:
            cf = m["cf"]
            assert abs(cf[0] + cf[2] - 1) <= 1e-15 and abs(cf[1] + cf[3] - 1) <= 1e-15
            q = q * np.where(b == 1, cf[1], cf[0])
            C.append(float(np.sum(q)))
    f = np.ones(psi.size)
    last, kk = 1.0, 0
    for i, (m, b) in enumerate(zip(members, bits)):
        cf, u = m["cf"], float(urow[int(m["chan"])])
        if int(m["kind"]) == TOP_MIX:
            j = cf[0] <= u * cf[1]
            f0, f1 = (cf[4], cf[5]) if j else (cf[2], cf[3])
        else:
            tot, c = C[kk], C[kk + 1]
            d = tot - c
            thr = u * tot
            if not (c > thr) and (tot > thr or d > 0.0):
                if i == 0:
                    return None, 0
                return psi * f / (math.sqrt(last) if kk else 1.0), i
            last, kk = c, kk + 1
            f0, f1 = cf[4], cf[5]
        f = f * np.where(b == 1, f1, f0)
    return psi * f / math.sqrt(last), len(members)


def run(plan: dict, U: np.ndarray, groups: bool = False, stats: dict = None):
    """Per-trajectory <Z_q> (T x n), squared norms (T) and the channel order
    met (one list of channel indices).  groups: draw the marked runs of
    inline channels as trajectories of whole waves do (counted in stats:
    'grouped' runs, 'fallback' runs with a jump)."""
    n, ne, pool = plan["n"], plan["n_eff"], plan["pool"]
    T = U.shape[0]
    Z = np.empty((T, n))
    N = np.empty(T)
    order = []
    if stats is not None:
        stats.setdefault("grouped", 0)
        stats.setdefault("fallback", 0)
    for t in range(T):
        psi = np.zeros(1 << ne, dtype=complex)
        psi[0] = 1
        for ph in plan["phases"]:
            # the flag that lets the kernel drop an exchange barrier
            kinds = [int(o["kind"]) for o in plan["ops"][int(ph["ob"]):int(ph["oe"])]]
            assert bool(int(ph["flags"]) & PHASE_REDUCES) == (TOP_KRAUS in kinds)
            skip = 0
            for idx in range(int(ph["ob"]), int(ph["oe"])):
                if skip:
                    skip -= 1
                    continue
                op = plan["ops"][idx]
                k = int(op["grp"])
                if groups and k > 1:
                    members = plan["ops"][idx:idx + k]
                    out, used = _group(psi, members, ph["reg"], U[t])
                    if stats is not None:
                        stats["grouped" if used == k else "fallback"] += 1
                    if used:
                        psi = out
                        skip = used - 1
                        if t == 0:
                            order.extend(int(m["chan"]) for m in members[:used])
                        continue
                kind = int(op["kind"])
                if kind == TOP_DTHR:
                    qs = [int(q) for q in op["dq"][:int(op["nd"])]]
                    assert not set(qs) & set(int(q) for q in ph["reg"])
                    f = pool[int(op["mat"]):int(op["mat"]) + (1 << len(qs))]
                    psi = apply_matrix(psi, qs, np.diag(f))
                    continue
                if kind == TOP_DREG:
                    # 16 factors by register slot: the diagonal on the four register qubits
                    f = pool[int(op["mat"]):int(op["mat"]) + 16]
                    if op["real"]:
                        assert np.all(f.imag == 0)
                    psi = apply_matrix(psi, [int(q) for q in ph["reg"]], np.diag(f))
                    continue
                if kind == TOP_MATS:
                    # nd one-qubit matrices: register bit (dmask >> 2j) & 3, 2x2 column-major
                    assert 2 <= int(op["nd"]) <= 4
                    for j in range(int(op["nd"])):
                        b = (int(op["dmask"]) >> (2 * j)) & 3
                        off = int(op["mat"]) + 4 * j
                        psi = apply_matrix(psi, [int(ph["reg"][b])], pool[off:off + 4].reshape(2, 2).T)
                    continue
                if kind == TOP_DMIX2:
                    # two TOP_DMIX: register bits mask and dmask, thread qubits dq
                    f = pool[int(op["mat"]):int(op["mat"]) + 8]
                    for j, m in enumerate((op["mask"], op["dmask"])):
                        qr = _qubits(m, ph["reg"])
                        assert len(qr) == 1
                        psi = apply_matrix(psi, [qr[0], int(op["dq"][j])], np.diag(f[4 * j:4 * j + 4]))
                    continue
                if kind == TOP_DRM:
                    # 16 factors by register slot, then a TOP_DMIX's four
                    f = pool[int(op["mat"]):int(op["mat"]) + 20]
                    psi = apply_matrix(psi, [int(q) for q in ph["reg"]], np.diag(f[:16]))
                    qr = _qubits(op["mask"], ph["reg"])
                    assert len(qr) == 1
                    psi = apply_matrix(psi, [qr[0], int(op["dq"][0])], np.diag(f[16:20]))
                    continue
                if kind == TOP_DMIX:
                    # factor index: register qubit the low bit, thread qubit the high bit
                    qr = _qubits(op["mask"], ph["reg"])
                    assert len(qr) == 1
                    qt = int(op["dq"][0])
                    f = pool[int(op["mat"]):int(op["mat"]) + 4]
                    psi = apply_matrix(psi, [qr[0], qt], np.diag(f))
                    continue
                qs = _qubits(op["mask"], ph["reg"])
                d = 1 << len(qs)
                if kind == TOP_MAT:
                    psi = apply_matrix(psi, qs, _mat(pool, op, d))
                    continue
                nk, off = int(op["nk"]), int(op["mat"])
                if t == 0:
                    order.append(int(op["chan"]))
                if kind == TOP_MIX:
                    w = list(pool[off:off + nk].imag)
                    assert np.array_equal(pool[off:off + nk].real, np.cumsum(w))
                    mats = off + nk
                else:
                    rho = _reduced(psi, qs)
                    w = [float(np.sum(pool[off + i * d * d: off + (i + 1) * d * d].reshape(d, d) * rho.T).real)
                         for i in range(nk)]
                    mats = off + nk * d * d
                if t == 0:
                    # the per-operator flags the kernel's fast paths rely on
                    for i in range(nk):
                        K = _colmajor(pool, mats + i * d * d, d)
                        isdiag = np.count_nonzero(K - np.diag(np.diag(K))) == 0
                        assert bool((int(op["dmask"]) >> i) & 1) == isdiag
                        assert bool((int(op["rmask"]) >> i) & 1) == (isdiag and np.all(np.diag(K).imag == 0))
                    if kind == TOP_KRAUS:
                        G = [pool[off + i * d * d: off + (i + 1) * d * d].reshape(d, d) for i in range(nk)]
                        assert bool(op["gdiag"]) == all(np.count_nonzero(g - np.diag(np.diag(g))) == 0 for g in G)
                j = _draw(w, float(U[t, int(op["chan"])]))
                psi = apply_matrix(psi, qs, _colmajor(pool, mats + j * d * d, d))
                if kind == TOP_KRAUS:
                    psi = psi / math.sqrt(w[j])
        p = np.abs(psi) ** 2
        x = np.arange(psi.size)
        Z[t] = [np.sum(p * (1 - 2 * ((x >> q) & 1))) for q in range(n)]
        N[t] = p.sum()
    return Z, N, order
