"""CPU emulation of the pass kernel, driven by descriptors exported from the
library planner (vqd_prog_export).  Test-only: it lets the planner and the
descriptor encoding be checked against the oracle without a GPU.

It reproduces what k_pass does with each descriptor field: the tile/thread/
register-slot address split, dense (column-major) and flip-pattern matrices
with real coefficients packed two per entry, diagonal factors indexed by
register slots or by global bits in each index mode, one-qubit maps in their
Pauli transfer form, phantom bits.  The LDS
exchange between phases only moves values between threads of a tile, so it
is emulated by scattering back to the state and gathering again.
"""
from __future__ import annotations

import numpy as np

MAGIC = 0x56514450
HERM_PASS, HERM_MIRROR, HERM_HALF_IN = 1, 2, 4
HERM_LINE_SHIFT = 4
HERM_STRIDE_SHIFT = 8


def _dtypes(sz_pass, sz_phase, sz_op):
    dpass = np.dtype({"names": ["L", "ngb", "pb", "pe", "phantom", "xcd", "rt_mat", "rt_count",
                                "n_tiles", "group_gpos", "herm"],
                      "formats": ["<u4", "<u4", "<u4", "<u4", "<u4", "<u4", "<u4", "<u4", "<u8",
                                  ("<u4", 32), "<u4"],
                      "offsets": [0, 4, 8, 12, 16, 20, 24, 28, 32, 40, 168], "itemsize": sz_pass})
    dphase = np.dtype({"names": ["ob", "oe", "reg_local", "reg_gpos", "thr_local", "thr_gpos"],
                       "formats": ["<u4", "<u4", ("<u4", 4), ("<u4", 4), ("<u4", 9), ("<u4", 9)],
                       "offsets": [0, 4, 8, 24, 40, 76], "itemsize": sz_phase})
    dop = np.dtype({"names": ["kind", "opmask", "mat", "real", "mode", "nbits", "gpos"],
                    "formats": ["<u4", "<u4", "<u4", "<u4", "<u4", "<u4", ("<u4", 4)],
                    "offsets": [0, 4, 8, 12, 16, 20, 24], "itemsize": sz_op})
    return dpass, dphase, dop


def parse(blob: bytes):
    h = np.frombuffer(blob, dtype="<u4", count=12)
    assert h[0] == MAGIC and h[1] == 1
    npass, nphase, nop, nmat, szp, szh, szo = (int(x) for x in h[2:9])
    dpass, dphase, dop = _dtypes(szp, szh, szo)
    off = 48
    passes = np.frombuffer(blob, dtype=dpass, count=npass, offset=off)
    off += npass * szp
    phases = np.frombuffer(blob, dtype=dphase, count=nphase, offset=off)
    off += nphase * szh
    ops = np.frombuffer(blob, dtype=dop, count=nop, offset=off)
    off += nop * szo
    mats = np.frombuffer(blob, dtype="<f8", count=2 * nmat, offset=off).view(np.complex128)
    return {"n": int(h[9]), "passes": passes, "phases": phases, "ops": ops, "mats": mats}


def _dep4(v, mask):
    out, k = 0, 0
    for b in range(4):
        if mask >> b & 1:
            if v >> k & 1:
                out |= 1 << b
            k += 1
    return out


def _coefs(mats, off, count, real):
    if real:
        packed = mats[off:off + (count + 1) // 2]
        return np.stack([packed.real, packed.imag], axis=1).reshape(-1)[:count].astype(complex)
    return mats[off:off + count]


def _flip(mask, x):
    if mask == 5:
        return 5 if x else 0
    if mask == 10:
        return 10 if x else 0
    return (5 if x & 1 else 0) | (10 if x & 2 else 0)


def herm_tile(flags: int, m: int, t: int):
    """The kernel's launch order in Hermitian mode: launch index t -> (i, j,
    stored).  Blocks (I, J), I <= J < NB = 2^(m-c), folded row I with row
    NB-1-I; members a, b < 2^c s = min(8, blocks) launch indices apart; c and
    s from the flags."""
    c = (flags >> HERM_LINE_SHIFT) & 3
    st = (flags >> HERM_STRIDE_SHIFT) & 15
    NB = 1 << (m - c)
    NBB = NB * (NB + 1) // 2
    q0, lo = t // st, t % st
    k, hi = q0 & ((1 << (2 * c)) - 1), q0 >> (2 * c)
    beta = hi * st + lo
    I = J = 0
    if NB > 1:
        a, b = beta // (NB + 1), beta % (NB + 1)
        if b < NB - a:
            I, J = a, a + b
        else:
            I = NB - 1 - a
            J = I + (b - (NB - a))
    ma, mb = k & ((1 << c) - 1), k >> c
    i, j = (I << c) | ma, (J << c) | mb
    ok = beta < NBB and (I < J or ma <= mb)
    return (i & ((1 << m) - 1), j & ((1 << m) - 1), ok)


def run(plan, amps: np.ndarray) -> np.ndarray:
    """Apply every pass of `plan` to the vectorised state `amps` (complex128)."""
    amps = amps.copy()
    n2 = 2 * plan["n"]
    mats = plan["mats"]
    n = plan["n"]
    prev_pass = None
    for P in plan["passes"]:
        L = int(P["L"])
        nthr_bits = L - 4
        T = int(P["n_tiles"])
        ngb = int(P["ngb"])
        herm = bool(P["herm"])
        if herm:
            # Hermitian mode: the group pairs i <= j, i in the row group bits and
            # j in the column group bits; tiles with i < j also write their mirror
            m = ngb // 2
            N = 1 << m
            pairs = [(i, j) for t in range(T) for (i, j, ok) in [herm_tile(int(P["herm"]), m, t)] if ok]
            assert sorted(pairs) == [(i, j) for i in range(N) for j in range(i, N)]
            T = len(pairs)
            gb = np.zeros(T, dtype=np.uint64)
            for t, (i, j) in enumerate(pairs):
                for k in range(m):
                    gb[t] |= np.uint64(((i >> k) & 1) << int(P["group_gpos"][k]))
                    gb[t] |= np.uint64(((j >> k) & 1) << int(P["group_gpos"][m + k]))
            mirror = np.array([i != j for i, j in pairs])
            flags = int(P["herm"])
            assert flags & HERM_PASS
        else:
            gb = np.zeros(T, dtype=np.uint64)
            tiles = np.arange(T, dtype=np.uint64)
            for i in range(ngb):
                gb |= ((tiles >> np.uint64(i)) & np.uint64(1)) << np.uint64(P["group_gpos"][i])
        for ph in range(int(P["pb"]), int(P["pe"])):
            H = plan["phases"][ph]
            thr = np.arange(1 << nthr_bits, dtype=np.uint64)
            tg = np.zeros_like(thr)
            for i in range(nthr_bits):
                tg |= ((thr >> np.uint64(i)) & np.uint64(1)) << np.uint64(H["thr_gpos"][i])
            rg = [np.uint64(1) << np.uint64(H["reg_gpos"][b]) for b in range(4)]
            slot = np.zeros(16, dtype=np.uint64)
            for e in range(16):
                for b in range(4):
                    if e >> b & 1:
                        slot[e] |= rg[b]
            base = gb[:, None] | tg[None, :]                       # (T, threads)
            gidx = base[:, :, None] | slot[None, None, :]          # (T, threads, 16)
            valid = (gidx >> np.uint64(n2)) == 0
            gi = np.where(valid, gidx, 0).astype(np.int64)
            a = np.where(valid, amps[gi], 0)
            if herm and ph == int(P["pb"]) and flags & HERM_HALF_IN:
                # the previous pass stored only its group pairs i <= j: the
                # others come from the transposed index, conjugated
                Pp = prev_pass
                mp = int(Pp["ngb"]) // 2
                gu = gidx.astype(np.uint64)
                ip = np.zeros(gu.shape, dtype=np.int64)
                jp = np.zeros(gu.shape, dtype=np.int64)
                for k in range(mp):
                    ip |= ((gu >> np.uint64(Pp["group_gpos"][k])) & np.uint64(1)).astype(np.int64) << k
                    jp |= ((gu >> np.uint64(Pp["group_gpos"][mp + k])) & np.uint64(1)).astype(np.int64) << k
                D = np.uint64((1 << n) - 1)
                mu = ((gu >> np.uint64(n)) | ((gu & D) << np.uint64(n))).astype(np.int64)
                a = np.where(ip > jp, np.conj(amps[mu]), a)
            for oi in range(int(H["ob"]), int(H["oe"])):
                op = plan["ops"][oi]
                kind, mask, real = int(op["kind"]), int(op["opmask"]), bool(op["real"])
                if kind in (1, 2):
                    nb = bin(mask).count("1")
                    dim = 1 << nb
                    rest = (~mask) & 15
                    y = np.zeros_like(a)
                    if kind == 1:          # dense, column-major
                        C = _coefs(mats, int(op["mat"]), dim * dim, real)
                        for j in range(dim):
                            for i in range(dim):
                                for g in range(16 >> nb):
                                    so = _dep4(i, mask) | _dep4(g, rest)
                                    si = _dep4(j, mask) | _dep4(g, rest)
                                    y[..., so] += C[j * dim + i] * a[..., si]
                    else:                  # flip pattern
                        nx = 4 if mask == 15 else 2
                        W = _coefs(mats, int(op["mat"]), nx * dim, real)
                        for x in range(nx):
                            for i in range(dim):
                                for g in range(16 >> nb):
                                    so = _dep4(i, mask) | _dep4(g, rest)
                                    y[..., so] += W[x * dim + i] * a[..., so ^ _flip(mask, x)]
                    a = y
                elif kind == 5:            # Pauli transfer form of a trace-preserving one-qubit map
                    H5 = _coefs(mats, int(op["mat"]), 12, True).real.reshape(3, 4)
                    H5 = np.vstack([[0.5, 0.0, 0.0, 0.0], H5])
                    rest = (~mask) & 15
                    y = np.zeros_like(a)
                    for g in range(4):
                        s0, s1, s2, s3 = (_dep4(l, mask) | _dep4(g, rest) for l in range(4))
                        # block B[u][v] at local index u + 2v; components Tr(P B)
                        comp = np.stack([a[..., s0] + a[..., s3], a[..., s1] + a[..., s2],
                                         1j * (a[..., s2] - a[..., s1]), a[..., s0] - a[..., s3]])
                        h = np.tensordot(H5, comp, axes=(1, 0))
                        y[..., s0] = h[0] + h[3]
                        y[..., s3] = h[0] - h[3]
                        y[..., s2] = h[1] - 1j * h[2]
                        y[..., s1] = h[1] + 1j * h[2]
                    a = y
                elif kind == 3:
                    F = _coefs(mats, int(op["mat"]), 16, real)
                    a = a * F[None, None, :]
                elif kind == 4:
                    T = mats[int(P["rt_mat"]) + int(op["mat"]):]
                    rt = np.zeros(gidx.shape, dtype=np.int64)
                    mode = int(op["mode"])
                    src = gidx if mode == 3 else np.broadcast_to(base[:, :, None], gidx.shape)
                    for j in range(int(op["nbits"])):
                        rt |= ((src >> np.uint64(op["gpos"][j])) & np.uint64(1)).astype(np.int64) << j
                    if mode in (1, 2):
                        r0 = 0 if mode == 1 else 1
                        e = np.arange(16)
                        c = ((e >> r0) & 1) | (((e >> (r0 + 2)) & 1) << 1)
                        idx = c[None, None, :] + 4 * rt
                    else:
                        idx = rt
                    a = a * T[idx]
                else:
                    raise AssertionError("unknown kernel op kind %d" % kind)
            amps[gi[valid]] = a[valid]
        prev_pass = P
        if herm and flags & HERM_MIRROR:
            # the conjugate transpose of each tile with i < j into its mirror
            idx = gi[mirror].reshape(-1).astype(np.uint64)
            D = np.uint64((1 << n) - 1)
            mu = (idx >> np.uint64(n)) | ((idx & D) << np.uint64(n))
            amps[mu.astype(np.int64)] = np.conj(amps[idx.astype(np.int64)])
    return amps
