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
                                "n_tiles", "group_gpos", "herm", "out_gpos", "swap_out"],
                      "formats": ["<u4", "<u4", "<u4", "<u4", "<u4", "<u4", "<u4", "<u4", "<u8",
                                  ("<u4", 32), "<u4", ("<u4", 32), "<u4"],
                      "offsets": [0, 4, 8, 12, 16, 20, 24, 28, 32, 40, 168, 300, 428], "itemsize": sz_pass})
    dphase = np.dtype({"names": ["ob", "oe", "reg_local", "reg_gpos", "thr_local", "thr_gpos", "reg_mpos",
                                 "thr_mpos"],
                       "formats": ["<u4", "<u4", ("<u4", 4), ("<u4", 4), ("<u4", 9), ("<u4", 9), ("<u4", 4),
                                   ("<u4", 9)],
                       "offsets": [0, 4, 8, 24, 40, 76, 304, 320], "itemsize": sz_phase})
    dop = np.dtype({"names": ["kind", "opmask", "mat", "real", "mode", "nbits", "gpos", "lpos"],
                    "formats": ["<u4", "<u4", "<u4", "<u4", "<u4", "<u4", ("<u4", 4), ("<u4", 4)],
                    "offsets": [0, 4, 8, 12, 16, 20, 24, 40], "itemsize": sz_op})
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


def _bits(values, positions, count):
    """Index with bit positions[i] set where bit i of values is set."""
    out = np.zeros(values.shape, dtype=np.uint64)
    for i in range(count):
        out |= ((values >> np.uint64(i)) & np.uint64(1)) << np.uint64(positions[i])
    return out


def _mirror(idx, n):
    D = np.uint64((1 << n) - 1)
    return (idx >> np.uint64(n)) | ((idx & D) << np.uint64(n))


def _apply_op(op, a, mats, P, li, gb, tl):
    """One kernel op on a[tiles, threads, 16]; li, tl: local index of each
    element and of its thread part; gb: the tiles' group bases."""
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
        return y
    if kind == 5:              # Pauli transfer form of a trace-preserving one-qubit map
        H5 = np.vstack([[0.5, 0.0, 0.0, 0.0], _coefs(mats, int(op["mat"]), 12, True).real.reshape(3, 4)])
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
        return y
    if kind == 3:
        return a * _coefs(mats, int(op["mat"]), 16, real)[None, None, :]
    if kind == 4:
        # table index bit j: from the group base at gpos[j], or from local
        # index bit lpos[j] (of the thread part only, except in mode 3)
        T = mats[int(P["rt_mat"]) + int(op["mat"]):]
        mode = int(op["mode"])
        loc = li if mode == 3 else np.broadcast_to(tl[:, None], li.shape)
        rt = np.zeros((gb.shape[0],) + li.shape, dtype=np.int64)
        for j in range(int(op["nbits"])):
            lp, gp = int(op["lpos"][j]), int(op["gpos"][j])
            if lp == 0xFF:
                bit = ((gb >> np.uint64(gp)) & np.uint64(1)).astype(np.int64)[:, None, None]
            else:
                bit = ((loc >> np.uint64(lp)) & np.uint64(1)).astype(np.int64)[None, :, :]
            rt = rt | (bit << j)
        if mode in (1, 2):
            r0 = 0 if mode == 1 else 1
            e = np.arange(16)
            c = ((e >> r0) & 1) | (((e >> (r0 + 2)) & 1) << 1)
            idx = c[None, None, :] + 4 * rt
        else:
            idx = rt
        return a * T[idx]
    raise AssertionError("unknown kernel op kind %d" % kind)


def _phase_parts(H, nthr):
    """Local and global index parts of each thread and register slot, and the
    global parts of their transposes (the phase's mirror tables)."""
    thr = np.arange(1 << nthr, dtype=np.uint64)
    tl = _bits(thr, H["thr_local"], nthr)
    tg = _bits(thr, H["thr_gpos"], nthr)
    tm = _bits(thr, H["thr_mpos"], nthr)
    e = np.arange(16, dtype=np.uint64)
    sl = _bits(e, H["reg_local"], 4)
    sg = _bits(e, H["reg_gpos"], 4)
    sm = _bits(e, H["reg_mpos"], 4)
    return tl, tg, sl, sg, tm, sm


def run(plan, amps: np.ndarray) -> np.ndarray:
    """Apply every pass of `plan` to the vectorised state `amps` (complex128),
    as the kernel does: a tile is loaded with the first phase's positions
    (from the transpose where the previous pass stored only the other half),
    each phase reads and writes the tile's local array by its local
    positions (the LDS exchange), and the last phase's positions store it,
    with the group bits of the layout the pass stores (out_gpos), into the
    other buffer when the pass changes the layout.  A buffer entered by such
    a pass starts as NaN: an amplitude read before it is written shows."""
    n = plan["n"]
    n2 = 2 * n
    mats = plan["mats"]
    bufs = [amps.copy(), None]
    cur = 0
    prev_pass = None
    for P in plan["passes"]:
        L = int(P["L"])
        nthr = L - 4
        T = int(P["n_tiles"])
        ngb = int(P["ngb"])
        herm = bool(P["herm"])
        flags = int(P["herm"])
        if herm:
            # the group pairs i <= j, i in the row group bits and j in the
            # column group bits; tiles with i < j also write their mirror
            m = ngb // 2
            N = 1 << m
            pairs = [(i, j) for t in range(T) for (i, j, ok) in [herm_tile(flags, m, t)] if ok]
            assert sorted(pairs) == [(i, j) for i in range(N) for j in range(i, N)]
            ii = np.array([i for i, _ in pairs], dtype=np.uint64)
            jj = np.array([j for _, j in pairs], dtype=np.uint64)
            gq = list(P["group_gpos"][:m]) + list(P["group_gpos"][m:2 * m])
            oq = list(P["out_gpos"][:m]) + list(P["out_gpos"][m:2 * m])
            ij = ii | (jj << np.uint64(m))
            ji = jj | (ii << np.uint64(m))
            gb = _bits(ij, gq, 2 * m)
            gbs = _bits(ij, oq, 2 * m)
            gbm = _bits(ji, gq, 2 * m)          # the transposed tile's base, loaded layout
            gbms = _bits(ji, oq, 2 * m)         # and stored layout
            mirror = ii != jj
            assert flags & HERM_PASS
        else:
            tiles = np.arange(T, dtype=np.uint64)
            gb = _bits(tiles, P["group_gpos"], ngb)
            gbs = _bits(tiles, P["out_gpos"], ngb)
            mirror = np.zeros(T, dtype=bool)
        T = gb.shape[0]
        src = bufs[cur]
        if int(P["swap_out"]):
            dst_i = 1 - cur
            bufs[dst_i] = np.full_like(src, np.nan)
        else:
            dst_i = cur
        pb, pe = int(P["pb"]), int(P["pe"])
        # load
        tl0, tg0, sl0, sg0, tm0, sm0 = _phase_parts(plan["phases"][pb], nthr)
        gidx = gb[:, None, None] | tg0[None, :, None] | sg0[None, None, :]
        valid = (gidx >> np.uint64(n2)) == 0
        gi = np.where(valid, gidx, 0).astype(np.int64)
        a = np.where(valid, src[gi], 0)
        if herm and flags & HERM_HALF_IN:
            # the previous pass stored only its group pairs i <= j (in the
            # layout it stored): the others come from the transpose, conjugated
            Pp = prev_pass
            mp = int(Pp["ngb"]) // 2
            ip = np.zeros(gidx.shape, dtype=np.int64)
            jp = np.zeros(gidx.shape, dtype=np.int64)
            for k in range(mp):
                ip |= ((gidx >> np.uint64(Pp["out_gpos"][k])) & np.uint64(1)).astype(np.int64) << k
                jp |= ((gidx >> np.uint64(Pp["out_gpos"][mp + k])) & np.uint64(1)).astype(np.int64) << k
            midx = gbm[:, None, None] | tm0[None, :, None] | sm0[None, None, :]
            a = np.where(ip > jp, np.conj(src[midx.astype(np.int64)]), a)
        X = np.zeros((T, 1 << L), dtype=np.complex128)
        li = (tl0[:, None] | sl0[None, :]).astype(np.int64)
        X[:, li] = a
        # phases
        for ph in range(pb, pe):
            H = plan["phases"][ph]
            tl, _, sl, _, _, _ = _phase_parts(H, nthr)
            li = (tl[:, None] | sl[None, :]).astype(np.int64)
            a = X[:, li]
            for oi in range(int(H["ob"]), int(H["oe"])):
                a = _apply_op(plan["ops"][oi], a, mats, P, li.astype(np.uint64), gb, tl)
            X[:, li] = a
        # store
        tlL, tgL, slL, sgL, tmL, smL = _phase_parts(plan["phases"][pe - 1], nthr)
        li = (tlL[:, None] | slL[None, :]).astype(np.int64)
        a = X[:, li]
        sidx = gbs[:, None, None] | tgL[None, :, None] | sgL[None, None, :]
        ok = (sidx >> np.uint64(n2)) == 0
        dst = bufs[dst_i]
        dst[sidx[ok].astype(np.int64)] = a[ok]
        if herm and flags & HERM_MIRROR:
            sel = np.broadcast_to(mirror[:, None, None], sidx.shape) & ok
            midx = gbms[:, None, None] | tmL[None, :, None] | smL[None, None, :]
            dst[midx[sel].astype(np.int64)] = np.conj(a[sel])
        cur = dst_i
        prev_pass = P
    assert cur == 0, "the plan ends in the second buffer"
    return bufs[0]
