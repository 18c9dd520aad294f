"""Learned surrogate of a parametric noisy circuit, with the batched emulator
as its data source, its fallback and the judge of its error.

* :class:`TemplateEmulator` -- exact <Z_i> of many parameter settings of one
  circuit structure: a parametric template in the batched kernel, run in
  chunks that reuse one device arena.
* :class:`SurrogateModel` -- the MLP ensemble (library kernels) with a
  training loop (shuffled mini-batches, Adam, cosine learning-rate decay) and
  prediction with fallback: samples whose ensemble spread exceeds the
  threshold are recomputed by the emulator.

Everything that touches the data runs in the library's kernels; this module
only draws the shuffling permutation and moves tensors between calls.
"""
from __future__ import annotations

import math
import time
from typing import Callable, Optional

import numpy as np

from . import vqd


class TemplateEmulator:
    """Batched exact emulation of one circuit structure for many settings.

    ``structure``: list of ``(kind, qubits)`` (extra tuple entries ignored);
    ``run(params)`` takes ``[count, n_ops, 4]`` per-op parameters and returns
    the ``[count, n]`` float64 device tensor of <Z_i>."""

    def __init__(self, n: int, structure, chunk: int = 8192, device: str = "cuda", opts=None):
        self.n = n
        self.structure = [(s[0], tuple(s[1])) for s in structure]
        self.chunk = chunk
        self.device = device
        self.opts = opts              # vqd.PlanOpts for the template, or the library default
        self._arena = None
        self._out = None
        self.last_gpu_s = 0.0         # time of the batched launches alone in the last run()
        self.last_idle_s = 0.0        # device time between consecutive chunks' launches in the last run()

    def run(self, params: np.ndarray):
        """The host work of a chunk (coefficients of every instance, and a
        contiguous copy of its parameters when ``params`` is a strided view)
        runs while the previous chunk's launch is still on the GPU."""
        import torch
        P = np.asarray(params, dtype=np.float64)
        count = P.shape[0]
        res = torch.empty((count, self.n), dtype=torch.float64, device=self.device)
        prev = None
        events = []
        for lo in range(0, count, self.chunk):
            hi = min(count, lo + self.chunk)
            b = vqd.Batch()
            tid = b.add_template(self.n, self.structure)
            idx = b.add_instances(tid, P[lo:hi])
            if self.opts is not None:
                b.set_opts(self.n, self.opts)
            b.arena, b.out = self._arena, self._out
            b.compile(device=self.device)
            self._arena, self._out = b.arena, b.out
            # freeing the previous chunk's plan synchronises the device: do it
            # only now, after this chunk's host work, so that work overlapped
            # the previous launch
            if prev is not None:
                prev.close()
            ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            ev[0].record()
            b.run()
            ev[1].record()
            events.append(ev)
            # one template's instances get consecutive output slots, so the
            # results are one device slice; no host copy here, which would
            # wait for the launch and keep the next chunk's host work from
            # overlapping it
            first, last = b.offsets(idx[0])[1], b.offsets(idx[-1])[1]
            if last - first == (hi - lo - 1) * self.n:
                res[lo:hi] = self._out[first:first + (hi - lo) * self.n].view(hi - lo, self.n)
            else:
                outs = np.fromiter((b.offsets(i)[1] for i in idx), dtype=np.int64, count=hi - lo)
                sel = torch.from_numpy(outs).pin_memory().to(self.device, non_blocking=True)
                res[lo:hi] = self._out[sel[:, None] + torch.arange(self.n, device=self.device)]
            prev = b
        if prev is not None:
            prev.close()
        torch.cuda.synchronize()
        self.last_gpu_s = sum(a.elapsed_time(z) for a, z in events) / 1e3
        self.last_idle_s = sum(events[k - 1][1].elapsed_time(events[k][0]) for k in range(1, len(events))) / 1e3
        return res

    def reserve(self, params: np.ndarray):
        """Allocate the device buffers (state arena, outputs) of one full
        chunk of these settings now, so that a later run() only reuses them."""
        P = np.ascontiguousarray(params[:self.chunk], dtype=np.float64)
        b = vqd.Batch()
        tid = b.add_template(self.n, self.structure)
        b.add_instances(tid, P)
        if self.opts is not None:
            b.set_opts(self.n, self.opts)
        b.arena, b.out = self._arena, self._out
        b.compile(device=self.device)
        self._arena, self._out = b.arena, b.out
        b.close()

    def autotune(self, params: np.ndarray, cache_path: str, sample: int = 1024):
        """Pick the template's tile shape with the batched autotuner (timed
        on ``sample`` instances, result cached in ``cache_path``)."""
        P = np.ascontiguousarray(params[:sample], dtype=np.float64)
        b = vqd.Batch()
        tid = b.add_template(self.n, self.structure)
        b.add_instances(tid, P)
        b.compile(device=self.device)
        b.autotune(cache_path, max_per_n=sample)
        o = b.plan_opts(self.n)
        self.opts = vqd.plan_opts(tile_bits=o["tile_bits"], min_contig_bits=o["min_contig_bits"],
                                  max_ops_per_pass=o["max_ops_per_pass"], fuse_blocks=bool(o["fuse_blocks"]),
                                  pad_coalesce=bool(o["pad_coalesce"]))
        b.close()
        return o

    def release(self):
        self._arena = None
        self._out = None


class SurrogateModel:
    """MLP ensemble over scaled inputs ``x`` ([*, 24] float32) predicting
    ``y`` ([*, 10]); see vqd.Surrogate for the network and number formats."""

    def __init__(self, init_params: np.ndarray, max_batch: int = 4096):
        self.net = vqd.Surrogate(members=init_params.shape[0], max_batch=max_batch, params=init_params)
        self.history = []
        # spread threshold under which a prediction is accepted; set only by
        # calibrate() against the emulator.  None: every sample falls back.
        self.threshold: Optional[float] = None

    def fit(self, x, y, epochs: int, batch: int = 1024, lr: float = 2e-3, lr_min: float = 1e-5,
            seed: int = 0, log: Optional[Callable[[str], None]] = None):
        """Shuffled mini-batch Adam over device tensors x, y (float32).  The
        learning rate follows a cosine from lr to lr_min over all steps."""
        import torch
        n = x.shape[0]
        steps_per_epoch = n // batch
        total = epochs * steps_per_epoch
        rng = np.random.default_rng(seed)
        loss = torch.zeros(self.net.members, dtype=torch.float32, device=x.device)
        t0 = time.perf_counter()
        k = 0
        for ep in range(epochs):
            perm = torch.as_tensor(rng.permutation(n).astype(np.int32), device=x.device)
            acc = torch.zeros_like(loss)
            for s in range(steps_per_epoch):
                a = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * k / max(1, total)))
                self.net.train_step(x, y, a, idx=perm[s * batch:(s + 1) * batch], loss=loss)
                acc += loss
                k += 1
            mean_loss = (acc / max(1, steps_per_epoch)).cpu().numpy()
            self.history.append(mean_loss)
            if log:
                log("epoch %d  loss %s  (%.1f s)" % (ep, np.array2string(mean_loss, precision=6),
                                                     time.perf_counter() - t0))
        return self

    def predict(self, x):
        return self.net.predict(x)

    def calibrate(self, x, exact, tol: float = 1e-2, quantile: float = 1.0) -> float:
        """Set and return the spread threshold: a prediction is accepted when
        its spread is strictly below it.  Chosen on a held-out set (inputs x,
        exact values from the emulator, the judge) as the largest threshold
        under which the accepted samples stay within max_i |dZ_i| < tol; with
        quantile < 1, that fraction of them must.  Samples whose spread ties
        a rejected one are rejected with it.  0 (accept nothing) when even
        the lowest-spread sample misses."""
        mean, spread = self.net.predict(x)
        err = (mean.double() - exact).abs().max(dim=1).values.cpu().numpy()
        sp = spread.double().cpu().numpy()
        order = np.argsort(sp, kind="stable")
        bad = err[order] >= tol
        # accepted set {spread < thr} grows along `order`; keep the longest
        # prefix whose miss fraction stays within 1 - quantile
        misses = np.cumsum(bad)
        ok = misses <= (1.0 - quantile) * np.arange(1, len(order) + 1)
        if not ok[0]:
            thr = 0.0
        elif ok.all():
            # every held-out sample is good: accept up to the largest spread seen
            thr = float(np.nextafter(sp[order[-1]], np.inf))
        else:
            # the first sample outside the prefix sets the bound (strict <)
            thr = float(sp[order[int(np.nonzero(~ok)[0][0])]])
        self.threshold = thr
        return thr

    def predict_with_fallback(self, x, fallback: Callable[[np.ndarray], "object"],
                              threshold: Optional[float] = None):
        """Ensemble mean where the spread is strictly below the threshold;
        elsewhere ``fallback(indices)`` (exact values, device [k, 10]).  The
        threshold defaults to the one set by calibrate(); without one every
        sample falls back, so no answer is accepted that the emulator has not
        vouched for.  Returns (values [B, 10] float32 device tensor,
        fell_back bool device tensor).  A threshold that accepts nothing
        (none, or at most 0: spreads are never negative) leaves the network
        unconsulted: every sample goes to the fallback at once."""
        import torch
        thr = self.threshold if threshold is None else threshold
        if thr is None or thr <= 0.0:
            B = x.shape[0]
            vals = fallback(np.arange(B)).to(torch.float32)
            return vals, torch.ones(B, dtype=torch.bool, device=vals.device)
        mean, spread = self.net.predict(x)
        fell = spread >= thr
        idx = torch.nonzero(fell).flatten()
        if idx.numel():
            mean[idx] = fallback(idx.cpu().numpy()).to(mean.dtype)
        return mean, fell


def measure_gain(model: SurrogateModel, emulator: TemplateEmulator, params: np.ndarray, x,
                 threshold: Optional[float] = None, tol: float = 1e-2) -> dict:
    """Throughput of the surrogate with fallback against the emulator alone
    on the same samples, the emulator also judging the surrogate's error.

    The emulator's rate counts every sample (all exact).  The surrogate's
    time covers inference plus the emulation of the samples that fell back;
    its rate at the accuracy target counts only answers with max_i |dZ_i| <
    ``tol`` (fallback answers are exact)."""
    import torch

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    B = params.shape[0]
    thr = model.threshold if threshold is None else threshold
    exact, t_emu = timed(lambda: emulator.run(params))
    (vals, fell), t_sur = timed(lambda: model.predict_with_fallback(
        x, lambda idx: emulator.run(params if len(idx) == B else params[idx]), thr))
    err = (vals.double() - exact).abs().max(dim=1).values
    fell_np = fell.cpu().numpy()
    err_np = err.cpu().numpy()
    acc = ~fell_np
    good = int((err_np < tol).sum())
    return {
        "samples": B,
        "threshold": thr,
        "emulator_evals_per_s": round(B / t_emu, 1),
        "surrogate_evals_per_s": round(B / t_sur, 1),
        "surrogate_good_evals_per_s": round(good / t_sur, 1),
        "gain_at_tol": round((good / t_sur) / (B / t_emu), 3),
        "fallback_fraction": round(float(fell_np.mean()), 4),
        "accepted_within_tol_fraction": round(float((err_np[acc] < tol).mean()) if acc.any() else 1.0, 4),
        "max_abs_dz_accepted": float(err_np[acc].max()) if acc.any() else 0.0,
        "median_abs_dz_accepted": float(np.median(err_np[acc])) if acc.any() else 0.0,
        "emulator_s": round(t_emu, 4),
        "surrogate_s": round(t_sur, 4),
    }
