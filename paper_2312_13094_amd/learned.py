"""Learned coarse-grid correction: orchestration of libfd calls.

A space-order-4 propagation on a 2x coarser grid with a 2x larger time step
is corrected after every coarse step by the 3-layer BF16 network of
``fdnn.h`` toward the space-order-8 fine-grid solution:

    u~(n+1) = coarse leapfrog step of (u(n), u(n-1))             [fd_step_lagged]
    s       = rms(u~(n+1))                                        [nn_rms]
    u(n+1)  = u~(n+1) + k s N(u~/s, u(n)/s, v^ u~/s)  outside B   [nn_* kernels]
            = u~(n+1)                                 inside B

with v^ = (v - 3000)/1500, a fixed output gain k = 1e-3 (the one-step
residual is about that fraction of the field, so the network's output is
O(1)) and B a 5^3 box of coarse nodes around the source.  The network has no
biases and its velocity channel multiplies the field, so N(0) = 0: it cannot
create a wavefield where there is none.  Inside B the residual is the
mismatch of the two grids' discrete point sources, which depends on the
source wavelet the network does not see; B is excluded from the correction
and from the loss.

Training data come from the plain solver: fine solves are restricted to the
coarse nodes (even fine indices) at coarse times, the coarse step is taken
from the restricted states, and the network learns the one-step residual
(teacher forcing), with a cosine-decayed Adam step.  The plain fine solve
is both the reference for the trace error and the fallback when the
corrected run turns non-finite or its amplitude grows late in the run (a
learned correction can feed an unstable mode; the physical field only decays
once the source has stopped).

This module only allocates caller-side buffers and sequences library calls;
every arithmetic step runs in libfd's kernels (restriction to the coarse
nodes is a strided device copy).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import fd as FD
from . import nn as NN
from .synth import Learned


def _restrict(g_fine, f, out):
    """Fine padded field -> dense coarse volume (values at even fine indices)."""
    out.copy_(g_fine.domain(f)[::2, ::2, ::2])


@dataclass
class Sample:
    ut: torch.Tensor       # coarse step result u~(n+1), dense
    u0: torch.Tensor       # u(n), dense
    target: torch.Tensor   # restricted fine u(n+1) - u~(n+1), dense
    model: int             # index into the model list


@dataclass
class RunResult:
    traces: np.ndarray     # [nt_coarse][nrec]
    seconds: float
    fallback: bool = False
    info: dict = field(default_factory=dict)


class LearnedCorrector:
    GAIN = 1e-3          # output gain k
    SKIP_HALF = 2        # half-width of the source box B, coarse nodes

    def __init__(self, cfg: Learned, params=None, device: int = 0):
        self.cfg = c = cfg
        self.dev = torch.device("cuda", device)
        nf, nc = c.n_fine, c.n_coarse
        self.fine = FD.Grid((nf,) * 3, (c.h_fine,) * 3, c.so_fine, c.dt_fine, c.vmax,
                            nbl=c.nbl_fine, device=device)
        self.coarse = FD.Grid((nc,) * 3, (c.h_coarse,) * 3, c.so_coarse, c.dt_coarse, c.vmax,
                              nbl=c.nbl_coarse, device=device)
        self.net = NN.Net((nc,) * 3, params, device, bias=False)
        sc = [i // 2 for i in c.src_idx]
        w = self.SKIP_HALF
        self.skip = NN.box([max(0, i - w) for i in sc], [min(nc, i + w + 1) for i in sc])
        self._zero = torch.zeros(nc ** 3, dtype=torch.float32, device=self.dev)
        src, rec = c.src_fine(), c.rec_fine()          # physical coordinates, shared
        self.Sf, self.Rf = self.fine.sparse(src), self.fine.sparse(rec)
        self.Sc, self.Rc = self.coarse.sparse(src), self.coarse.sparse(rec)
        self.qf = torch.from_numpy(c.q_fine()).to(self.dev)
        self.qc = torch.from_numpy(c.q_coarse()).to(self.dev)
        self.vhat = torch.zeros((nc,) * 3, dtype=torch.float32, device=self.dev)
        self.fa, self.fb = self.fine.field(), self.fine.field()
        self.ca, self.cb = self.coarse.field(), self.coarse.field()
        self.cview = NN.grid_view(self.coarse)
        self.dview = NN.dense_view((nc,) * 3)

    # -- models -------------------------------------------------------------
    def set_model(self, vel_fine: np.ndarray):
        vf = torch.from_numpy(np.ascontiguousarray(vel_fine, dtype=np.float32)).to(self.dev)
        self.fine.set_model(vf)
        vc = vf[::2, ::2, ::2].contiguous()
        self.coarse.set_model(vc)
        if not getattr(self, "_tuned", False):
            # the library's autotuner picks both grids' step tiles once (the
            # plain fine solve, the reference, is tuned too)
            self.tiles = {"fine": self.fine.autotune(), "coarse": self.coarse.autotune()}
            self._tuned = True
        # network input channel: (v - 3000) / 1500
        self.vhat.copy_(vc).sub_(3000.0).div_(1500.0)

    # -- plain solvers ---------------------------------------------------------
    def fine_solve(self, snapshot_steps=()):
        """Plain fine run.  Returns (traces at coarse times [nt_c][nr],
        seconds, {fine step k: restricted u(k)} for k in snapshot_steps)."""
        c = self.cfg
        self.fa.zero_()
        self.fb.zero_()
        d = torch.zeros((c.nt_fine, self.Rf.n), dtype=torch.float32, device=self.dev)
        snaps = {}
        stops = sorted(set(int(k) for k in snapshot_steps if 0 < k <= c.nt_fine))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k0 = 0
        for k in stops + [c.nt_fine]:
            if k > k0:
                self.fine.forward([self.fa, self.fb], self.Sf, self.qf[k0:], self.Rf, d[k0:], k - k0)
                k0 = k
            if k in stops:
                out = torch.empty((c.n_coarse,) * 3, dtype=torch.float32, device=self.dev)
                _restrict(self.fine, self.fa, out)
                snaps[k] = out
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        # coarse step n samples u at fine step 2n + 2, i.e. fine trace index 2n + 1
        tr = d[1::2].double().cpu().numpy()
        return tr, secs, snaps

    def coarse_solve(self):
        """Plain coarse run (no correction)."""
        c = self.cfg
        self.ca.zero_()
        self.cb.zero_()
        d = torch.zeros((c.nt_coarse, self.Rc.n), dtype=torch.float32, device=self.dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.coarse.forward([self.ca, self.cb], self.Sc, self.qc, self.Rc, d, c.nt_coarse)
        torch.cuda.synchronize()
        return d.double().cpu().numpy(), time.perf_counter() - t0

    def plain_coarse_solve(self, so, vel_fine):
        """Equal-error baseline: a plain run on the coarse grid and time step
        with space order `so` (its own handle, tile picked by the autotuner).
        Returns (traces [nt_coarse][nr], seconds)."""
        c = self.cfg
        if not hasattr(self, "_plain"):
            self._plain = {}
        if so not in self._plain:
            g = FD.Grid((c.n_coarse,) * 3, (c.h_coarse,) * 3, so, c.dt_coarse, c.vmax,
                        nbl=c.nbl_coarse, device=self.dev.index or 0)
            S, R = g.sparse(c.src_fine()), g.sparse(c.rec_fine())
            self._plain[so] = (g, S, R, g.field(), g.field(), False)
        g, S, R, a, b, tuned = self._plain[so]
        vf = torch.from_numpy(np.ascontiguousarray(vel_fine, dtype=np.float32)).to(self.dev)
        g.set_model(vf[::2, ::2, ::2].contiguous())
        if not tuned:
            g.autotune()
            self._plain[so] = (g, S, R, a, b, True)
        a.zero_()
        b.zero_()
        d = torch.zeros((c.nt_coarse, R.n), dtype=torch.float32, device=self.dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.forward([a, b], S, self.qc, R, d, c.nt_coarse)
        torch.cuda.synchronize()
        return d.double().cpu().numpy(), time.perf_counter() - t0

    # -- learned run ---------------------------------------------------------
    def coarse_step(self, n, u, um_up):
        """Plain coarse update n in place: um_up (u(n-1)) becomes u~(n+1)."""
        self.coarse.step(u, um_up, self.Sc, self.qc[n])

    def correct(self, new, old, scale=None):
        """new <- new + k s N(new/s, old/s, vhat new/s) outside B, s = rms(new)
        (computed into scale, nn_rms_scratch_floats() floats; the network's own
        buffer if None)."""
        net = self.net
        sc = net.scale if scale is None else scale
        net.rms(new, self.cview, sc)
        # layer 1 forms the network input (new/s, old/s, vhat new/s) itself
        net.forward(keep=False, out=new, base=new, vbase=self.cview, vout=self.cview,
                    scale=sc, ydense=False, gain=self.GAIN, skip=self.skip,
                    fields=(new, self.cview, old, self.cview, self.vhat, self.dview, True))

    def _scales(self):
        """One RMS buffer per coarse step: row n's first value is then the RMS
        of prediction n, the history the guard reads, with no copy."""
        return torch.zeros((self.cfg.nt_coarse, int(NN.lib().nn_rms_scratch_floats())),
                           dtype=torch.float32, device=self.dev)

    def _corrected_run(self, d, hist):
        """The whole corrected coarse run from rest: traces into d, the RMS of
        coarse prediction n into hist[n, 0] (hist from _scales), non-finite
        values flagged in net.flag.  Enqueues only (no host synchronisation),
        so it can be captured into a graph."""
        c = self.cfg
        self.ca.zero_()
        self.cb.zero_()
        self.net.flag.zero_()
        u, um = self.ca, self.cb
        for n in range(c.nt_coarse):
            # the update's launch that injects the source also records the
            # corrected level it reads (the previous update's)
            self.coarse.step(u, um, self.Sc, self.qc[n], self.Rc if n else None,
                             d[n - 1] if n else None, lagged=True)
            self.correct(um, u, hist[n])
            u, um = um, u
        self.coarse.sample(u, self.Rc, d[c.nt_coarse - 1])

    def learned_solve(self, guard=True, graph=False):
        """Corrected coarse run; falls back to the plain fine solve if the
        corrected wavefield turns non-finite or its RMS in the last quarter of
        the run exceeds twice its peak over the first three quarters.

        graph=True records the run into a HIP graph on first use (the
        coarse model and network weights are read from the same buffers on
        every replay, so later models and weights need no new capture) and
        replays it; the time reported is the replay's."""
        c = self.cfg
        if graph:
            if getattr(self, "_graph", None) is None:
                self._gd = torch.zeros((c.nt_coarse, self.Rc.n), dtype=torch.float32,
                                       device=self.dev)
                self._gh = self._scales()
                torch.cuda.synchronize()
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    self._corrected_run(self._gd, self._gh)
                torch.cuda.synchronize()
                self._graph = g
            d, hist = self._gd, self._gh
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            self._graph.replay()
        else:
            d = torch.zeros((c.nt_coarse, self.Rc.n), dtype=torch.float32, device=self.dev)
            hist = self._scales()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            self._corrected_run(d, hist)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        tr = d.double().cpu().numpy()
        h = hist[:, 0].cpu().numpy()
        q = (3 * len(h)) // 4
        growth = len(h) > 4 and h[q:].max() > 2.0 * h[:q].max()
        bad = bool(self.net.flag.item()) or not np.isfinite(tr).all() or not np.isfinite(h).all()
        if guard and (bad or growth):
            ftr, fsecs, _ = self.fine_solve()
            return RunResult(ftr, secs + fsecs, fallback=True,
                             info={"learned_seconds": secs, "non_finite": bad, "growth": growth})
        return RunResult(tr, secs)

    # -- training data and training -----------------------------------------
    def make_samples(self, seeds, coarse_steps, model_store):
        """Teacher-forcing samples for every seed and coarse step n in
        coarse_steps (1 <= n < nt_coarse)."""
        c = self.cfg
        samples = []
        for seed in seeds:
            self.set_model(c.velocity(seed))
            model_store.append(self.vhat.clone())
            mi = len(model_store) - 1
            ks = []
            for n in coarse_steps:
                ks += [2 * n - 2, 2 * n, 2 * n + 2]
            _, _, snaps = self.fine_solve(snapshot_steps=[k for k in ks if k > 0])
            zero = torch.zeros((c.n_coarse,) * 3, dtype=torch.float32, device=self.dev)
            for n in coarse_steps:
                um = snaps.get(2 * n - 2, zero)
                u0 = snaps[2 * n]
                up = snaps[2 * n + 2]
                self.ca.zero_()
                self.cb.zero_()
                self.coarse.domain(self.ca).copy_(u0)
                self.coarse.domain(self.cb).copy_(um)
                self.coarse_step(n, self.ca, self.cb)
                ut = self.coarse.domain(self.cb).contiguous()
                samples.append(Sample(ut, u0.clone(), (up - ut).contiguous(), mi))
        return samples

    def _load(self, s, models):
        net = self.net
        net.rms(s.ut, self.dview)
        net.pack_input(s.ut, self.dview, s.u0, self.dview, models[s.model], self.dview,
                       scale=net.scale, c_times_a=True)

    def train(self, samples, models, iters, lr=2e-3, seed=0, batch=4, log_every=0):
        """Adam on the one-step MSE of the scaled residual r / (k s) outside B,
        gradients summed over `batch` random samples per step, step size
        lr (1 + cos(pi i / iters)) / 2; returns the loss history."""
        rng = np.random.default_rng(seed)
        net = self.net
        hist = []
        for it in range(iters):
            net.loss.zero_()
            for b in range(batch):
                s = samples[int(rng.integers(len(samples)))]
                self._load(s, models)
                net.forward(keep=True)
                net.backward(s.target, scale=net.scale, gain=self.GAIN, skip=self.skip,
                             accumulate=b > 0)
            net.adam(lr=lr * 0.5 * (1.0 + np.cos(np.pi * it / iters)))
            if log_every and (it % log_every == 0 or it == iters - 1):
                hist.append((it, net.loss.item()))
        return hist

    def sample_loss(self, samples, models):
        """Mean one-step loss of the current network over `samples`, and that
        of the uncorrected coarse step (a zero prediction)."""
        net = self.net
        nz, ny, nx = net.shape
        L = NN.lib()
        tot, base = 0.0, 0.0
        for s in samples:
            self._load(s, models)
            net.forward(keep=True)
            net.loss.zero_()
            net.backward(s.target, scale=net.scale, gain=self.GAIN, skip=self.skip)
            tot += net.loss.item()
            net.loss.zero_()
            NN._chk(L.nn_mse(nz, ny, nx, NN._p(self._zero), NN._p(s.target), NN._p(net.scale),
                             self.GAIN, NN._bp(self.skip), NN._p(net.g8), NN._p(net.loss),
                             NN._s()))
            base += net.loss.item()
        return tot / len(samples), base / len(samples)


def trace_error(a, ref):
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))
