"""Learned warm start of steady-state thermal two-phase solves.

A solve runs the LB step from an initial state until the one-step
residual max over {rho, T} of ||phi^n - phi^(n-1)||_inf / ||phi^n||_inf
falls below a target.  The warm start replaces the initial density and
temperature by the network's prediction of the steady fields (the
distributions start at equilibrium with zero velocity, as a cold start
does).  When the prediction is poor (its own one-step residual above
`reject`), the solve falls back to the cold start, so the LB step always
judges the result.

Training data are solver trajectories: batches of cases run to the target
by `solve`, their initial fields as input and their steady fields as
target.  The network (nn.UNet) trains on the GPU with its own kernels.
"""
import time

import numpy as np

from .lbm import CORRECTED, Batch, LbmError
from .nn import UNet


def _scalars(cases, Tc):
    """Per-case (T0/T_c, tau_f, tau_g), T0 the mean initial temperature."""
    return np.array([[float(T.mean()) / Tc, p["tau_f"], p["tau_g"]] for p, _, T in cases])


def solve(cases, precision="fp64", inits=None, target=1e-8, cap=200000, chunk=1000,
          treatment=CORRECTED, graph=50, keep=True, physical=False, log=None, log_every=20000):
    """Run every case (a list of (params, rho, T)) from its initial fields
    (or from inits[i] = (rho, T) when given) to the residual target, in one
    batch with converged lattices frozen.  `physical` starts each lattice
    at rest in the forcing scheme's velocity (stored momentum -F/2,
    lbm_init_fields_physical) instead of at zero stored momentum.  Checks the residual every
    `chunk` steps.  FP64 storage by default: with FP32 storage the one-step
    residual stalls between 1e-7 and 1e-6 (rounding of the stored
    distributions).  Returns a dict with per-case steps (None when the cap or
    a non-finite value stopped it), the wall time, the number of given
    initial states the library refused (those lattices start cold, e.g. a
    prediction with a negative density), and (keep) the final fields as
    FP64 host arrays.  `log` (a callable) gets a progress line
    every `log_every` steps."""
    import torch
    t0 = time.perf_counter()
    refs = [(float(r.mean()), float(t.mean())) for _, r, t in cases]
    b = Batch([c[0] for c in cases], precision, refs=refs)
    fallback = 0
    for i, (m, (p, rho, T)) in enumerate(zip(b.members, cases)):
        if inits is not None and inits[i] is not None:
            try:
                m.init_fields(*inits[i], physical=physical)
                continue
            except LbmError:
                fallback += 1  # not a valid state (e.g. a negative density): the cold start
        m.init_fields(rho, T, physical=physical)
    if graph:
        b.use_graph(graph)
    n = len(cases)
    steps = [None] * n
    failed = [False] * n
    done = 0
    while done < cap:
        open_ = [steps[i] is None and not failed[i] for i in range(n)]
        if not any(open_):
            break
        b.set_active(open_)
        b.step(chunk - 1, treatment)
        done += chunk
        res, status = b.step_residuals(treatment)
        for i in range(n):
            if open_[i]:
                if status[i] != 0 or not np.isfinite(res[i]):
                    failed[i] = True
                elif res[i] < target:
                    steps[i] = done
        if log and done % log_every == 0:
            log("solve: %d steps, %d of %d open, %.1f s" % (
                done, sum(steps[i] is None and not failed[i] for i in range(n)), n, time.perf_counter() - t0))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"steps": steps, "failed": failed, "wall_s": wall, "cap": cap, "invalid_inits": fallback}
    if keep:
        fields = []
        for i in range(n):
            rho, ux, uy, T = b[i].moments(check=False)
            fields.append((rho, T))
        out["fields"] = fields
    b.close()
    return out


def solve_single(cases, precision="fp64", target=1e-8, cap=200000, chunk=1000, treatment=CORRECTED):
    """The plain way: one lattice at a time (single-lattice launches), cold
    start, residual checked every `chunk` steps.  Returns per-case steps and
    the wall time."""
    import torch
    from .lbm import Lattice
    t0 = time.perf_counter()
    steps = []
    for p, rho, T in cases:
        g = Lattice(p, precision)
        g.init_fields(rho, T)
        done, st = 0, None
        while done < cap:
            g.step(chunk - 1, treatment)
            done += chunk
            try:
                r = g.step_residual(treatment)
            except RuntimeError:
                break
            if r < target:
                st = done
                break
        steps.append(st)
        g.close()
    torch.cuda.synchronize()
    return {"steps": steps, "wall_s": time.perf_counter() - t0, "cap": cap}


def load_params(path):
    with np.load(path) as z:
        return {k: z[k].astype(np.float64) for k in z.files}


class WarmStart:
    """The network plus its training and inference on n x n cases."""

    def __init__(self, n, batch=8, Tc=None, seed=0, params=None):
        from . import inputs
        from .nn import init_params
        self.n, self.B = n, batch
        self.Tc = Tc if Tc is not None else inputs.cs_tc()
        self.net = UNet(batch, n, n, wrap_x=True, params=params if params is not None else init_params(seed))

    def _upload(self, arrays):
        import torch
        return torch.from_numpy(np.ascontiguousarray(np.stack(arrays))).to("cuda")

    def dataset(self, cases, steady):
        """Device tensors of a training set: initial fields, scalars and the
        normalised steady fields (FP32 [N, n, n, 2])."""
        import torch
        N = len(cases)
        rho0 = self._upload([c[1] for c in cases])
        T0 = self._upload([c[2] for c in cases])
        sc = torch.from_numpy(_scalars(cases, self.Tc)).to("cuda")
        tgt = torch.empty((N, self.n, self.n, 2), dtype=torch.float32, device="cuda")
        rho1 = self._upload([s[0] for s in steady])
        T1 = self._upload([s[1] for s in steady])
        # normalise one batch-sized slice at a time with the network's packer
        for k in range(0, N, self.B):
            idx = list(range(k, min(N, k + self.B)))
            if len(idx) < self.B:
                idx += [idx[-1]] * (self.B - len(idx))
            sel = torch.tensor(idx, device="cuda")
            out = torch.empty((self.B, self.n, self.n, 2), dtype=torch.float32, device="cuda")
            self.net.pack_target(rho1.index_select(0, sel).contiguous(), T1.index_select(0, sel).contiguous(),
                                 self.Tc, out)
            m = min(self.B, N - k)
            tgt[k:k + m] = out[:m]
        return {"rho": rho0, "T": T0, "s": sc, "target": tgt, "N": N}

    def _batch(self, data, idx):
        import torch
        sel = torch.tensor(idx, device="cuda")
        self.net.pack_input(data["rho"].index_select(0, sel).contiguous(),
                            data["T"].index_select(0, sel).contiguous(),
                            data["s"].index_select(0, sel).contiguous(), self.Tc)
        return data["target"].index_select(0, sel).contiguous()

    def train(self, data, epochs=20, lr=2e-3, seed=0, log=None):
        """Adam over shuffled mini-batches; returns the mean loss per epoch."""
        import torch
        rng = np.random.default_rng(seed)
        N = data["N"]
        if N < self.B:
            raise ValueError("need at least %d training cases, got %d" % (self.B, N))
        hist = []
        for ep in range(epochs):
            order = rng.permutation(N)
            nb = N // self.B
            losses = torch.zeros(nb, dtype=torch.float32, device="cuda")
            for k in range(nb):
                tgt = self._batch(data, order[k * self.B:(k + 1) * self.B].tolist())
                self.net.forward()
                self.net.backward(tgt)
                losses[k:k + 1].copy_(self.net.loss_dev)
                self.net.adam(lr * (0.5 * (1 + np.cos(np.pi * ep / epochs))))
            hist.append(float(losses.mean().item()))
            if log:
                log("epoch %d loss %.3e" % (ep, hist[-1]))
        return hist

    def predict(self, cases, conserve_mass=True):
        """Predicted steady (rho, T) FP64 host arrays for each case.  The LB
        step conserves mass, so the predicted density is rescaled to the
        initial field's total mass (a warm start must not change which
        steady state the solve reaches)."""
        import torch
        out = []
        N = len(cases)
        for k in range(0, N, self.B):
            chunk = cases[k:k + self.B]
            pad = chunk + [chunk[-1]] * (self.B - len(chunk))
            rho = self._upload([c[1] for c in pad])
            T = self._upload([c[2] for c in pad])
            sc = torch.from_numpy(_scalars(pad, self.Tc)).to("cuda")
            self.net.pack_input(rho, T, sc, self.Tc)
            self.net.forward()
            r1 = torch.empty_like(rho)
            t1 = torch.empty_like(T)
            self.net.unpack(r1, t1, self.Tc)
            r1, t1 = r1.cpu().numpy(), t1.cpu().numpy()
            for j in range(len(chunk)):
                rj = r1[j]
                if conserve_mass:
                    rj = rj * (float(chunk[j][1].sum()) / float(rj.sum()))
                out.append((rj, t1[j]))
        return out


def residuals(cases, fields, precision="fp64", treatment=CORRECTED, physical=False):
    """One-step residual of each (rho, T) used as an initial state (inf
    where the step fails); `physical` as in solve."""
    refs = [(float(r.mean()), float(t.mean())) for _, r, t in cases]
    b = Batch([c[0] for c in cases], precision, refs=refs)
    out = []
    for m, fr in zip(b.members, fields):
        try:
            m.init_fields(*fr, physical=physical)
            r = m.step_residual(treatment)
        except RuntimeError:
            r = np.inf
        out.append(r if np.isfinite(r) else np.inf)
    b.close()
    return out


def screen(cases, preds, precision="fp64", reject=1e-3, factor=1.0, treatment=CORRECTED,
           physical=False):
    """Keep a prediction as the initial state when its one-step residual is
    at most `reject` or not above `factor` (default 1) times the cold
    start's own initial residual (a cold start of these two-phase states
    already has a one-step residual of about 3e-2, so an absolute 1e-3
    alone would reject every start); otherwise, or when non-finite, None
    (the cold start).  Returns (kept, predicted residuals, cold residuals).
    `physical` judges both from the start at rest in the forcing scheme (as
    in solve)."""
    rp = residuals(cases, preds, precision, treatment, physical)
    rc = residuals(cases, [(c[1], c[2]) for c in cases], precision, treatment, physical)
    keep = [pr if (r <= reject or r <= factor * c) else None for pr, r, c in zip(preds, rp, rc)]
    return keep, rp, rc
