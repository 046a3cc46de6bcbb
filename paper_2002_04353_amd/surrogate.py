"""Surrogate of the ALE lattice-Boltzmann solver's load histories.

A fully connected network (5 -> 256 -> 256 -> 256 -> 256, tanh hidden
layers) maps a pitch+plunge case's parameters (Ma, k, A, h/c, plunge phase),
scaled to [-1, 1] over the ensemble's ranges, to its lift and moment
coefficient histories: c_L and c_m at 128 equally spaced times over the
first ``steps`` solver steps after the impulsive start (outputs 0..127 and
128..255), standardized per output over the training set.

Training data come from the solver itself (``solver_histories``: batches of
cases, each on its own mesh or on one shared mesh, forces integrated on the
GPU every steps/128 steps); the network is trained on the GPU by the BF16
matrix-core kernels of ``include/alelb_mlp.h`` (``mlp.MLP``).  ``baselines``
gives what the method offers without the network: the training mean, the
nearest training case and a linear fit in the scaled parameters.  The solver stays the reference: a
query outside the training box, or asking for a tolerance tighter than the
validated error, is answered by running the solver (``Surrogate.predict_or_solve``).
"""

from __future__ import annotations

import time

import numpy as np

from . import alelb, cases, mlp

PARAMS = ("Ma", "k", "A_deg", "h_c", "phase_h")
SAMPLES = 128
WIDTHS = (5, 256, 256, 256, 2 * SAMPLES)


def scale_params(motion) -> np.ndarray:
    """(Ma, k, A_deg, h_c, phase_h) rows -> [-1, 1] over the ensemble's ranges."""
    m = np.atleast_2d(np.asarray(motion, dtype=np.float64))
    lo = np.array([cases.ENSEMBLE_RANGES[k][0] for k in PARAMS])
    hi = np.array([cases.ENSEMBLE_RANGES[k][1] for k in PARAMS])
    return (2.0 * (m - lo) / (hi - lo) - 1.0).astype(np.float32)


def solver_histories(mesh, motion, steps, samples=SAMPLES, precision="fp32", batch=64, Re=1850.0):
    """Run the solver for every parameter row (cases batched ``batch`` at a
    time) and return (Y [n, 2 samples] = (c_L, c_m) histories, seconds of wall
    time spent in the solver, including set-up).  ``mesh`` is one mesh for
    every row, or a list with one mesh per row.  A case the solver cannot
    carry through (the unshifted D2Q9 model diverges in a corner of fast,
    high-Mach plunges) has non-finite entries in its row."""
    motion = np.atleast_2d(np.asarray(motion, dtype=np.float64))
    if steps % samples:
        raise ValueError("steps must be a multiple of samples")
    meshes = list(mesh) if isinstance(mesh, (list, tuple)) else [mesh] * motion.shape[0]
    if len(meshes) != motion.shape[0]:
        raise ValueError("one mesh per parameter row")
    every = steps // samples
    Y = np.empty((motion.shape[0], 2 * samples))
    t0 = time.perf_counter()
    arrays = {}
    for c0 in range(0, motion.shape[0], batch):
        rows = motion[c0:c0 + batch]
        ms = meshes[c0:c0 + batch]
        prm, init = [], []
        for r, m in zip(rows, ms):
            p, u = cases.pitch_plunge_params(*r, Re=Re)
            prm.append(p)
            N = m.n_nodes
            init.append(dict(rho=np.ones(N), ux=np.full(N, u), uy=np.zeros(N), T=np.full(N, 0.3)))
        arr = [arrays.setdefault(id(m), m.arrays()) for m in ms]
        s = alelb.Solver(arr, prm, precision=precision, flags=alelb.F_GRAPH, stream=0)
        s.init_fields(**cases.concat_init(init))
        for j in range(samples):
            s.step(every)
            f = s.forces_batch()
            Y[c0:c0 + len(rows), j] = [x["cl"] for x in f]
            Y[c0:c0 + len(rows), samples + j] = [x["cm"] for x in f]
        s.close()
    return Y, time.perf_counter() - t0


class Surrogate:
    """The network, its output standardization, and the solver fallback."""

    def __init__(self, mesh, steps, widths=WIDTHS, max_batch=4096, seed=0):
        self.mesh = mesh
        self.steps = int(steps)
        self.widths = tuple(widths)
        self.net = mlp.MLP(widths, max_batch)
        self.net.set_params(glorot(widths, seed))
        self.mean = np.zeros(widths[-1], dtype=np.float32)
        self.std = np.ones(widths[-1], dtype=np.float32)
        self.val_rms = None  # validated RMS error of (c_L, c_m) against the solver

    def fit(self, X, Y, iters=3000, lr=2e-3, batch=256, seed=0, lr_final=1e-4):
        """Adam on the standardized targets with a cosine-decayed learning rate:
        full-batch steps on device-resident data when the set fits one batch,
        else random minibatches.  Returns the loss history."""
        import torch
        self.mean = Y.mean(axis=0).astype(np.float32)
        self.std = (Y.std(axis=0) + 1e-6).astype(np.float32)
        Ys = ((Y - self.mean) / self.std).astype(np.float32)
        X = np.ascontiguousarray(X, dtype=np.float32)
        rng = np.random.default_rng(seed)
        losses = []
        full = X.shape[0] <= batch
        if full:
            xd = torch.from_numpy(X).cuda()
            yd = torch.from_numpy(np.ascontiguousarray(Ys)).cuda()
            torch.cuda.synchronize()
        lrs = [lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * it / iters)) for it in range(iters)]
        if full:
            return self.net.train_steps(xd.data_ptr(), yd.data_ptr(), lrs, on_device=True, batch=X.shape[0])
        for a in lrs:
            idx = rng.choice(X.shape[0], size=batch, replace=False)
            losses.append(self.net.train_step(X[idx], Ys[idx], lr=a))
        return np.array(losses)

    def predict(self, X) -> np.ndarray:
        return self.net.forward(np.asarray(X, dtype=np.float32)) * self.std + self.mean

    def validate(self, motion, Y):
        """RMS error of c_L and c_m against solver histories of held-out cases."""
        P = self.predict(scale_params(motion))
        n = SAMPLES
        self.val_rms = (float(np.sqrt(np.mean((P[:, :n] - Y[:, :n]) ** 2))),
                        float(np.sqrt(np.mean((P[:, n:] - Y[:, n:]) ** 2))))
        return self.val_rms

    def predict_or_solve(self, motion, tolerance=None):
        """Histories for the parameter rows: from the network when every row is
        inside the training box and the validated error meets ``tolerance``
        (RMS of c_L), else from the solver.  Returns (Y, 'surrogate'|'solver')."""
        x = scale_params(motion)
        inside = bool(np.all(np.abs(x) <= 1.0))
        good = tolerance is None or (self.val_rms is not None and self.val_rms[0] <= tolerance)
        if inside and good:
            return self.predict(x), "surrogate"
        Y, _ = solver_histories(self.mesh, motion, self.steps)
        return Y, "solver"

    def close(self):
        self.net.close()


def baselines(Xtr, Ytr, Xte):
    """What the method offers for new parameters without the network, each a
    prediction [n_test, outputs]: the training mean; the history of the
    nearest training case in the scaled parameters (the phase taken on the
    circle); a least-squares fit affine in the scaled parameters (the phase
    through its sine and cosine)."""
    Xtr = np.asarray(Xtr, dtype=np.float64)
    Xte = np.asarray(Xte, dtype=np.float64)

    def feats(X):
        ph = np.pi * (X[:, 4] + 1.0)  # back to radians over [0, 2 pi]
        return np.column_stack([np.ones(len(X)), X[:, :4], np.sin(ph), np.cos(ph)])

    mean = np.broadcast_to(Ytr.mean(axis=0), (len(Xte), Ytr.shape[1]))
    d = Xtr[None, :, :4] - Xte[:, None, :4]
    dph = np.abs(Xtr[None, :, 4] - Xte[:, None, 4])
    dph = np.minimum(dph, 2.0 - dph)  # the phase's scaled range [-1, 1] is one period
    nn = Ytr[np.argmin((d ** 2).sum(axis=2) + dph ** 2, axis=1)]
    coef, *_ = np.linalg.lstsq(feats(Xtr), Ytr, rcond=None)
    lin = feats(Xte) @ coef
    return {"mean": mean, "nearest": nn, "linear": lin}


def rms_cl_cm(P, Y):
    n = Y.shape[1] // 2
    return (float(np.sqrt(np.mean((P[:, :n] - Y[:, :n]) ** 2))), float(np.sqrt(np.mean((P[:, n:] - Y[:, n:]) ** 2))))


def glorot(widths, seed=0) -> np.ndarray:
    """Glorot-uniform weights, zero biases, packed like the network's parameters."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(widths) - 1):
        n_in, n_out = widths[l], widths[l + 1]
        lim = np.sqrt(6.0 / (n_in + n_out))
        parts.append(rng.uniform(-lim, lim, size=n_out * n_in))
        parts.append(np.zeros(n_out))
    return np.concatenate(parts).astype(np.float32)
