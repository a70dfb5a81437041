"""Learned surrogate of the noisy QAOA simulator and the parameter search it guides.

The network maps (QAOA angles gamma_1..p, beta_1..p, leak, dephasing and decay rates) to
(energy per site, success probability) of the simulated circuit (Sec. IV).  It is trained on
the simulator's own batched outputs (mpdo_run_batch) by the library's GPU kernels
(include/mpdo_mlp.h): FP32 weights, BF16 matrix-core products, FP32 accumulation.

Every angle enters the circuit through exp(-i gamma Z(x)Z) or exp(-i beta X), which are -1 on
the qubit levels at angle pi and leave the other levels alone, so the observables are periodic
with period pi in each angle: the angles live on a torus and enter the network through the
harmonics sin(2a), cos(2a), sin(4a), cos(4a).

Search: minimise the energy per site over the 2p angles (taken modulo pi) at fixed noise rates.
Both searches use the same local optimiser on the simulator (BFGS, finite-difference gradients;
every function value is one simulator call) and restart it from random angles when it stops
short of the target.  They differ in where the local runs start:
  plain     from random angles;
  guided    the surrogate is minimised from many starts by input gradients (no simulator
            calls); its best distinct proposals are judged by the simulator in one batch, and
            the local runs start from them, best judged first.  The simulator is the judge of
            every reported value and the fallback when the surrogate is off.

Nothing here runs without a GPU: the simulator and the network are the HIP library.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import math
import time
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import circuits, mpdo

EXPORTS = ("mpdo_mlp_param_count", "mpdo_mlp_create", "mpdo_mlp_destroy", "mpdo_mlp_set_params",
           "mpdo_mlp_get_params", "mpdo_mlp_forward", "mpdo_mlp_loss_grad", "mpdo_mlp_train_step",
           "mpdo_mlp_input_grad", "mpdo_mlp_last_error")

_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int)


def _lib():
    lib = mpdo.load_library()
    if getattr(lib, "_mlp_bound", False):
        return lib
    h = C.c_void_p
    lib.mpdo_mlp_param_count.argtypes = [C.c_int, _ip]
    lib.mpdo_mlp_param_count.restype = C.c_size_t
    lib.mpdo_mlp_create.argtypes = [C.c_int, _ip, C.c_int, C.c_void_p, C.POINTER(h)]
    lib.mpdo_mlp_destroy.argtypes = [h]
    lib.mpdo_mlp_set_params.argtypes = [h, _fp]
    lib.mpdo_mlp_get_params.argtypes = [h, _fp]
    lib.mpdo_mlp_forward.argtypes = [h, C.c_int, _fp, _fp]
    lib.mpdo_mlp_loss_grad.argtypes = [h, C.c_int, _fp, _fp, _fp, _fp]
    lib.mpdo_mlp_train_step.argtypes = [h, C.c_int, _fp, _fp, C.c_float, _fp]
    lib.mpdo_mlp_input_grad.argtypes = [h, C.c_int, _fp, _fp, _fp, _fp]
    lib.mpdo_mlp_last_error.argtypes = [h]
    lib.mpdo_mlp_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("mpdo_mlp_param_count", "mpdo_mlp_last_error"):
            getattr(lib, name).restype = C.c_int
    lib._mlp_bound = True
    return lib


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _p(a: np.ndarray):
    return a.ctypes.data_as(_fp)


class MLP:
    """The library's GPU network (FP32 parameters, BF16 products)."""

    def __init__(self, widths, max_batch: int, seed: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the surrogate network runs on the GPU; no CPU fallback exists")
        self.lib = _lib()
        self.widths = [int(w) for w in widths]
        self.max_batch = int(max_batch)
        w = (C.c_int * len(self.widths))(*self.widths)
        self.h = C.c_void_p()
        st = self.lib.mpdo_mlp_create(len(self.widths) - 1, w, self.max_batch, None, C.byref(self.h))
        if st != 0:
            raise mpdo.MpdoError(st, "mpdo_mlp_create failed (%d)" % st)
        self.n_params = int(self.lib.mpdo_mlp_param_count(len(self.widths) - 1, w))
        self.set_params(self.initial_params(seed))

    def initial_params(self, seed: int) -> np.ndarray:
        """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
        rng = np.random.default_rng(seed)
        parts = []
        for i, o in zip(self.widths[:-1], self.widths[1:]):
            lim = 1.0 / math.sqrt(i)
            parts.append(rng.uniform(-lim, lim, size=o * i))
            parts.append(np.zeros(o))
        return np.concatenate(parts)

    def _check(self, st):
        if st != 0:
            msg = self.lib.mpdo_mlp_last_error(self.h)
            raise mpdo.MpdoError(st, msg.decode() if msg else "")

    def close(self):
        if self.h:
            self.lib.mpdo_mlp_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        p = _f32(p)
        assert p.size == self.n_params
        self._check(self.lib.mpdo_mlp_set_params(self.h, _p(p)))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        self._check(self.lib.mpdo_mlp_get_params(self.h, _p(out)))
        return out

    def forward(self, x) -> np.ndarray:
        x = _f32(x)
        out = np.zeros((x.shape[0], self.widths[-1]), dtype=np.float32)
        for s in range(0, x.shape[0], self.max_batch):
            xs = _f32(x[s:s + self.max_batch])
            ys = np.zeros((xs.shape[0], self.widths[-1]), dtype=np.float32)
            self._check(self.lib.mpdo_mlp_forward(self.h, xs.shape[0], _p(xs), _p(ys)))
            out[s:s + xs.shape[0]] = ys
        return out

    def loss_grad(self, x, t):
        x, t = _f32(x), _f32(t)
        loss = np.zeros(1, dtype=np.float32)
        g = np.zeros(self.n_params, dtype=np.float32)
        self._check(self.lib.mpdo_mlp_loss_grad(self.h, x.shape[0], _p(x), _p(t), _p(loss), _p(g)))
        return float(loss[0]), g

    def train_step(self, x, t, lr: float) -> float:
        x, t = _f32(x), _f32(t)
        loss = np.zeros(1, dtype=np.float32)
        self._check(self.lib.mpdo_mlp_train_step(self.h, x.shape[0], _p(x), _p(t), C.c_float(lr), _p(loss)))
        return float(loss[0])

    def input_grad(self, x, w_out):
        x, w = _f32(x), _f32(w_out)
        y = np.zeros((x.shape[0], self.widths[-1]), dtype=np.float32)
        dx = np.zeros_like(x)
        self._check(self.lib.mpdo_mlp_input_grad(self.h, x.shape[0], _p(x), _p(w), _p(y), _p(dx)))
        return y, dx


# ------------------------------------------------------------------------ the simulated task
@dataclass
class Task:
    n: int = 20
    d: int = 4
    p: int = 3
    chi: int = 64
    rate_lo: float = 1e-4
    rate_hi: float = 1e-2

    @property
    def n_in(self) -> int:
        return 8 * self.p + 3


HARMONICS = (2.0, 4.0)   # frequencies of the angle features (period pi and pi/2)


def features(task: Task, angles: np.ndarray, rates: np.ndarray) -> np.ndarray:
    """Network inputs: sin(k a), cos(k a) for k in HARMONICS and every angle, then the log-rates
    mapped from [rate_lo, rate_hi] to [-1, 1]."""
    angles = np.atleast_2d(angles)
    rates = np.atleast_2d(rates)
    if rates.shape[0] == 1 and angles.shape[0] > 1:
        rates = np.repeat(rates, angles.shape[0], axis=0)
    parts = []
    for k in HARMONICS:
        parts += [np.sin(k * angles), np.cos(k * angles)]
    lo, hi = math.log(task.rate_lo), math.log(task.rate_hi)
    parts.append(2.0 * (np.log(rates) - lo) / (hi - lo) - 1.0)
    return np.concatenate(parts, axis=1)


def angle_grad(angles: np.ndarray, dfeat: np.ndarray) -> np.ndarray:
    """Chain rule of features(): gradient over the angles from the gradient over the inputs."""
    angles = np.atleast_2d(angles)
    m = angles.shape[1]
    g = np.zeros_like(angles)
    pos = 0
    for k in HARMONICS:
        g += dfeat[:, pos:pos + m] * k * np.cos(k * angles)
        g -= dfeat[:, pos + m:pos + 2 * m] * k * np.sin(k * angles)
        pos += 2 * m
    return g


def wrap_distance(a, b) -> np.ndarray:
    """Largest per-angle distance on the torus of period pi."""
    h = 0.5 * math.pi
    return np.max(np.abs(np.mod(np.asarray(a) - np.asarray(b) + h, math.pi) - h), axis=-1)


def spec_of(task: Task, angles, rates, seed: int = 0):
    from workloads.qaoa import CircuitSpec
    p = task.p
    return CircuitSpec(n=task.n, d=task.d, p=p, gamma=tuple(float(x) for x in angles[:p]),
                       beta=tuple(float(x) for x in angles[p:]), p_leak=float(rates[0]),
                       p_deph=float(rates[1]), p_decay=float(rates[2]), chi=task.chi, seed=seed, name="surrogate")


class Simulator:
    """Simulator calls with a counter (each circuit is one call): one point runs on a context
    kept for the task, several points go through the batch runtime."""

    def __init__(self, task: Task, n_workers: int = 16):
        self.task = task
        self.n_workers = n_workers
        self.calls = 0
        self._m = None

    def _one(self, a, r) -> np.ndarray:
        t = self.task
        if self._m is None:
            self._m = mpdo.MPDO(t.n, t.d, t.chi)
        circuits.run_circuit(spec_of(t, a, r), m=self._m)
        o = circuits.observables(self._m)
        return np.array([[o["energy_per_site"], o["p_success"]]])

    def __call__(self, angles: np.ndarray, rates: np.ndarray) -> np.ndarray:
        angles = np.atleast_2d(angles)
        rates = np.atleast_2d(rates)
        if rates.shape[0] == 1 and angles.shape[0] > 1:
            rates = np.repeat(rates, angles.shape[0], axis=0)
        if angles.shape[0] == 1:
            self.calls += 1
            return self._one(angles[0], rates[0])
        descs = [circuits.describe(spec_of(self.task, a, r)) for a, r in zip(angles, rates)]
        res = mpdo.run_batch(descs, n_workers=min(self.n_workers, len(descs)))
        out = np.zeros((len(descs), 2))
        for i, r in enumerate(res):
            if r["status"] != 0:
                raise mpdo.MpdoError(r["status"], "simulator call failed")
            s = circuits.summarize(r["values"], self.task.n, self.task.d)
            out[i] = (s["energy_per_site"], s["p_success"])
        self.calls += len(descs)
        return out


def make_dataset(sim: Simulator, count: int, seed: int, chunk: int = 2048, log=None):
    """Uniform angles on [0, pi) and log-uniform rates on [rate_lo, rate_hi], simulated in batches."""
    rng = np.random.default_rng(seed)
    t = sim.task
    angles = rng.uniform(0.0, math.pi, size=(count, 2 * t.p))
    rates = np.exp(rng.uniform(math.log(t.rate_lo), math.log(t.rate_hi), size=(count, 3)))
    y = np.zeros((count, 2))
    for s in range(0, count, chunk):
        y[s:s + chunk] = sim(angles[s:s + chunk], rates[s:s + chunk])
        if log is not None:
            log("[surrogate] simulated %d of %d circuits" % (min(count, s + chunk), count))
    return features(t, angles, rates), y, angles, rates


def train(net: MLP, X, Y, epochs: int = 200, batch: int = 256, lr: float = 2e-3, seed: int = 0):
    """Adam on standardised targets; returns (mean, std) of the targets and the loss history."""
    rng = np.random.default_rng(seed)
    mu, sd = Y.mean(axis=0), Y.std(axis=0) + 1e-12
    Yn = (Y - mu) / sd
    hist = []
    n = X.shape[0]
    for ep in range(epochs):
        perm = rng.permutation(n)
        tot = 0.0
        for s in range(0, n, batch):
            idx = perm[s:s + batch]
            step_lr = lr * (0.1 ** (ep / max(1, epochs - 1)))   # exponential decay to lr/10
            tot += net.train_step(X[idx], Yn[idx], step_lr) * len(idx)
        hist.append(tot / n)
    return mu, sd, hist


class Surrogate:
    def __init__(self, net: MLP, task: Task, mu, sd):
        self.net, self.task, self.mu, self.sd = net, task, mu, sd

    def predict(self, angles, rates) -> np.ndarray:
        return self.net.forward(features(self.task, angles, rates)) * self.sd + self.mu

    def minimise_energy(self, rates, starts: int = 512, steps: int = 300, lr: float = 0.05, seed: int = 0):
        """Projected gradient descent on the predicted energy over the angles, from many starts."""
        rng = np.random.default_rng(seed)
        t = self.task
        a = rng.uniform(0.0, math.pi, size=(starts, 2 * t.p))
        r = np.repeat(np.atleast_2d(rates), starts, axis=0)
        w = np.array([self.sd[0], 0.0], dtype=np.float32)     # d energy / d output
        m = np.zeros_like(a)
        v = np.zeros_like(a)
        for k in range(1, steps + 1):
            _, dx = self.net.input_grad(features(t, a, r), w)
            g = angle_grad(a, dx.astype(np.float64))
            m = 0.9 * m + 0.1 * g
            v = 0.999 * v + 0.001 * g * g
            a = a - lr * (m / (1 - 0.9 ** k)) / (np.sqrt(v / (1 - 0.999 ** k)) + 1e-8)
        a = np.mod(a, math.pi)
        e = self.predict(a, r)[:, 0]
        order = np.argsort(e)
        return a[order], e[order]

    def proposals(self, rates, count: int, sep: float = 0.25, seed: int = 0) -> np.ndarray:
        """The best `count` surrogate minima that differ by more than `sep` rad in some angle."""
        cand, _ = self.minimise_energy(rates, seed=seed)
        picks = []
        for a in cand:
            if all(wrap_distance(a, b) > sep for b in picks):
                picks.append(a)
            if len(picks) == count:
                break
        return np.array(picks)


# ------------------------------------------------------------------------ searches
class _Stop(Exception):
    pass


class Tracker:
    """Counts simulator calls of one search and keeps the best value after each call."""

    def __init__(self, sim: Simulator, rates, budget: int, target: float):
        self.sim, self.rates, self.budget, self.target = sim, np.asarray(rates, dtype=float), budget, target
        self.history = []
        self.best_x, self.best = None, float("inf")

    def done(self) -> bool:
        return len(self.history) >= self.budget or self.best <= self.target

    def record(self, xs, values):
        for x, v in zip(xs, values):
            if v < self.best:
                self.best_x, self.best = np.mod(x, math.pi), float(v)
            self.history.append(self.best)

    def batch(self, xs) -> np.ndarray:
        xs = np.mod(np.atleast_2d(xs), math.pi)[: max(0, self.budget - len(self.history))]
        vals = self.sim(xs, self.rates)[:, 0] if len(xs) > 1 else \
            np.array([self.sim(xs[0], self.rates)[0, 0]]) if len(xs) else np.zeros(0)
        self.record(xs, vals)
        return vals

    def __call__(self, x) -> float:
        if self.done():
            raise _Stop
        return float(self.batch(x)[0])


def local_search(tr: Tracker, x0, gtol: float = 1e-7, fd_step: float = 1e-6):
    """BFGS on the simulator from x0, stopping at the tracker's budget or target.  The gradient
    is a forward difference: the point and its 2p shifted copies are one batch of simulator
    calls (each circuit counts as one call)."""
    from scipy.optimize import minimize
    eye = np.eye(len(x0)) * fd_step

    def value_and_grad(x):
        if tr.done():
            raise _Stop
        pts = np.vstack([x, x + eye])
        vals = tr.batch(pts)
        if len(vals) < len(pts):
            raise _Stop
        return float(vals[0]), (vals[1:] - vals[0]) / fd_step

    try:
        minimize(value_and_grad, np.asarray(x0, dtype=float), jac=True, method="BFGS",
                 options={"gtol": gtol, "maxiter": 10 ** 6})
    except _Stop:
        pass


def plain_search(sim: Simulator, rates, budget: int, target: float = -np.inf, seed: int = 0,
                 log=None) -> dict:
    """Local runs from random angles until the target or the budget is reached."""
    rng = np.random.default_rng(seed)
    tr = Tracker(sim, rates, budget, target)
    while not tr.done():
        local_search(tr, rng.uniform(0.0, math.pi, size=2 * sim.task.p))
        if log is not None:
            log("[surrogate]     plain: %d calls, best %.7f" % (len(tr.history), tr.best))
    return {"x": tr.best_x, "energy": tr.best, "calls": len(tr.history), "history": tr.history}


def guided_search(sim: Simulator, sur: Surrogate, rates, budget: int, target: float = -np.inf,
                  proposals: int = 4, seed: int = 0, log=None) -> dict:
    """Surrogate proposals judged in one batch, local runs from them (best judged first), then
    the plain search's random restarts if the target is still not reached."""
    tr = Tracker(sim, rates, budget, target)
    picks = sur.proposals(rates, proposals, seed=seed)
    judged = tr.batch(picks)
    pred = sur.predict(picks, rates)[:, 0]
    res = {"proposal_max_abs_err": float(np.max(np.abs(judged - pred[:len(judged)]))) if len(judged) else None}
    rng = np.random.default_rng(seed)
    starts = [picks[i] for i in np.argsort(judged)]
    while not tr.done():
        local_search(tr, starts.pop(0) if starts else rng.uniform(0.0, math.pi, size=2 * sim.task.p))
        if log is not None:
            log("[surrogate]     guided: %d calls, best %.7f" % (len(tr.history), tr.best))
    res.update({"x": tr.best_x, "energy": tr.best, "calls": len(tr.history), "history": tr.history})
    return res


def calls_to_reach(hist, target: float) -> Optional[int]:
    for i, v in enumerate(hist):
        if v <= target:
            return i + 1
    return None


def experiment(task: Task, n_data: int, epochs: int, rate_sets, budget: int, runs: int = 3,
               proposals: int = 4, seed: int = 0, widths=None, n_workers: int = 16, log=print,
               chunk: int = 2048) -> dict:
    """Dataset -> training -> for each noise setting: reference optimum, then the simulator calls
    the plain and the guided search need to come within 1e-3 of it."""
    def say(msg):
        log("[surrogate] " + msg)

    t0 = time.time()
    sim = Simulator(task, n_workers)
    X, Y, _, _ = make_dataset(sim, n_data, seed, chunk=chunk, log=log)
    t_data = time.time() - t0
    say("dataset of %d circuits in %.1f s" % (n_data, t_data))
    widths = widths or [task.n_in, 256, 256, 256, 2]
    net = MLP(widths, max_batch=1024, seed=seed)
    t0 = time.time()
    mu, sd, hist = train(net, X, Y, epochs=epochs, seed=seed)
    t_train = time.time() - t0
    say("trained %d epochs in %.1f s, loss %.3e" % (epochs, t_train, hist[-1]))
    sur = Surrogate(net, task, mu, sd)
    _, Yt, at, rt = make_dataset(Simulator(task, n_workers), 256, seed + 1)
    err = np.abs(sur.predict(at, rt) - Yt)
    say("held-out |error|: energy rms %.2e max %.2e, success max %.2e"
        % (math.sqrt(np.mean(err[:, 0] ** 2)), err[:, 0].max(), err[:, 1].max()))
    out = {"task": task.__dict__, "n_data": n_data, "epochs": epochs, "widths": widths,
           "data_seconds": t_data, "train_seconds": t_train, "final_train_loss": hist[-1],
           "heldout_rms_err_energy": float(math.sqrt(np.mean(err[:, 0] ** 2))),
           "heldout_max_abs_err": err.max(axis=0).tolist(), "budget": budget, "searches": []}
    for rates in rate_sets:
        rates = np.asarray(rates, dtype=float)
        # every run spends its whole budget; the optimum is the best value any run found, and
        # each run is scored by the calls it needed to come within 1e-3 of it
        runs_p, runs_g = [], []
        for s in range(runs):
            runs_p.append(plain_search(Simulator(task, n_workers), rates, budget, seed=200 + s, log=log))
            runs_g.append(guided_search(Simulator(task, n_workers), sur, rates, budget, proposals=proposals,
                                        seed=300 + s, log=log))
            say("rates %s run %d: plain best %.7f, guided best %.7f"
                % (rates.tolist(), s, runs_p[-1]["energy"], runs_g[-1]["energy"]))
        e_star = min(r["energy"] for r in runs_p + runs_g)
        target = e_star + 1e-3
        pc = [calls_to_reach(r["history"], target) for r in runs_p]
        gc = [calls_to_reach(r["history"], target) for r in runs_g]
        say("rates %s: optimum %.7f; calls to within 1e-3: plain %s, guided %s" % (rates.tolist(), e_star, pc, gc))
        out["searches"].append({"rates": rates.tolist(), "optimum_energy_per_site": e_star, "target": target,
                                "plain_calls": pc, "guided_calls": gc,
                                "plain_best": [r["energy"] for r in runs_p],
                                "guided_best": [r["energy"] for r in runs_g],
                                "proposal_max_abs_err": [r["proposal_max_abs_err"] for r in runs_g]})
    return out


def main():
    ap = argparse.ArgumentParser(description="train the surrogate and compare searches")
    ap.add_argument("--n", type=int, default=20)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--chi", type=int, default=64)
    ap.add_argument("--data", type=int, default=2048)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--budget", type=int, default=1500)
    ap.add_argument("--runs", type=int, default=3)
    ap.add_argument("--rates", type=float, nargs=3, action="append",
                    help="noise setting (leak, dephasing, decay); repeat for several")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--proposals", type=int, default=4)
    ap.add_argument("--chunk", type=int, default=2048, help="circuits per batch call while building the data")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    task = Task(n=a.n, p=a.p, chi=a.chi)
    rate_sets = a.rates or [[1e-3, 1e-3, 1e-3]]
    res = experiment(task, a.data, a.epochs, rate_sets, budget=a.budget, runs=a.runs, seed=a.seed,
                     proposals=a.proposals, chunk=a.chunk, log=lambda m: print(m, flush=True))
    line = json.dumps(res)
    print(line)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
