"""Learned surrogate of the noisy QAOA simulator and the parameter search it guides.

The network maps (QAOA angles gamma_1..p, beta_1..p, leak, dephasing and decay rates) to
(energy per site, success probability) of the simulated circuit (Sec. IV).  It is trained on
the simulator's own batched outputs (mpdo_run_batch) by the library's GPU kernels
(include/mpdo_mlp.h): FP32 weights, BF16 matrix-core products, FP32 accumulation.

Search: minimise the energy per site over the 2p angles at fixed noise rates.
  plain     Nelder-Mead on the simulator; every function value is one simulator call.
  guided    the surrogate is minimised from many starts, by input gradients (free); its best
            proposals are judged by the simulator (one call each); Nelder-Mead on the
            simulator then refines the best judged point from a small simplex.  The simulator
            is the judge of every reported value and the fallback when the surrogate is off.

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
        return 2 * self.p + 3


def features(task: Task, angles: np.ndarray, rates: np.ndarray) -> np.ndarray:
    """Inputs in [-1, 1]: angles / (pi/2) - 1 and log-rates mapped from [rate_lo, rate_hi]."""
    angles = np.atleast_2d(angles)
    rates = np.atleast_2d(rates)
    a = angles / (0.5 * math.pi) - 1.0
    lo, hi = math.log(task.rate_lo), math.log(task.rate_hi)
    r = 2.0 * (np.log(rates) - lo) / (hi - lo) - 1.0
    return np.concatenate([a, r], axis=1)


def spec_of(task: Task, angles, rates, seed: int = 0):
    from workloads.qaoa import CircuitSpec
    p = task.p
    return CircuitSpec(n=task.n, d=task.d, p=p, gamma=tuple(float(x) for x in angles[:p]),
                       beta=tuple(float(x) for x in angles[p:]), p_leak=float(rates[0]),
                       p_deph=float(rates[1]), p_decay=float(rates[2]), chi=task.chi, seed=seed, name="surrogate")


class Simulator:
    """Batched simulator calls with a counter (each circuit is one call)."""

    def __init__(self, task: Task, n_workers: int = 16):
        self.task = task
        self.n_workers = n_workers
        self.calls = 0

    def __call__(self, angles: np.ndarray, rates: np.ndarray) -> np.ndarray:
        angles = np.atleast_2d(angles)
        rates = np.atleast_2d(rates)
        if rates.shape[0] == 1 and angles.shape[0] > 1:
            rates = np.repeat(rates, angles.shape[0], axis=0)
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


def make_dataset(sim: Simulator, count: int, seed: int):
    rng = np.random.default_rng(seed)
    t = sim.task
    angles = rng.uniform(0.0, math.pi, size=(count, 2 * t.p))
    rates = np.exp(rng.uniform(math.log(t.rate_lo), math.log(t.rate_hi), size=(count, 3)))
    y = sim(angles, rates)
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
            g = dx[:, :2 * t.p] / (0.5 * math.pi)             # chain rule of the feature map
            m = 0.9 * m + 0.1 * g
            v = 0.999 * v + 0.001 * g * g
            a = a - lr * (m / (1 - 0.9 ** k)) / (np.sqrt(v / (1 - 0.999 ** k)) + 1e-8)
            a = np.clip(a, 0.0, math.pi)
        e = self.predict(a, r)[:, 0]
        order = np.argsort(e)
        return a[order], e[order]


# ------------------------------------------------------------------------ searches
def _nelder_mead(f, x0, scale, budget: int, target: float, xatol: float = 1e-4):
    """Nelder-Mead on f (one simulator call per value); stops at the budget or once the best
    value is <= target.  Returns (best_x, best_f, history of best values by call)."""
    from scipy.optimize import minimize
    hist = []
    best = [None, float("inf")]

    class Done(Exception):
        pass

    def fw(x):
        if len(hist) >= budget:
            raise Done
        x = np.clip(x, 0.0, math.pi)
        v = float(f(x))
        if v < best[1]:
            best[0], best[1] = x.copy(), v
        hist.append(best[1])
        if best[1] <= target:
            raise Done
        return v

    dim = len(x0)
    simplex = np.vstack([x0] + [x0 + scale * np.eye(dim)[i] for i in range(dim)])
    try:
        minimize(fw, x0, method="Nelder-Mead",
                 options={"initial_simplex": simplex, "xatol": xatol, "fatol": 1e-7, "maxfev": budget})
    except Done:
        pass
    return best[0], best[1], hist


def plain_search(sim: Simulator, rates, budget: int, target: float = -np.inf, seed: int = 0):
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(0.0, math.pi, size=2 * sim.task.p)
    start = sim.calls
    x, e, hist = _nelder_mead(lambda a: sim(a, rates)[0, 0], x0, 0.4, budget, target)
    return {"x": x, "energy": e, "calls": sim.calls - start, "history": hist}


def guided_search(sim: Simulator, sur: Surrogate, rates, budget: int, target: float = -np.inf,
                  proposals: int = 4, seed: int = 0):
    start = sim.calls
    cand, pred = sur.minimise_energy(rates, seed=seed)
    # distinct proposals (angles differing by more than 0.05 rad somewhere)
    picks = []
    for a in cand:
        if all(np.max(np.abs(a - b)) > 0.05 for b in picks):
            picks.append(a)
        if len(picks) == proposals:
            break
    judged = sim(np.array(picks), rates)[:, 0]          # the simulator judges the proposals
    hist = list(np.minimum.accumulate(judged))
    i = int(np.argmin(judged))
    x0, e0 = picks[i], float(judged[i])
    res = {"x": x0, "energy": e0, "proposal_error": float(abs(judged[i] - sur.predict(x0, rates)[0, 0]))}
    if e0 > target and budget > len(picks):
        x, e, h = _nelder_mead(lambda a: sim(a, rates)[0, 0], x0, 0.05, budget - len(picks), target)
        if e < e0:
            res["x"], res["energy"] = x, e
        hist += [min(hist[-1], v) for v in h]
    res["calls"] = sim.calls - start
    res["history"] = hist
    return res


def calls_to_reach(hist, target: float) -> Optional[int]:
    for i, v in enumerate(hist):
        if v <= target:
            return i + 1
    return None


def experiment(task: Task, n_data: int, epochs: int, rates, budget: int, seed: int = 0,
               widths=None, n_workers: int = 16) -> dict:
    """Dataset -> training -> reference optimum -> calls of the plain and guided searches."""
    t0 = time.time()
    sim = Simulator(task, n_workers)
    X, Y, _, _ = make_dataset(sim, n_data, seed)
    t_data = time.time() - t0
    widths = widths or [task.n_in, 256, 256, 256, 2]
    net = MLP(widths, max_batch=1024, seed=seed)
    t0 = time.time()
    mu, sd, hist = train(net, X, Y, epochs=epochs, seed=seed)
    t_train = time.time() - t0
    sur = Surrogate(net, task, mu, sd)
    # held-out error
    Xt, Yt, at, rt = make_dataset(Simulator(task, n_workers), 256, seed + 1)
    pred = sur.predict(at, rt)
    err = np.abs(pred - Yt).max(axis=0)
    rates = np.asarray(rates, dtype=float)
    # reference optimum: the best of long plain searches and of the guided search's best point
    ref = []
    for s in range(3):
        ref.append(plain_search(Simulator(task, n_workers), rates, budget=4 * budget, seed=100 + s)["energy"])
    g_ref = guided_search(Simulator(task, n_workers), sur, rates, budget=4 * budget, seed=seed)
    e_star = min(min(ref), g_ref["energy"])
    target = e_star + 1e-3
    plain_calls, guided_calls = [], []
    for s in range(3):
        pr = plain_search(Simulator(task, n_workers), rates, budget=budget, target=target, seed=200 + s)
        gr = guided_search(Simulator(task, n_workers), sur, rates, budget=budget, target=target, seed=300 + s)
        plain_calls.append(calls_to_reach(pr["history"], target))
        guided_calls.append(calls_to_reach(gr["history"], target))
    return {"task": task.__dict__, "rates": rates.tolist(), "n_data": n_data, "data_seconds": t_data,
            "train_seconds": t_train, "final_train_loss": hist[-1], "heldout_max_abs_err": err.tolist(),
            "optimum_energy_per_site": e_star, "target": target, "budget": budget,
            "plain_calls": plain_calls, "guided_calls": guided_calls,
            "simulator_calls_for_data": n_data}


def main():
    ap = argparse.ArgumentParser(description="train the surrogate and compare searches")
    ap.add_argument("--n", type=int, default=20)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--chi", type=int, default=64)
    ap.add_argument("--data", type=int, default=2048)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--budget", type=int, default=400)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    task = Task(n=a.n, p=a.p, chi=a.chi)
    res = experiment(task, a.data, a.epochs, rates=[1e-3, 1e-3, 1e-3], budget=a.budget, seed=a.seed)
    line = json.dumps(res)
    print(line)
    if a.out:
        with open(a.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
