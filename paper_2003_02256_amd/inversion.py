"""Random-walk Metropolis inversion over the batched curve and misfit calls.

The method needs many dispersion curves: an inversion compares the curves of
many candidate models with the experimental one (Section 2.1; Algorithm 2
gives the misfit of one model), and quantifying uncertainty needs more of
them still.  This client runs a population of chains.  At every step each
chain proposes a perturbed model.  All proposals go through one batched
launch on the device that computes their dispersion curves and reduces
Algorithm 2's misfit of each (`masw_dispersion_batch_misfit`), and only the
misfits come back to the host.  Each chain then accepts its proposal with the Metropolis rule for
the target density exp(-misfit / temperature).

The chain logic (`perturb`, `metropolis_accept`, `run_chains`) is plain host
code on arrays with one row per chain; `DeviceEvaluator` is the only part
that touches the GPU, and any callable that maps a Population (or a list of
models) to their misfits can stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Sequence

import numpy as np

from . import MASW_NO_REFINE, MASW_PREC_FP64, MASW_PREC_SPLIT, MASW_SEARCH_INERTIA, masw_dispersion_batch_misfit


@dataclass
class LayeredModel:
    """N finite layers over a half-space (h: [N]; alpha, beta, rho: [N+1])."""

    h: np.ndarray
    alpha: np.ndarray
    beta: np.ndarray
    rho: np.ndarray

    @property
    def n_layers(self) -> int:
        return int(self.h.shape[0])

    def copy(self) -> "LayeredModel":
        return LayeredModel(self.h.copy(), self.alpha.copy(), self.beta.copy(), self.rho.copy())


def perturb(rng: np.random.Generator, m, step: float) -> LayeredModel:
    """Proposal: every beta_j and h_j times (1 + step N(0, 1)), each layer
    keeping its alpha/beta ratio (its Poisson ratio) and its density.  Draw
    order: beta[N+1], then h[N]."""
    ratio = np.asarray(m.alpha, np.float64) / np.asarray(m.beta, np.float64)
    beta = np.asarray(m.beta, np.float64) * (1.0 + step * rng.standard_normal(len(m.beta)))
    h = np.asarray(m.h, np.float64) * (1.0 + step * rng.standard_normal(len(m.h)))
    beta = np.maximum(beta, 1.0)
    h = np.maximum(h, 1e-3)
    return LayeredModel(h, ratio * beta, beta, np.asarray(m.rho, np.float64).copy())


def metropolis_accept(rng: np.random.Generator, current: np.ndarray, proposed: np.ndarray,
                      temperature: float) -> np.ndarray:
    """Accept where log u < -(proposed - current) / temperature, u ~ U(0, 1):
    always when the misfit does not grow; never when the proposal's misfit
    is NaN (a curve with no sign change).  One uniform per chain."""
    u = rng.uniform(size=current.shape[0])
    with np.errstate(invalid="ignore", over="ignore"):
        delta = (proposed - current) / temperature
        ok = np.isfinite(proposed) & ((delta <= 0.0) | (np.log(np.maximum(u, 1e-300)) < -delta))
        # a chain stuck on a NaN misfit moves to any finite proposal
        ok |= ~np.isfinite(current) & np.isfinite(proposed)
    return ok


@dataclass
class Population:
    """Models of equal layer count, one per row: h [C, N]; alpha, beta, rho
    [C, N+1].  Indexing and iteration give LayeredModel views."""

    h: np.ndarray
    alpha: np.ndarray
    beta: np.ndarray
    rho: np.ndarray

    def __len__(self) -> int:
        return int(self.beta.shape[0])

    def __getitem__(self, i: int) -> LayeredModel:
        return LayeredModel(self.h[i], self.alpha[i], self.beta[i], self.rho[i])

    def __iter__(self):
        return (self[i] for i in range(len(self)))

    @staticmethod
    def stack(models: Sequence) -> "Population":
        n = {int(np.asarray(m.h).shape[0]) for m in models}
        if len(n) > 1:
            raise ValueError("all models must have the same number of layers")
        f = lambda name: np.stack([np.asarray(getattr(m, name), np.float64) for m in models])
        return Population(f("h"), f("alpha"), f("beta"), f("rho"))


@dataclass
class ChainResult:
    best_models: List[LayeredModel]
    best_misfit: np.ndarray          # [chains]
    final_misfit: np.ndarray         # [chains]
    start_misfit: np.ndarray         # [chains]
    accepted: np.ndarray             # [chains] accepted proposals
    iterations: int
    trace: np.ndarray = field(repr=False, default=None)  # [iterations + 1, chains] current misfit

    @property
    def acceptance_rate(self) -> float:
        return float(self.accepted.sum()) / float(max(1, self.accepted.size * self.iterations))


def run_chains(evaluate: Callable[[Sequence], np.ndarray], start: Sequence, iterations: int,
               step: float = 0.02, temperature: float = 0.01, seed: int = 0) -> ChainResult:
    """Advance len(start) chains `iterations` steps.  The start models must
    share their layer count.  `evaluate(population)` returns the misfit of
    each model of a Population (NaN allowed).  A proposal is `perturb`'s,
    drawn for all chains at once; draw order per step: beta [chains, N+1],
    then h [chains, N], then one uniform per chain (metropolis_accept)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cur = Population.stack(start)
    ratio = cur.alpha / cur.beta
    mis = np.asarray(evaluate(cur), np.float64).copy()
    best = Population(cur.h.copy(), cur.alpha.copy(), cur.beta.copy(), cur.rho.copy())
    best_mis = mis.copy()
    accepted = np.zeros(len(cur), np.int64)
    trace = np.empty((iterations + 1, len(cur)))
    trace[0] = mis
    start_mis = mis.copy()
    for it in range(iterations):
        beta = np.maximum(cur.beta * (1.0 + step * rng.standard_normal(cur.beta.shape)), 1.0)
        h = np.maximum(cur.h * (1.0 + step * rng.standard_normal(cur.h.shape)), 1e-3)
        prop = Population(h, ratio * beta, beta, cur.rho)
        pm = np.asarray(evaluate(prop), np.float64)
        ok = metropolis_accept(rng, mis, pm, temperature)
        rows = ok[:, None]
        cur = Population(np.where(rows, prop.h, cur.h), np.where(rows, prop.alpha, cur.alpha),
                         np.where(rows, prop.beta, cur.beta), cur.rho)
        mis = np.where(ok, pm, mis)
        accepted += ok
        better = ok & ~(best_mis <= pm)  # also replaces a NaN best
        if better.any():
            b = better[:, None]
            best = Population(np.where(b, prop.h, best.h), np.where(b, prop.alpha, best.alpha),
                              np.where(b, prop.beta, best.beta), best.rho)
            best_mis = np.where(better, pm, best_mis)
        trace[it + 1] = mis
    best_models = [LayeredModel(m.h.copy(), m.alpha.copy(), m.beta.copy(), m.rho.copy()) for m in best]
    return ChainResult(best_models, best_mis, mis.copy(), start_mis, accepted, iterations, trace)


class DeviceEvaluator:
    """Misfits of many models against one experimental curve on the GPU.

    All models share the test-velocity grid and the wavelengths of the
    experimental curve C_e.  One call flattens the models, runs the batched
    sweep with device-resident outputs (C_t only: the misfit uses the grid
    velocity of each pick, so the root refinement is skipped) with Algorithm
    2's misfit reduced in the same launch (masw_dispersion_batch_misfit), and
    copies back only the misfits.  With
    inertia=True the picks come from the FP64 inertia-count search
    (MASW_SEARCH_INERTIA; prec is then FP64), whose C_t equal the FP64 walk's
    bit for bit."""

    def __init__(self, ctx, c_test, lambdas, C_e, prec: int = MASW_PREC_SPLIT, device: str = "cuda:0",
                 inertia: bool = False):
        import torch

        self.torch = torch
        self.ctx = ctx
        self.dev = torch.device(device)
        self.prec = MASW_PREC_FP64 if inertia else prec
        self.flags = MASW_NO_REFINE | (MASW_SEARCH_INERTIA if inertia else 0)
        self.lam = np.ascontiguousarray(lambdas, np.float64)
        self.C_e = np.ascontiguousarray(C_e, np.float64)
        if self.C_e.shape != self.lam.shape:
            raise ValueError("C_e and lambdas must have the same length")
        self.c = torch.as_tensor(np.ascontiguousarray(c_test, np.float64), device=self.dev)
        self._per_n = {}  # chains -> (lambda_off, lam, C_e) tiled on the device
        self.models_evaluated = 0

    def _tiled(self, n: int):
        if n not in self._per_n:
            W = self.lam.shape[0]
            t = lambda x: self.torch.as_tensor(np.ascontiguousarray(x), device=self.dev)
            self._per_n[n] = (t(np.arange(n + 1, dtype=np.int32) * np.int32(W)), t(np.tile(self.lam, n)),
                              t(np.tile(self.C_e, n)))
        return self._per_n[n]

    def __call__(self, models) -> np.ndarray:
        torch, dev = self.torch, self.dev
        pop = models if isinstance(models, Population) else Population.stack(list(models))
        n, N = len(pop), int(pop.h.shape[1])
        lam_off, lam, ce = self._tiled(n)
        t = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float64).ravel(), device=dev)
        layer_off = torch.as_tensor(np.arange(n + 1, dtype=np.int32) * np.int32(N), device=dev)
        W = int(lam.shape[0])
        f64, i32 = torch.float64, torch.int32
        ct = torch.empty(W, dtype=f64, device=dev)
        idx = torch.empty(W, dtype=i32, device=dev)
        st = torch.empty(W, dtype=i32, device=dev)
        mis = torch.empty(n, dtype=f64, device=dev)
        masw_dispersion_batch_misfit(self.ctx, self.c, layer_off, t(pop.h), t(pop.alpha), t(pop.beta), t(pop.rho),
                                     lam_off, lam, self.prec, self.flags, None, ct, idx, st, None, ce, mis)
        self.models_evaluated += n
        return mis.cpu().numpy()


def synthetic_curve(C_t: np.ndarray, rel_noise: float, seed: int = 0) -> np.ndarray:
    """An experimental curve stand-in: a model's C_t times (1 + rel_noise N(0, 1))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.asarray(C_t, np.float64) * (1.0 + rel_noise * rng.standard_normal(len(C_t)))


def misfit_scale(C_e: np.ndarray, dc: float) -> float:
    """The misfit of an error of one grid step dc at every wavelength,
    mean(dc / C_e): a natural unit for the temperature."""
    C_e = np.asarray(C_e, np.float64)
    return float(np.mean(dc / C_e)) if C_e.size else math.nan
