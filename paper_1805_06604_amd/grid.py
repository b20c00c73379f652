"""Batched multi-start and parameter-grid runs of E-A-HALS and E-ANLS on one GPU.

This is the tuning protocol of arXiv 1805.06604, section 5.3. Every parameter set (β₀, η, γ, γ̄,
hp) runs on several data sets and random initializations, and the runs are scored by the error
measure of eq. (relerr):
E(k) = ρ(k) − e_min, where e_min is the lowest final error of any run on the same data set
(0 for exactly factorable data). For each hp, the best and worst parameter sets are those with the
smallest and largest final mean E.

All runs of a grid go through one batch (``Batch``): each run is an independent problem advanced
by the grouped kernels, so a grid of about a thousand small solves costs a few hundred batch
iterations rather than a thousand solves. This module only schedules runs and averages the traces
the library returns.
"""
from __future__ import annotations

import argparse
import dataclasses
import itertools
import json

import numpy as np

from .binding import Batch, Inner

# The grid of section 5.3 (3^4 extrapolated variants and the plain algorithm); for E-A-HALS on
# the synthetic sets the extra (1.005, 1.001) pair tried there is included.
BETA0 = (0.25, 0.5, 0.75)
ETA = (1.5, 2.0, 3.0)
GAMMAS_ANLS = ((1.01, 1.005), (1.05, 1.01), (1.1, 1.05))
GAMMAS = ((1.005, 1.001),) + GAMMAS_ANLS
HP = (1, 2, 3)


@dataclasses.dataclass(frozen=True)
class Variant:
    hp: int
    beta0: float
    eta: float
    gamma: float
    gamma_bar: float

    @property
    def plain(self) -> bool:
        """β₀ = 0: no extrapolation (A-HALS)."""
        return self.beta0 == 0.0

    def params(self) -> dict:
        return dict(hp=self.hp, beta0=self.beta0, eta=self.eta, gamma=self.gamma,
                    gamma_bar=self.gamma_bar)

    def label(self) -> str:
        """Parameters of the variant (A-HALS / ANLS when plain)."""
        if self.plain:
            return "plain"
        return (f"hp={self.hp} beta0={self.beta0:g} eta={self.eta:g} "
                f"gamma={self.gamma:g} gamma_bar={self.gamma_bar:g}")


PLAIN = Variant(hp=1, beta0=0.0, eta=1.5, gamma=1.01, gamma_bar=1.005)


def grid_variants(beta0=BETA0, eta=ETA, gammas=GAMMAS, hp=HP, plain=True) -> list[Variant]:
    """Every combination of the grid, plus plain A-HALS."""
    out = [Variant(h, b, e, g, gb) for h, b, e, (g, gb) in itertools.product(hp, beta0, eta, gammas)]
    return ([PLAIN] if plain else []) + out


def run(problems, variants, max_iter, inner_k=10, hbm_budget=8 << 30, max_active=4096,
        check_every=50, inner_rule=Inner.FIXED):
    """Solves every (variant, problem) pair with max_iter outer iterations through one batch.
    Each problem carries its own X, W0 and H0, so a problem stands for one data set with one
    initialization. inner_rule FIXED runs E-A-HALS (inner_k sweeps), EXACT runs E-ANLS.
    Returns the Results as a list of lists, indexed [variant][problem]."""
    res = [[None] * len(problems) for _ in variants]
    with Batch(hbm_budget, max_active=max_active, check_every=check_every) as B:
        tickets = {}
        for vi, v in enumerate(variants):
            for pi, p in enumerate(problems):
                t = B.submit(p.X, p.r, p.W0, p.H0, max_iter=max_iter, inner_k=inner_k,
                             inner_rule=inner_rule, **v.params())
                tickets[t] = (vi, pi)
        while tickets:
            B.step(check_every)
            for t in list(tickets):
                g = B.result(t)
                if g is not None:
                    vi, pi = tickets.pop(t)
                    res[vi][pi] = g
    return res


def error_curves(results, e_min):
    """E(k) per run: array [variant][problem][k], with e_min per problem."""
    tr = np.array([[g.trace for g in row] for row in results])
    return tr - np.asarray(e_min)[None, :, None]


def summarize(variants, results, e_min=None):
    """Final mean and standard deviation of ρ and of E per variant, and the best and worst
    variant for each hp by the final mean E. If e_min is None, it is the lowest final ρ per
    problem over all variants."""
    final = np.array([[g.trace[-1] for g in row] for row in results])
    if e_min is None:
        e_min = final.min(axis=0)
    E = final - np.asarray(e_min)[None, :]
    rows = [dict(variant=v.label(), hp=v.hp, rho_mean=float(final[i].mean()),
                 rho_std=float(final[i].std(ddof=1)) if final.shape[1] > 1 else 0.0,
                 E_mean=float(E[i].mean()))
            for i, v in enumerate(variants)]
    best_worst = {}
    for hp in sorted({v.hp for v in variants if not v.plain}):
        idx = [i for i, v in enumerate(variants) if v.hp == hp and not v.plain]
        best = min(idx, key=lambda i: E[i].mean())
        worst = max(idx, key=lambda i: E[i].mean())
        best_worst[hp] = dict(best=rows[best], worst=rows[worst])
    return dict(rows=rows, best_worst=best_worst, e_min=[float(x) for x in e_min])


def main(argv=None):
    import time

    import nmf_synth as S

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--kind", choices=["lowrank", "fullrank"], default="fullrank")
    ap.add_argument("--seeds", type=int, default=10)
    ap.add_argument("--iters", type=int, default=500)
    ap.add_argument("--r", type=int, default=20)
    ap.add_argument("--algo", choices=["e-a-hals", "e-anls"], default="e-a-hals")
    args = ap.parse_args(argv)
    gen = S.lowrank if args.kind == "lowrank" else S.fullrank
    problems = [gen(s, r=args.r) for s in range(args.seeds)]
    anls = args.algo == "e-anls"
    variants = grid_variants(gammas=GAMMAS_ANLS) if anls else grid_variants()
    t0 = time.perf_counter()
    results = run(problems, variants, args.iters, inner_rule=Inner.EXACT if anls else Inner.FIXED)
    dt = time.perf_counter() - t0
    summ = summarize(variants, results, e_min=[0.0] * len(problems) if args.kind == "lowrank" else None)
    out = dict(algo=args.algo, kind=args.kind, seeds=args.seeds, iters=args.iters,
               runs=len(variants) * len(problems),
               seconds=dt, best_worst=summ["best_worst"],
               plain=summ["rows"][0])
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
