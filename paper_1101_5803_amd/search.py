"""Genetic search over the seven lens parameters, with the batched solve as fitness.

The outer loop of the method (Sec. 3.1.1 and App. A.1): a real-valued genetic
algorithm proposes lens parameter sets and the semilinear solve scores each
by chi^2 at its L-curve corner (Sec. 2.6).  This module is host logic in
FP64; every fitness evaluation is one batched call of the device solve, and
the optional surrogate runs on the device MLP kernels.

One generation of the simplified Ferret GA:
  * duplicate the population; each copy moves towards a partner by a fraction
    |xi| * XOver.strength of the distance (X-type crossover, probability 1);
  * each gene mutates with probability PMutate by a Gaussian step of
    mutation.scale (genes live in the unit box: the prior box mapped to
    [0, 1]; the two angle genes wrap, the others are clipped);
  * binary tournament: modified individual perm[i] meets unmodified
    individual i and replaces it only when its fitness is strictly lower.
Linkage learning, niching, adaptive control and islands are not modelled.
All random numbers are inputs (a dict of one generation's draws).

The final source refinement (SourceRefinement, Sec. 3.2) runs the same GA
over the source nodes within bounds about the regularised solution, with
the device's batched candidate-source chi^2 as fitness.

The swarm (SwarmSearch, Sec. 3.1.2 and App. A.2) is the second outer loop:
particles pulled towards their own and the swarm's best positions, moved
along Locust's exact damped-oscillator orbits or by Eq. 21 itself.

Surrogate screening (not in the paper): each parent proposes `fanout`
candidates; the device MLP predicts ln chi^2 of every candidate; each
parent's best-predicted candidate goes to the full solve and the tournament.
Every full solve joins the surrogate's training set.
"""
from __future__ import annotations

import dataclasses
import json
import math

import numpy as np
import torch

from . import ops

PERIODIC_GENES = (2, 4)   # position angle of the lens and of the shear


@dataclasses.dataclass(frozen=True)
class GAConfig:
    xover_strength: float = 0.25
    pmutate: float = 0.05
    mutation_scale: float = 0.25

    @classmethod
    def from_json(cls, path: str) -> "GAConfig":
        """Ferret strategy parameters from a JSON file with Ferret's key names."""
        with open(path) as f:
            d = json.load(f)
        return cls(xover_strength=float(d.get("XOver.strength", 0.25)), pmutate=float(d.get("mutation.PMutate", 0.05)),
                   mutation_scale=float(d.get("mutation.scale", 0.25)))


@dataclasses.dataclass(frozen=True)
class Box:
    """Prior box: unit genes u map to lo + u (hi - lo)."""
    lo: np.ndarray
    hi: np.ndarray

    def to_phys(self, u: np.ndarray) -> np.ndarray:
        return self.lo + np.asarray(u, dtype=np.float64) * (self.hi - self.lo)

    def to_unit(self, p: np.ndarray) -> np.ndarray:
        return (np.asarray(p, dtype=np.float64) - self.lo) / (self.hi - self.lo)


def make_offspring(X: np.ndarray, parent: np.ndarray, partner: np.ndarray, xi: np.ndarray, mut_u: np.ndarray,
                   mut_z: np.ndarray, cfg: GAConfig, periodic=PERIODIC_GENES) -> np.ndarray:
    """Crossover + mutation of copies of X[parent] (one row per candidate); the genes in `periodic`
    wrap, the others are clipped to [0, 1]."""
    base = X[parent]
    step = (np.abs(xi) * cfg.xover_strength)[:, None]
    Y = base + step * (X[partner] - base)
    Y = Y + np.where(mut_u < cfg.pmutate, cfg.mutation_scale * mut_z, 0.0)
    wrap = np.zeros(X.shape[1], dtype=bool)
    wrap[list(periodic)] = True
    return np.where(wrap[None, :], np.mod(Y, 1.0), np.clip(Y, 0.0, 1.0))


def tournament(X, fX, Y, fY, perm):
    """Candidate perm[i] against incumbent i; the candidate wins only when strictly better."""
    win = fY[perm] < fX
    return np.where(win[:, None], Y[perm], X), np.where(win, fY[perm], fX)


class SolverFitness:
    """chi^2 at the L-curve corner of lens parameter sets, from one batched device solve.

    Every member uses the same source grid side `ns`.  A member whose solve
    or corner is not valid (no mapped pixel, invalid parameters, degenerate
    L-curve) or whose corner solve did not converge gets fitness +inf.  A
    member whose curve has an unconverged point elsewhere keeps its corner
    (its corner status says so).
    """

    def __init__(self, solver: ops.Solver, box: Box, ns: int, lambdas, tol: float = 1e-7, maxit: int = 4000):
        self.solver, self.box, self.ns = solver, box, int(ns)
        self.lambdas = [float(x) for x in lambdas]
        self.tol, self.maxit = float(tol), int(maxit)
        self.evals = 0
        self._out = None
        self._cap = 0

    def __call__(self, U: np.ndarray) -> np.ndarray:
        U = np.asarray(U, dtype=np.float64)
        n = U.shape[0]
        dev = self.solver.device
        if n > self._cap:
            self._cap = n
            self._out = self.solver.alloc_result(n * self.ns * self.ns, n, len(self.lambdas))
        out = {k: v for k, v in self._out.items()}
        lens = torch.tensor(self.box.to_phys(U), dtype=torch.float64, device=dev)
        ns = torch.full((n,), self.ns, dtype=torch.int32, device=dev)
        res = self.solver.solve_semilinear(lens, ns, self.lambdas, tol=self.tol, maxit=self.maxit, max_ns=self.ns,
                                           out=out)
        chi2 = res["chi2"][:n].cpu().numpy()
        k = res["k_star"][:n].cpu().numpy()
        cs = res["corner_status"][:n].cpu().numpy()
        st = res["status"][:n].cpu().numpy()
        self.evals += n
        f = np.full(n, np.inf)
        ok = (k >= 0) & np.isin(cs, (0, 1, 3))
        rows = np.nonzero(ok)[0]
        ok[rows] = st[rows, k[rows]] == 0
        f[ok] = chi2[np.nonzero(ok)[0], k[ok]]
        return f


class Surrogate:
    """Device MLP predicting ln chi^2 from unit genes (inputs 2u - 1, standardised target).

    Targets above the `clip_quantile` quantile of the training set are clipped
    to it, so the network spends its capacity on the low-chi^2 region that the
    screen has to rank; the rest of the box only needs to predict "bad".
    """

    def __init__(self, device, seed: int = 0, lr: float = 1e-3, batch: int = 1024, clip_quantile: float = 0.1):
        rng = np.random.default_rng(seed)
        w = []
        for a, b in ((7, 256), (256, 256), (256, 1)):
            lim = math.sqrt(6.0 / a)
            w.append((rng.uniform(-lim, lim, size=(a, b)), np.zeros(b)))
        self.device = device
        self.params = ops.mlp_pack(w, device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.lr, self.batch = float(lr), int(batch)
        self.clip_quantile = float(clip_quantile)   # targets above this quantile are clipped to it
        self.mu, self.sd = 0.0, 1.0

    def predict(self, U: np.ndarray) -> np.ndarray:
        x = torch.tensor(2.0 * np.asarray(U) - 1.0, dtype=torch.float32, device=self.device)
        y = ops.mlp_forward(self.params, x).cpu().numpy().astype(np.float64)
        return self.mu + self.sd * y

    def train(self, U: np.ndarray, lnf: np.ndarray, steps: int, seed: int) -> float:
        """`steps` Adam steps on minibatches drawn (seeded) from (U, ln f); returns the last batch loss."""
        U = np.asarray(U, dtype=np.float64)
        lnf = np.asarray(lnf, dtype=np.float64)
        if self.clip_quantile < 1.0:
            lnf = np.minimum(lnf, np.quantile(lnf, self.clip_quantile))
        self.mu, self.sd = float(lnf.mean()), float(lnf.std() + 1e-12)
        x = torch.tensor(2.0 * U - 1.0, dtype=torch.float32, device=self.device)
        y = torch.tensor((lnf - self.mu) / self.sd, dtype=torch.float32, device=self.device)
        rng = np.random.default_rng(seed)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        n = U.shape[0]
        b = min(self.batch, n)
        for _ in range(steps):
            idx = torch.tensor(rng.choice(n, size=b, replace=False), device=self.device)
            self.t += 1
            ops.mlp_train_step(self.params, self.m, self.v, x[idx].contiguous(), y[idx].contiguous(), self.lr, self.t,
                               loss=loss)
        return float(loss.item())

    def state(self) -> dict:
        return dict(s_params=self.params.cpu().numpy(), s_m=self.m.cpu().numpy(), s_v=self.v.cpu().numpy(),
                    s_t=self.t, s_mu=self.mu, s_sd=self.sd)

    def load_state(self, z) -> None:
        self.params = torch.tensor(z["s_params"], device=self.device)
        self.m = torch.tensor(z["s_m"], device=self.device)
        self.v = torch.tensor(z["s_v"], device=self.device)
        self.t = int(z["s_t"])
        self.mu, self.sd = float(z["s_mu"]), float(z["s_sd"])


class GeneticSearch:
    """Plain GA: every offspring is fully solved.  `fitness` maps unit genes (n, 7) -> (n,)."""

    def __init__(self, fitness, X0: np.ndarray, cfg: GAConfig = GAConfig(), log=None):
        self.fitness, self.cfg, self.log = fitness, cfg, log
        self.X = np.array(X0, dtype=np.float64)
        self.fX = fitness(self.X)
        self.generation = 0
        self.full_solves = self.X.shape[0]
        self.history = [float(np.min(self.fX))]
        self.data_U = [self.X.copy()]
        self.data_f = [self.fX.copy()]

    @property
    def pop(self) -> int:
        return self.X.shape[0]

    def _record(self, Y, fY, extra=None):
        self.data_U.append(Y)
        self.data_f.append(fY)
        self.generation += 1
        self.full_solves += Y.shape[0]
        self.history.append(float(np.min(self.fX)))
        if self.log is not None:
            rec = dict(generation=self.generation, full_solves=self.full_solves, best=self.history[-1],
                       median=float(np.median(self.fX)))
            rec.update(extra or {})
            self.log(rec)

    def step(self, draws: dict) -> None:
        """One generation from one generation's draws (arrays of length pop)."""
        P = self.pop
        Y = make_offspring(self.X, np.arange(P), draws["partner"], draws["xstrength"], draws["mut_mask"],
                           draws["mut_step"], self.cfg)
        fY = self.fitness(Y)
        self.X, self.fX = tournament(self.X, self.fX, Y, fY, draws["perm"])
        self._record(Y, fY)

    def training_set(self):
        U = np.concatenate(self.data_U)
        f = np.concatenate(self.data_f)
        ok = np.isfinite(f) & (f > 0)
        return U[ok], np.log(f[ok])

    def save(self, path: str) -> None:
        np.savez(path, X=self.X, fX=self.fX, generation=self.generation, full_solves=self.full_solves,
                 history=np.array(self.history), data_U=np.concatenate(self.data_U),
                 data_f=np.concatenate(self.data_f), **self._extra_state())

    def _extra_state(self) -> dict:
        return {}

    @classmethod
    def resume(cls, path: str, fitness, cfg: GAConfig = GAConfig(), log=None, **kw):
        """Rebuild a search from a checkpoint without re-evaluating anything."""
        z = np.load(path, allow_pickle=False)
        self = cls.__new__(cls)
        self.fitness, self.cfg, self.log = fitness, cfg, log
        self.X, self.fX = z["X"].copy(), z["fX"].copy()
        self.generation, self.full_solves = int(z["generation"]), int(z["full_solves"])
        self.history = [float(v) for v in z["history"]]
        self.data_U, self.data_f = [z["data_U"].copy()], [z["data_f"].copy()]
        self._resume_extra(z, **kw)
        return self

    def _resume_extra(self, z, **kw) -> None:
        pass


class ScreenedSearch(GeneticSearch):
    """GA whose offspring are pre-screened by the device surrogate.

    Each generation: fanout * pop candidates (candidate c descends from parent
    c mod pop) and a surrogate prediction of ln chi^2 for all of them.  pop
    candidates are fully solved and enter the tournament:
      * select="per_parent" (default): each parent's candidate with the lowest
        prediction (ties to the first), so every parent still has exactly one
        child, as in the plain GA;
      * select="global": the pop lowest predictions over all candidates.
    Then `train_steps` Adam steps on every full solve so far.
    """

    def __init__(self, fitness, X0, surrogate: Surrogate, fanout: int = 10, train_steps: int = 50,
                 cfg: GAConfig = GAConfig(), log=None, pretrain_steps: int = 200, select: str = "per_parent"):
        super().__init__(fitness, X0, cfg, log)
        if select not in ("per_parent", "global"):
            raise ValueError("select must be 'per_parent' or 'global'")
        self.select = select
        self.surrogate, self.fanout, self.train_steps = surrogate, int(fanout), int(train_steps)
        U, lnf = self.training_set()
        if pretrain_steps and U.shape[0]:
            self.surrogate.train(U, lnf, pretrain_steps, seed=0)

    def step(self, draws: dict) -> None:
        """One generation from draws of length fanout * pop."""
        P = self.pop
        C = self.fanout * P
        cand = make_offspring(self.X, np.arange(C) % P, draws["partner"][:C] % P, draws["xstrength"][:C],
                              draws["mut_mask"][:C], draws["mut_step"][:C], self.cfg)
        pred = self.surrogate.predict(cand)
        if self.select == "global":
            pick = np.argsort(pred, kind="stable")[:P]
        else:   # candidates of parent p are p, p + P, p + 2P, ...
            pick = np.arange(P) + P * np.argmin(pred.reshape(self.fanout, P), axis=0)
        Y = cand[pick]
        fY = self.fitness(Y)
        perm = draws["perm"][:C]
        perm = perm[perm < P]
        self.X, self.fX = tournament(self.X, self.fX, Y, fY, perm)
        ok = np.isfinite(fY)
        rmse = float(np.sqrt(np.mean((pred[pick][ok] - np.log(fY[ok])) ** 2))) if ok.any() else float("nan")
        rank = _spearman(pred[pick][ok], fY[ok]) if ok.sum() > 2 else float("nan")
        loss = float("nan")
        self._record(Y, fY, dict(surrogate_rmse=rmse, surrogate_rank_corr=rank))
        if self.train_steps:
            U, lnf = self.training_set()
            loss = self.surrogate.train(U, lnf, self.train_steps, seed=self.generation)
        if self.log is not None:
            self.log(dict(generation=self.generation, surrogate_train_loss=loss))

    def _extra_state(self) -> dict:
        return dict(fanout=self.fanout, train_steps=self.train_steps, select=self.select, **self.surrogate.state())

    def _resume_extra(self, z, surrogate: Surrogate | None = None) -> None:
        self.fanout, self.train_steps = int(z["fanout"]), int(z["train_steps"])
        self.select = str(z["select"])
        self.surrogate = surrogate
        self.surrogate.load_state(z)


@dataclasses.dataclass(frozen=True)
class SwarmConfig:
    """Locust strategy parameters (App. A.2) and the orbit form."""
    cp: float = 1.0        # personal-best spring constant
    cg: float = 0.5        # swarm-best spring constant
    dt: float = 1.0        # time step
    tdamp: float = 10.0    # damping time in units of the critical one
    exact: bool = True     # exact damped-oscillator orbits (Locust); False: the Euler form of Eq. 21


class SwarmSearch:
    """Particle swarm over unit genes (Sec. 3.1.2, Eq. 21; App. A.2).

    Every particle is pulled towards its own best position and the swarm's
    best by springs c_p xi_p and c_g xi_g and damped over t_damp =
    TDamp / (2 sqrt((c_p + c_g) / 2)) (TDamp = 1: critical damping at the
    mean spring constant).  With `exact` each step moves the particles along
    the exact solution of that damped oscillator with the springs held fixed
    (as Locust does); otherwise by Eq. 21 itself, the position moving with
    the velocity of the start of the step.  The angle genes wrap; another
    gene that leaves the unit box stops on the wall with zero velocity there.
    Velocities start at zero; a particle's best moves only on a strictly lower
    fitness; the swarm's best is the lowest personal best (first on a tie).
    `fitness` maps unit genes (n, 7) -> (n,); every step is one batched call.
    All random numbers are inputs (xi_p, xi_g: one U(0, 1) draw per particle
    and step).
    """

    def __init__(self, fitness, X0: np.ndarray, cfg: SwarmConfig = SwarmConfig(), log=None):
        self.fitness, self.cfg, self.log = fitness, cfg, log
        self.X = np.array(X0, dtype=np.float64)
        self.V = np.zeros_like(self.X)
        f = np.asarray(fitness(self.X), dtype=np.float64)
        self.P, self.fP = self.X.copy(), f.copy()
        self.g = int(np.argmin(self.fP))
        self.steps = 0
        self.evals = self.X.shape[0]
        self.history = [float(self.fP[self.g])]
        self.t_damp = cfg.tdamp / (2.0 * math.sqrt(0.5 * (cfg.cp + cfg.cg)))

    @property
    def best(self):
        return self.P[self.g].copy(), float(self.fP[self.g])

    def _move(self, xi_p: np.ndarray, xi_g: np.ndarray):
        c, dt = self.cfg, self.cfg.dt
        X, V = self.X, self.V
        kp = (c.cp * xi_p)[:, None]
        kg = (c.cg * xi_g)[:, None]
        G = self.P[self.g][None, :]
        if not c.exact:
            Vn = V * (1.0 - dt / self.t_damp) + (kp * (self.P - X) + kg * (G - X)) * dt
            return X + V * dt, Vn
        # exact orbit of y'' = -gamma y' - k y about the spring centre, per particle (k, gamma scalars)
        k = kp + kg
        kk = np.where(k > 0.0, k, 1.0)
        ctr = np.where(k > 0.0, (kp * self.P + kg * G) / kk, X)
        y0, v0 = X - ctr, V
        gam = 1.0 / self.t_damp
        disc = gam * gam - 4.0 * k
        Xn = np.empty_like(X)
        Vn = np.empty_like(V)
        # no spring: free damped motion
        free = (k <= 0.0)[:, 0]
        e = math.exp(-gam * dt)
        Xn[free] = X[free] + V[free] * (1.0 - e) / gam
        Vn[free] = V[free] * e
        under = (~free) & (disc < 0.0)[:, 0]
        if under.any():
            kk_ = k[under]
            w = np.sqrt(kk_ - 0.25 * gam * gam)
            ed = math.exp(-0.5 * gam * dt)
            cs, sn = np.cos(w * dt), np.sin(w * dt)
            a, b = y0[under], v0[under]
            Xn[under] = ctr[under] + ed * (a * cs + (b + 0.5 * gam * a) / w * sn)
            Vn[under] = ed * (b * cs - (0.5 * gam * b + kk_ * a) / w * sn)
        over = (~free) & (disc > 0.0)[:, 0]
        if over.any():
            sq = np.sqrt(disc[over])
            r1, r2 = 0.5 * (-gam + sq), 0.5 * (-gam - sq)
            a, b = y0[over], v0[over]
            c1 = (b - r2 * a) / (r1 - r2)
            c2 = a - c1
            e1, e2 = np.exp(r1 * dt), np.exp(r2 * dt)
            Xn[over] = ctr[over] + c1 * e1 + c2 * e2
            Vn[over] = r1 * c1 * e1 + r2 * c2 * e2
        crit = (~free) & (disc == 0.0)[:, 0]
        if crit.any():
            a, b = y0[crit], v0[crit]
            bb = b + 0.5 * gam * a
            ed = math.exp(-0.5 * gam * dt)
            Xn[crit] = ctr[crit] + (a + bb * dt) * ed
            Vn[crit] = (b - 0.5 * gam * bb * dt) * ed
        return Xn, Vn

    def step(self, xi_p: np.ndarray, xi_g: np.ndarray) -> None:
        """One swarm step from this step's draws (arrays of length N)."""
        X, V = self._move(np.asarray(xi_p, dtype=np.float64), np.asarray(xi_g, dtype=np.float64))
        for gdx in range(X.shape[1]):
            if gdx in PERIODIC_GENES:
                X[:, gdx] = np.mod(X[:, gdx], 1.0)
            else:
                out = (X[:, gdx] < 0.0) | (X[:, gdx] > 1.0)
                X[:, gdx] = np.clip(X[:, gdx], 0.0, 1.0)
                V[out, gdx] = 0.0
        self.X, self.V = X, V
        f = np.asarray(self.fitness(X), dtype=np.float64)
        better = f < self.fP
        self.P[better] = X[better]
        self.fP[better] = f[better]
        self.g = int(np.argmin(self.fP))
        self.steps += 1
        self.evals += X.shape[0]
        self.history.append(float(self.fP[self.g]))
        if self.log is not None:
            self.log(dict(step=self.steps, evals=self.evals, best=self.history[-1], median=float(np.median(f))))


class SourceRefinement:
    """Bounded genetic search over the source nodes for a fixed lens (Sec. 3.2).

    Every node is a free parameter within bounds that keep the source
    non-negative: a window about the optimally regularised solution s*
    (+-25 % of s*_i for s*_i >= 0, [0, |s*_i| + 15 %] for s*_i < 0), or the
    full box [0, 1.1 max s*] (Sec. 4).  Genes are unit coordinates, s = lo +
    u (hi - lo); one generation is the GA of GeneticSearch over all nodes,
    none of them periodic; the first generation holds s* (its unit
    coordinates) as individual 0.  The fitness is the image chi^2 of every
    candidate source, one device call per generation (sl_chi2_sources), and
    chi2_r = chi2 / (J - I) since the nodes are the free parameters.
    All random numbers are inputs.
    """

    def __init__(self, solver: ops.Solver | None, lens, ns: int, s_star, X0: np.ndarray, cfg: GAConfig = GAConfig(),
                 bounds: str = "window", log=None, fitness=None, n_pixels: int | None = None):
        """fitness (optional) maps physical sources (n, I) to chi^2 instead of the device call; n_pixels is
        J when no solver is given."""
        self.solver, self.cfg, self.log = solver, cfg, log
        self._fit = fitness
        self.lens = np.asarray(lens, dtype=np.float64)
        self.ns = int(ns)
        s = np.asarray(s_star, dtype=np.float64).reshape(-1)
        if bounds == "window":
            self.lo = np.where(s >= 0.0, 0.75 * s, 0.0)
            self.hi = np.where(s >= 0.0, 1.25 * s, 1.15 * np.abs(s))
        else:
            self.lo, self.hi = np.zeros_like(s), np.full_like(s, 1.1 * s.max())
        span = self.hi - self.lo
        u0 = np.clip(np.divide(s - self.lo, span, out=np.zeros_like(s), where=span > 0.0), 0.0, 1.0)
        self.X = np.array(X0, dtype=np.float64)
        self.X[0] = u0
        self.evals = 0
        self.fX = self._fitness(self.X)
        self.generation = 0
        self.history = [float(self.fX.min())]
        self.dof = (solver.grid.J if solver is not None else int(n_pixels)) - s.size

    def sources(self, U: np.ndarray) -> np.ndarray:
        return self.lo + np.asarray(U) * (self.hi - self.lo)

    def _fitness(self, U: np.ndarray) -> np.ndarray:
        self.evals += U.shape[0]
        if self._fit is not None:
            return np.asarray(self._fit(self.sources(U)), dtype=np.float64)
        S = torch.tensor(self.sources(U), dtype=torch.float64, device=self.solver.device)
        return self.solver.chi2_sources(self.lens, self.ns, S).cpu().numpy()

    @property
    def best(self):
        i = int(np.argmin(self.fX))
        return self.sources(self.X[i]), float(self.fX[i])

    def step(self, draws: dict) -> None:
        P = self.X.shape[0]
        Y = make_offspring(self.X, np.arange(P), draws["partner"], draws["xstrength"], draws["mut_mask"],
                           draws["mut_step"], self.cfg, periodic=())
        fY = self._fitness(Y)
        self.X, self.fX = tournament(self.X, self.fX, Y, fY, draws["perm"])
        self.generation += 1
        self.history.append(float(self.fX.min()))
        if self.log is not None:
            self.log(dict(generation=self.generation, evals=self.evals, best=self.history[-1],
                          best_chi2_r=self.history[-1] / self.dof))


def confidence_sets(P: np.ndarray, f: np.ndarray, dof: float, levels=(0.683, 0.954, 0.99), n_up: float | None = None):
    """Optimal set and confidence regions of the lens parameters (Sec. 3).

    P: (n, k) physical parameters of every evaluated solution, f: their chi^2,
    dof: the effective degrees of freedom of the best solution (J - gamma, the
    Monte Carlo estimate).  The fuzzy optimal set is chi^2 <= chi^2_min + N_u
    (N_u defaults to the 99 % threshold below).  The standard method (Press
    et al., joint confidence region of k parameters): chi^2 is rescaled by
    the best solution's reduced chi^2 (chi^2_min / dof) so that the best fit
    has chi^2_r = 1, and the region at level p holds the solutions within
    Delta(p) = the p quantile of the chi^2 distribution with k degrees of
    freedom of the minimum.  Returns dict(optimal=mask, levels={p: dict(mask,
    lo, hi)}) with per-parameter bounds over each region."""
    from scipy.stats import chi2 as chi2_dist
    P = np.asarray(P, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    ok = np.isfinite(f)
    i0 = int(np.argmin(np.where(ok, f, np.inf)))
    fmin = f[i0]
    scale = fmin / float(dof)
    k = P.shape[1]
    d99 = chi2_dist.ppf(max(levels), k)
    n_up = d99 * scale if n_up is None else float(n_up)
    out = {"optimal": ok & (f <= fmin + n_up), "best": P[i0].copy(), "chi2_r_min": scale, "levels": {}}
    for p in levels:
        m = ok & ((f - fmin) / scale <= chi2_dist.ppf(p, k))
        out["levels"][p] = {"mask": m, "delta_chi2": float(chi2_dist.ppf(p, k)),
                            "lo": P[m].min(axis=0), "hi": P[m].max(axis=0)}
    return out


def _spearman(a, b) -> float:
    ra = np.argsort(np.argsort(a))
    rb = np.argsort(np.argsort(b))
    return float(np.corrcoef(ra, rb)[0, 1])
