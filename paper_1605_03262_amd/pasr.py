"""Partially stirred reactor (PaSR) particle driver (App. C of the paper).

Many independent reactors of n_part particles each are advanced together, all
particles of all reactors forming one batch for the library's kernels.  Per
time step dt = 0.1 min(tau_res, tau_pair):
  * inflow/outflow: n_part dt / tau_res randomly chosen particles per reactor
    take an inflow composition (the fresh stream with probability 0.95, the
    pilot stream with 0.05, the premixed mass-flow split);
  * pairing: n_part dt / (2 tau_pair) random pairs, together with the inflowing
    particles and their partners, are shuffled into new pairs;
  * ceil(dt / dt_sub) sub-steps, dt_sub = 0.04 tau_mix, each a mixing
    fractional step (pyjac_mix_pairs: pairwise relaxation of enthalpy and mass
    fractions over the sub-step) followed by a reaction fractional step at
    constant pressure (pyjac_sdirk3_step, `react_steps` implicit steps).
The random events are drawn on the host from a seeded generator and passed to
the kernels (pairing array); every composition update runs on the GPU.

The paper advanced the reaction step with an adaptive general-purpose
integrator; here it is the library's own fixed-step SDIRK3 step, so the
particle states are representative of such a reactor (fresh, burning, mixed
and near-equilibrium compositions) rather than a converged trajectory.
"""
from __future__ import annotations

import math

import numpy as np

from . import NEWTON_FP64, Mechanism, _lib, _torch


class PaSR:
    def __init__(self, mech: Mechanism, n_reactors: int, fresh, pilot, p_pa: float, n_part: int = 100,
                 tau_res: float = 5e-3, tau_mix: float = 1e-3, tau_pair: float = 1e-3, react_steps: int = 4,
                 newton_iters: int = 10, seed: int = 0):
        """fresh, pilot: (T, Y_1..Y_{N-1}) compositions of the inflow streams
        (numpy, length N); p_pa: the reactor pressure.  newton_iters: the
        simplified-Newton iterations of each SDIRK3 stage (with 6, the
        acceptance test below rejected most full sub-steps of burning
        particles and their steps shrank to the floor; with 10 most particles
        take a sub-step in one implicit step)."""
        if n_part % 2:
            raise ValueError("n_part must be even")
        torch = _torch()
        self.mech, self.R, self.P = mech, n_reactors, n_part
        self.tau_res, self.tau_mix, self.tau_pair = tau_res, tau_mix, tau_pair
        self.react_steps, self.newton_iters = react_steps, newton_iters
        self.rng = np.random.default_rng(seed)
        self.fresh = np.asarray(fresh, dtype=np.float64)
        self.pilot = np.asarray(pilot, dtype=np.float64)
        N = mech.n_species
        n = n_reactors * n_part
        self.n = n
        # every particle starts from the pilot (burned) composition
        self.phi = torch.from_numpy(np.repeat(self.pilot[:, None], n, axis=1)).cuda()
        self.p = torch.full((n,), float(p_pa), dtype=torch.float64, device="cuda")
        self.partner = np.empty(n, dtype=np.int32)
        for r in range(n_reactors):
            idx = r * n_part + self.rng.permutation(n_part)
            self.partner[idx[0::2]] = idx[1::2]
            self.partner[idx[1::2]] = idx[0::2]
        self.dt = 0.1 * min(tau_res, tau_pair)
        self.n_sub = max(1, math.ceil(self.dt / (0.04 * tau_mix)))
        self.dt_sub = self.dt / self.n_sub
        self._work = torch.empty_like(self.phi)
        self._ws = torch.empty((max(_lib.pyjac_sdirk3_workspace_bytes(mech.handle, n, n, NEWTON_FP64), 1),),
                               dtype=torch.uint8, device="cuda")
        self._h = torch.full((n,), self.dt_sub / react_steps, dtype=torch.float64, device="cuda")
        self.time = 0.0

    def _count(self, mean: float) -> int:
        """Stochastic rounding of an expected event count."""
        base = math.floor(mean)
        return base + int(self.rng.random() < mean - base)

    def _events(self):
        """Inflow/outflow and pairing for one time step (host random draws)."""
        torch = _torch()
        inflow_idx, inflow_comp = [], []
        for r in range(self.R):
            base = r * self.P
            n_in = min(self._count(self.P * self.dt / self.tau_res), self.P)
            inflow = base + self.rng.choice(self.P, n_in, replace=False)
            for s in inflow:
                inflow_idx.append(s)
                inflow_comp.append(self.fresh if self.rng.random() < 0.95 else self.pilot)
            # pairs to re-pair: the inflowing particles with their partners and
            # n_part dt / (2 tau_pair) random pairs of the others
            members = set(inflow.tolist()) | {int(self.partner[s]) for s in inflow}
            others = [s for s in range(base, base + self.P) if s not in members and s < self.partner[s]
                      and int(self.partner[s]) not in members]
            n_pairs = min(self._count(0.5 * self.P * self.dt / self.tau_pair), len(others))
            for s in self.rng.choice(others, n_pairs, replace=False) if n_pairs else []:
                members.add(int(s))
                members.add(int(self.partner[s]))
            group = np.array(sorted(members), dtype=np.int64)
            self.rng.shuffle(group)
            self.partner[group[0::2]] = group[1::2]
            self.partner[group[1::2]] = group[0::2]
        if inflow_idx:
            idx = torch.from_numpy(np.array(inflow_idx, dtype=np.int64)).cuda()
            self.phi[:, idx] = torch.from_numpy(np.stack(inflow_comp, axis=1)).cuda()

    def step(self):
        """One time step dt: events, then n_sub mixing + reaction sub-steps."""
        torch = _torch()
        self._events()
        partner = torch.from_numpy(self.partner).cuda()
        w = 0.5 * (1.0 - math.exp(-2.0 * self.dt_sub / self.tau_mix))
        stream = torch.cuda.current_stream().cuda_stream
        M, n = self.mech, self.n
        for _ in range(self.n_sub):
            _lib.pyjac_mix_pairs(M.handle, n, n, self.phi.data_ptr(), partner.data_ptr(), w,
                                 self._work.data_ptr(), stream)
            self.phi, self._work = self._work, self.phi
            self._react(self.dt_sub)
        self.time += self.dt

    def _react(self, dt: float, max_tries: int = 60):
        """Reaction fractional step of length dt for every particle: implicit
        SDIRK3 steps with a per-particle step size.  A step is kept when it is
        finite, physical (mass fractions in [-1e-6, 1 + 1e-6], 200 K < T <
        6000 K, |dT| < 300 K) and its simplified Newton iterations converged
        (last increment <= 1e-4 of the step's change); otherwise the particle
        retries with a quarter of the step; after a kept step its step size
        doubles (up to dt).  A particle that exhausts the tries keeps the
        progress of its kept steps (counted in self.frozen).  The bookkeeping
        stays on the device; the host reads one count per try."""
        torch = _torch()
        n = self.n
        dev = self.phi.device
        t_rem = torch.full((n,), dt, dtype=torch.float64, device=dev)
        if not hasattr(self, "_hp"):
            self._hp = torch.full((n,), dt / self.react_steps, dtype=torch.float64, device=dev)
        h = torch.clamp(self._hp, max=dt)
        out = torch.empty_like(self.phi)
        for _ in range(max_tries):
            active = t_rem > 1e-9 * dt
            if not bool(active.any()):
                break
            hs = torch.where(active, torch.minimum(h, t_rem), torch.zeros_like(h))
            self._h.copy_(hs)
            _, dn = self.mech.sdirk3_step(self.phi, self.p, self._h, newton_iters=self.newton_iters,
                                          mode=NEWTON_FP64, out=out, workspace=self._ws)
            new, old = out, self.phi
            dmax = dn.max(dim=0).values
            Y = new[1:]
            change = (new - old).abs().max(dim=0).values
            ok = (torch.isfinite(new).all(dim=0) & torch.isfinite(dmax) & (dmax <= 1e-4 * change + 1e-12)
                  & (Y > -1e-6).all(dim=0) & (Y < 1 + 1e-6).all(dim=0) & (Y.sum(dim=0) < 1 + 1e-6)
                  & (new[0] > 200.0) & (new[0] < 6000.0) & ((new[0] - old[0]).abs() < 300.0))
            keep = active & ok
            self.phi = torch.where(keep[None, :], new, old)
            t_rem = torch.where(keep, t_rem - hs, t_rem)
            h = torch.where(keep, torch.clamp(2 * h, max=dt), torch.where(active, h / 4, h))
        stuck = t_rem > 1e-9 * dt
        self.frozen = getattr(self, "frozen", 0) + int(stuck.sum().item())
        self._hp = torch.clamp(h, min=1e-12)

    def run(self, n_res: float):
        """Advance n_res residence times."""
        steps = max(1, round(n_res * self.tau_res / self.dt))
        for _ in range(steps):
            self.step()
        return self.states()

    def states(self):
        """(phi [N, n], p [n]) of every particle, host copies."""
        _torch().cuda.synchronize()
        return self.phi.cpu().numpy(), self.p.cpu().numpy()


def burn(mech: Mechanism, comp, p_pa: float, t_end: float = 0.05, n_steps: int = 400, h0: float = 1e-8):
    """Constant-pressure adiabatic evolution of one composition toward
    equilibrium: implicit steps with geometrically growing size from h0 up to
    t_end (the pilot stream of the premixed PaSR, App. C).  It stops at the
    first step that gives a non-finite state and returns the state reached:
    for a start too stiff for h0 that is the input itself, which then burns
    inside the reactor under the particles' step control."""
    torch = _torch()
    phi = torch.from_numpy(np.asarray(comp, dtype=np.float64)[:, None].copy()).cuda()
    p = torch.full((1,), float(p_pa), dtype=torch.float64, device="cuda")
    ratio = (t_end / h0) ** (1.0 / n_steps)
    h = h0
    for _ in range(n_steps):
        hh = torch.full((1,), h, dtype=torch.float64, device="cuda")
        nxt, _ = mech.sdirk3_step(phi, p, hh, newton_iters=6, mode=NEWTON_FP64)
        if not bool(torch.isfinite(nxt).all()):
            break
        phi = nxt
        h *= ratio
    torch.cuda.synchronize()
    return phi[:, 0].cpu().numpy()
