"""Exact enumeration of the rail-KMC chain on tiny lattices (R*L <= ~12 sites).

TEST INFRASTRUCTURE ONLY.  An independent second route to the same Markov
chain as kmc_oracle.c, used to pin the oracle: instead of the bond-window sum,
each hop's energy change is taken as E(after) - E(before) of the lattice energy

    E(x) = sum_s q V_app(s) x_s + 1/2 sum_{i != j} K_ij x_i x_j ,
    V_app(s) = alpha V (s + 1/2) / L      (grounded site-0 electrode, SI S1.3),

with K_ij the screened Coulomb kernel (main text section 3: the effective field
is the bias plus the Coulomb field of nearby ions), inclusive cutoff along the
rail, rails interacting up to `rail_range` (minimal image, periodic lateral
edges, SI S1.4).  The rate is the Arrhenius form (main text Eq. hop_rate) with
the barrier shifted by half the energy change (detailed balance at zero bias,
main text Eq. 2 and the paragraph after it), p = min(nu0 dt exp(-(Ea+dE/2)/kT), 1).

A step is the pair (bond) checkerboard: half-step h updates every bond
(s, s+1) with s = h mod 2 independently, all probabilities taken from the state
at the start of the half-step.  The transition matrix of a half-step is the
product of independent Bernoulli hops over its candidate bonds, so the
distribution after n steps is P_n = T1(V_n) T0(V_n) ... P_0, computed exactly in
binary64.

Open electrodes (optional): each rail's ends exchange ions with two
reservoirs, the grounded one behind site 0 (virtual site -1) and the biased
one behind site L-1 (virtual site L).  A reservoir ion has the energy
mu + q V_app(virtual site) and does not interact; a transfer is one more bond
of the checkerboard (s = -1 and s = L - 1), with the electrode's barrier and
dE = E_lattice(after) - E_lattice(before) -+ (mu + q V_app(virtual site)) on
injection / extraction.  The ion number is then free, and the state space is
every 0/1 configuration.
"""
from __future__ import annotations

import itertools
import math
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np


class Lattice:
    def __init__(self, R: int, L: int, ions_per_rail: Optional[Sequence[int]], physics,
                 ea_site: Optional[np.ndarray] = None, electrodes: Optional[Sequence[float]] = None):
        self.R, self.L = R, L
        self.ph = physics
        self.ea_site = None if ea_site is None else np.asarray(ea_site, dtype=np.float64).reshape(R, L)
        # (ea_ground, mu_ground, ea_bias, mu_bias) of open electrodes, or None
        self.electrodes = None if electrodes is None else tuple(float(x) for x in electrodes)
        self.K = self._pair_matrix()
        if self.electrodes is not None:  # every configuration
            self.states = [np.array(bits, dtype=np.int8).reshape(R, L)
                           for bits in itertools.product((0, 1), repeat=R * L)]
            self.index = {s.tobytes(): i for i, s in enumerate(self.states)}
            return
        if ions_per_rail is None:  # energy evaluation only, no state space
            self.states, self.index = [], {}
            return
        rails = []
        for r in range(R):
            opts = [tuple(1 if s in comb else 0 for s in range(L))
                    for comb in itertools.combinations(range(L), ions_per_rail[r])]
            rails.append(opts)
        self.states = [np.array(sum((list(x) for x in combo), []), dtype=np.int8).reshape(R, L)
                       for combo in itertools.product(*rails)]
        self.index = {s.tobytes(): i for i, s in enumerate(self.states)}

    # minimal-image distance between rails r and rp on a ring of R rails
    def rail_distance(self, r: int, rp: int) -> int:
        a = (rp - r) % self.R
        return min(a, self.R - a)

    def _pair_matrix(self) -> np.ndarray:
        ph = self.ph
        R, L = self.R, self.L
        n = R * L
        K = np.zeros((n, n))
        for i in range(n):
            ri, si = divmod(i, L)
            for j in range(n):
                if i == j:
                    continue
                rj, sj = divmod(j, L)
                dr = self.rail_distance(ri, rj)
                ds = si - sj
                if abs(ds) > ph.cutoff_sites or dr > ph.rail_range:
                    continue
                d = math.hypot(ds, dr)
                if ph.screening_sites > 0:
                    K[i, j] = ph.coulomb_kappa_v * math.exp(-d / ph.screening_sites) / d
                else:
                    K[i, j] = ph.coulomb_kappa_v / d
        return K

    def energy(self, x: np.ndarray, V: float) -> float:
        ph = self.ph
        v_app = ph.field_coupling * V * (np.arange(self.L) + 0.5) / self.L
        e_field = float((x * v_app[None, :]).sum())
        f = x.reshape(-1).astype(np.float64)
        return e_field + 0.5 * float(f @ self.K @ f)

    def barrier(self, r: int, o: int) -> float:
        return self.ph.ea_ev if self.ea_site is None else float(self.ea_site[r, o])

    def hop_probability(self, x: np.ndarray, r: int, o: int, t: int, V: float) -> Tuple[float, float]:
        """(p, dE) of the hop o -> t on rail r from state x."""
        y = x.copy()
        y[r, o], y[r, t] = 0, 1
        dE = self.energy(y, V) - self.energy(x, V)
        ph = self.ph
        p = ph.nu0_hz * ph.dt_s * math.exp(-(self.barrier(r, o) + 0.5 * dE) / ph.kT_ev)
        return min(p, 1.0), dE

    def reservoir_energy(self, side: int, V: float) -> float:
        """Energy of an ion in the reservoir of `side` (0 grounded, 1 biased)."""
        ph = self.ph
        virt = -1 if side == 0 else self.L
        mu = self.electrodes[1] if side == 0 else self.electrodes[3]
        return mu + ph.field_coupling * V * (virt + 0.5) / self.L

    def transfer_probability(self, x: np.ndarray, r: int, side: int, V: float) -> Tuple[float, float]:
        """(p, dE) of the transfer across the boundary bond of `side` of rail r."""
        site = 0 if side == 0 else self.L - 1
        inject = x[r, site] == 0
        y = x.copy()
        y[r, site] = 1 if inject else 0
        e_res = self.reservoir_energy(side, V)
        dE = self.energy(y, V) - self.energy(x, V) + (-e_res if inject else e_res)
        ph = self.ph
        ea = self.electrodes[0] if side == 0 else self.electrodes[2]
        p = ph.nu0_hz * ph.dt_s * math.exp(-(ea + 0.5 * dE) / ph.kT_ev)
        return min(p, 1.0), dE

    def candidates(self, x: np.ndarray, h: int) -> List[Tuple[int, int, int]]:
        """(rail, origin, target) of the candidate bonds of half-step h; a
        boundary bond has the virtual site -1 or L as origin or target."""
        out = []
        for r in range(self.R):
            for s in range(h, self.L - 1, 2):
                if x[r, s] != x[r, s + 1]:
                    o, t = (s, s + 1) if x[r, s] else (s + 1, s)
                    out.append((r, o, t))
            if self.electrodes is not None:
                if h == 1:  # bond (-1, 0)
                    out.append((r, 0, -1) if x[r, 0] else (r, -1, 0))
                if (self.L - 1) % 2 == h:  # bond (L-1, L)
                    out.append((r, self.L - 1, self.L) if x[r, self.L - 1] else (r, self.L, self.L - 1))
        return out

    def _probability(self, x, r, o, t, V) -> float:
        if o in (-1, self.L) or t in (-1, self.L):
            return self.transfer_probability(x, r, 0 if -1 in (o, t) else 1, V)[0]
        return self.hop_probability(x, r, o, t, V)[0]

    @staticmethod
    def _apply(y, r, o, t, L):
        if 0 <= o < L:
            y[r, o] = 0
        if 0 <= t < L:
            y[r, t] = 1

    def half_step_matrix(self, h: int, V: float) -> Tuple[np.ndarray, np.ndarray]:
        """T[x', x] of half-step h, and the expected signed hop count per state
        (toward site 0 counts +1, toward site L-1 counts -1)."""
        n = len(self.states)
        T = np.zeros((n, n))
        flow = np.zeros(n)
        for i, x in enumerate(self.states):
            cands = self.candidates(x, h)
            probs = [self._probability(x, r, o, t, V) for (r, o, t) in cands]
            for k, (r, o, t) in enumerate(cands):
                flow[i] += probs[k] * (1.0 if t < o else -1.0)
            for acc in itertools.product((0, 1), repeat=len(cands)):
                pr = 1.0
                y = x.copy()
                for a, pc, (r, o, t) in zip(acc, probs, cands):
                    if a:
                        pr *= pc
                        self._apply(y, r, o, t, self.L)
                    else:
                        pr *= 1.0 - pc
                if pr == 0.0:
                    continue
                T[self.index[y.tobytes()], i] += pr
        return T, flow

    def evolve(self, P0: np.ndarray, voltages: Sequence[float]) -> Dict[str, np.ndarray]:
        """Exact distribution after each step; voltages[n] = V(t_n)."""
        cache: Dict[float, Tuple] = {}
        P = P0.astype(np.float64).copy()
        dists, net = [], []
        for V in voltages:
            if V not in cache:
                cache[V] = (self.half_step_matrix(0, V), self.half_step_matrix(1, V))
            (T0, f0), (T1, f1) = cache[V]
            e_net = float(f0 @ P)
            P = T0 @ P
            e_net += float(f1 @ P)
            P = T1 @ P
            dists.append(P.copy())
            net.append(e_net)
        return {"P": np.array(dists), "net": np.array(net)}

    def grand_canonical(self, V: float) -> np.ndarray:
        """exp(-beta (E(x) - mu* N(x))) over every configuration, normalised,
        with mu* the grounded reservoir's energy: the equilibrium measure when
        both reservoirs have the same energy and every site the same barrier
        (the transfers' barriers are the electrodes' own)."""
        beta = 1.0 / self.ph.kT_ev
        mu = self.reservoir_energy(0, V)
        e = np.array([self.energy(x, V) - mu * float(x.sum()) for x in self.states])
        w = np.exp(-beta * (e - e.min()))
        return w / w.sum()

    def boltzmann(self, V: float) -> np.ndarray:
        beta = 1.0 / self.ph.kT_ev
        e = np.array([self.energy(x, V) for x in self.states])
        if self.ea_site is not None:
            e = e - np.array([float((x * self.ea_site).sum()) for x in self.states])
        w = np.exp(-beta * (e - e.min()))
        return w / w.sum()

    def state_of(self, occ: np.ndarray) -> int:
        return self.index[np.asarray(occ, dtype=np.int8).reshape(self.R, self.L).tobytes()]
