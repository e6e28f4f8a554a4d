"""Seeded sum-of-products vibrational Hamiltonians (inputs only).

A model is stored in the sum-of-products form of the paper (Sec. II.A.3,
Eq. sum_of_tp): harmonic on-site terms plus monomials in the dimensionless
normal coordinates,

    H = sum_i omega_i/2 (p_i^2 + q_i^2) + sum_m f_m prod_{i in m} q_i^{k_i},

with each monomial stored once (its coefficient already folds in the 1/6 or
1/24 of the Taylor expansion and the permutation multiplicity).  Units are
cm^-1.  Only coefficients and index sets are drawn here; the per-mode operator
matrices are built independently by each consumer.

Draw order (numpy PCG64, ``default_rng(seed)``): omega (L draws), then the
pair couplings in lexicographic (i<j) order, then cubic terms, then quartic.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import List, Tuple

import numpy as np

Monomial = Tuple[Tuple[int, int], ...]  # ((mode, power), ...) sorted by mode


@dataclasses.dataclass
class SOPModel:
    """Hamiltonian H = sum_i omega_i (n_i + 1/2) + sum_m coef_m * prod q^k.

    ``dims[i]`` is the harmonic-oscillator basis size of mode i.
    ``monomials[m]`` is a tuple of (mode, power) pairs, modes strictly
    increasing; ``coefs[m]`` its coefficient in cm^-1.
    """

    name: str
    omega: np.ndarray
    dims: List[int]
    monomials: List[Monomial]
    coefs: np.ndarray
    seed: int = 0

    @property
    def n_modes(self) -> int:
        return len(self.omega)

    @property
    def zpe_harmonic(self) -> float:
        return float(0.5 * np.sum(self.omega))

    @property
    def n_terms(self) -> int:
        return self.n_modes + len(self.monomials)

    def to_json(self) -> dict:
        return {
            "name": self.name,
            "seed": self.seed,
            "omega": [float(x) for x in self.omega],
            "dims": [int(d) for d in self.dims],
            "monomials": [[[int(a), int(b)] for a, b in m] for m in self.monomials],
            "coefs": [float(c) for c in self.coefs],
        }

    @staticmethod
    def from_json(d: dict) -> "SOPModel":
        return SOPModel(
            name=d["name"],
            omega=np.asarray(d["omega"], dtype=np.float64),
            dims=[int(x) for x in d["dims"]],
            monomials=[tuple((int(a), int(b)) for a, b in m) for m in d["monomials"]],
            coefs=np.asarray(d["coefs"], dtype=np.float64),
            seed=int(d.get("seed", 0)),
        )


def _mono(modes) -> Monomial:
    """Multiset of modes -> sorted ((mode, power), ...)."""
    cnt = {}
    for i in modes:
        cnt[i] = cnt.get(i, 0) + 1
    return tuple(sorted(cnt.items()))


def coupled_oscillators(L: int, seed: int, wmin: float, wmax: float, d: int,
                        n_cubic: int = 0, cubic_max: float = 5.0,
                        coupling_scale: float = 0.02, name: str = "") -> SOPModel:
    """Quadratically coupled oscillators with optional random cubic terms.

    omega_i ~ U(wmin, wmax); c_ij ~ N(0, (s*sqrt(omega_i omega_j))^2) for
    every pair i<j, each pair entering the Hamiltonian once (the paper's
    bilinear coupling, Eq. coupled_harmonic_oscillator, sums each pair once);
    ``n_cubic`` distinct triples i<j<k with k_ijk = +-U(0, cubic_max).
    """
    rng = np.random.default_rng(seed)
    omega = rng.uniform(wmin, wmax, size=L)
    monos: List[Monomial] = []
    coefs: List[float] = []
    for i, j in itertools.combinations(range(L), 2):
        c = rng.normal(0.0, coupling_scale * math.sqrt(omega[i] * omega[j]))
        monos.append(_mono((i, j)))
        coefs.append(c)
    if n_cubic:
        n_tri = math.comb(L, 3)
        picks = rng.choice(n_tri, size=min(n_cubic, n_tri), replace=False)
        all_tri = list(itertools.combinations(range(L), 3))
        for t in sorted(int(p) for p in picks):
            mag = rng.uniform(0.0, cubic_max)
            sign = 1.0 if rng.random() < 0.5 else -1.0
            monos.append(_mono(all_tri[t]))
            coefs.append(sign * mag)
    return SOPModel(name or f"coupled_L{L}_s{seed}", omega, [d] * L, monos,
                    np.asarray(coefs, dtype=np.float64), seed)


def _hermite_range(d: int) -> float:
    """Largest Gauss-Hermite node of order d: the extent of the basis in q."""
    x, _ = np.polynomial.hermite.hermgauss(d)
    return float(np.max(np.abs(x)))


def _cuts_monotone(omega, dims, monos, coefs) -> bool:
    """Every 1-D cut V_i(q) (other coordinates zero) increases in |q| over the
    basis range of mode i.  An input-acceptance test for the random draw."""
    for i in range(len(omega)):
        poly = np.zeros(5)
        poly[2] = 0.5 * omega[i]
        for m, c in zip(monos, coefs):
            if len(m) == 1 and m[0][0] == i:
                poly[m[0][1]] += c
        qmax = _hermite_range(dims[i])
        q = np.linspace(0.0, qmax, 400)
        for s in (1.0, -1.0):
            v = np.polyval(poly[::-1], s * q)
            if np.any(np.diff(v) <= 0.0):
                return False
    return True


def quartic_force_field(L: int, seed: int, n_cubic: int, n_quartic: int,
                        wmin: float = 360.0, wmax: float = 3100.0,
                        fcubic: float = 50.0, fquartic: float = 10.0,
                        name: str = "") -> SOPModel:
    """Acetonitrile-sized synthetic quartic force field.

    omega ~ U(wmin, wmax) sorted descending; basis size per mode
    d_i = clip(round(6 + 8 (wmax - omega_i)/(wmax - wmin)), 6, 14) (softer
    modes get larger bases).  Cubic and quartic monomials are drawn without
    replacement from all multisets of modes; each coefficient is
    +-U(0, F) * prod_{i in m} sqrt(omega_i/omega_max), with q_i^4 forced
    positive.  The draw is accepted only if every 1-D cut of the potential is
    monotone in |q| over the basis range; otherwise seed+1000 is tried (the
    accepted seed is recorded in the model).
    """
    s = seed
    for _ in range(50):
        rng = np.random.default_rng(s)
        omega = np.sort(rng.uniform(wmin, wmax, size=L))[::-1].copy()
        dims = [int(np.clip(round(6 + 8 * (wmax - w) / (wmax - wmin)), 6, 14)) for w in omega]
        cub = list(itertools.combinations_with_replacement(range(L), 3))
        qua = list(itertools.combinations_with_replacement(range(L), 4))
        wmx = float(np.max(omega))
        monos: List[Monomial] = []
        coefs: List[float] = []
        for pool, nsel, F in ((cub, n_cubic, fcubic), (qua, n_quartic, fquartic)):
            picks = sorted(int(p) for p in rng.choice(len(pool), size=min(nsel, len(pool)), replace=False))
            for p in picks:
                modes = pool[p]
                mag = rng.uniform(0.0, F) * math.prod(math.sqrt(omega[i] / wmx) for i in modes)
                sign = 1.0 if rng.random() < 0.5 else -1.0
                m = _mono(modes)
                if len(m) == 1 and m[0][1] == 4:
                    sign = 1.0
                monos.append(m)
                coefs.append(sign * mag)
        if _cuts_monotone(omega, dims, monos, coefs):
            return SOPModel(name or f"qff_L{L}_s{s}", omega, dims, monos,
                            np.asarray(coefs, dtype=np.float64), s)
        s += 1000
    raise RuntimeError("no acceptable quartic force field draw")


def paper_64d_model(d: int = 8, L: int = 64, alpha: float = 0.1) -> SOPModel:
    """The paper's bilinearly coupled oscillators: omega_j = sqrt(j/2),
    alpha_ij = 0.1 for every pair (Sec. III.A, Eq. coupled_harmonic_oscillator)."""
    omega = np.sqrt(np.arange(1, L + 1) / 2.0)
    monos = [_mono((i, j)) for i, j in itertools.combinations(range(L), 2)]
    coefs = np.full(len(monos), alpha)
    return SOPModel(f"paper64d_L{L}", omega, [d] * L, monos, coefs, 0)


def make_config_model(config: str, seed: int | None = None, L: int | None = None) -> SOPModel:
    """The named synthetic workloads.

    c1: 6 modes, omega ~ U(500,3000), quadratic couplings, d=6 (seed 1).
    c2: 64 modes, omega ~ U(1000,3000), all-pairs quadratic + 200 cubic, d=8 (seed 2).
    c2q: c2 without the cubic terms.
    c3: 12-mode quartic force field, 108 cubic + 191 quartic terms (seed 3).
    c4-binary / c4-fork: ensemble members with L modes (seeded).
    """
    if config == "c1":
        return coupled_oscillators(6, 1 if seed is None else seed, 500.0, 3000.0, 6, name="c1")
    if config == "c2":
        return coupled_oscillators(64, 2 if seed is None else seed, 1000.0, 3000.0, 8, n_cubic=200, name="c2")
    if config == "c2q":
        return coupled_oscillators(64, 2 if seed is None else seed, 1000.0, 3000.0, 8, n_cubic=0, name="c2q")
    if config == "c3":
        return quartic_force_field(12, 3 if seed is None else seed, 108, 191, name="c3")
    if config == "c4-binary":
        assert L is not None and seed is not None
        return coupled_oscillators(L, seed, 1000.0, 3000.0, 8, n_cubic=round(200 * L / 64),
                                   name=f"c4b_L{L}_s{seed}")
    if config == "c4-fork":
        assert L is not None and seed is not None
        return quartic_force_field(L, seed, 9 * L, 16 * L, name=f"c4f_L{L}_s{seed}")
    raise ValueError(config)


def ensemble_members(n: int, seed0: int = 4000, D_range=(12, 48), k_range=(10, 84), L_range=(8, 64)):
    """Seeded ensemble of independent workloads: member i uses seed seed0 + i;
    even seeds take the coupled-oscillator generator on a balanced binary
    tree, odd seeds the quartic force-field generator on a fork-4 comb; the
    mode count L, bond dimension D and block size k are drawn uniformly
    (integers, inclusive ranges) from the member's own seed."""
    out = []
    for i in range(n):
        seed = seed0 + i
        rng = np.random.default_rng(seed)
        L = int(rng.integers(L_range[0], L_range[1] + 1))
        D = int(rng.integers(D_range[0], D_range[1] + 1))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        kind = "c4-binary" if seed % 2 == 0 else "c4-fork"
        out.append({"seed": seed, "kind": kind, "L": L, "D": D, "k": k,
                    "model": make_config_model(kind, seed=seed, L=L)})
    return out
