"""Seeded synthetic carbon clusters (the stand-in for the paper's fullerenes).

The paper times its method on AM1 fullerenes up to C840 (Results, fullerene
test set) whose coordinates and parameters are not available here.  These
clusters reproduce the shapes that matter for the electronic hot path: four
orbitals (s, px, py, pz) and four valence electrons per carbon, dense
all-pairs two-centre blocks (NDDO has no cutoff, Methods section 1), and a
symmetric n x n Fock matrix with n = 4 * N_atoms.

Draw order from ``numpy.random.default_rng(seed)`` (PCG64):
  1. positions by random sequential addition in a cube of side
     (N / density)^(1/3), rejecting any draw closer than ``r_min`` to an
     atom already placed (open boundaries);
  2. one set of five one-centre integrals for carbon, uniform in [5, 15] eV,
     in the order Gss, Gsp, Gpp, Gp2, Hsp (broadcast to every atom);
  3. per unordered atom pair (A < B, row-major over A then B) 55 noise values,
     the packed upper triangle of a symmetric 10 x 10 block, drawn as float32
     uniforms in [0, 1) and mapped to 2u - 1 in float32, so every value is
     exactly representable in single precision;
  4. Maxwell-Boltzmann velocities at 300 K with the centre-of-mass velocity
     removed.

Nothing here evaluates the model: the parameters in ``ModelParams`` are
handed to the oracle and to the HIP path as inputs.
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

# Physical constants used only to draw thermal velocities.
_KB_EV_PER_K = 8.617333262e-5          # Boltzmann constant, eV/K (CODATA 2018)
_EV_PER_AMU_TO_A2_PER_FS2 = 9.648533e-3  # 1 eV/amu expressed in (Angstrom/fs)^2


@dataclass(frozen=True)
class ModelParams:
    """Constants of the synthetic sp Hamiltonian (eV, Angstrom, amu).

    On-site energies eps_s / eps_p; hopping t(R) = t0 * exp(-(R - r0_hop) /
    lam_hop) times direction cosines; two-centre blocks coul_k /
    sqrt(R^2 + coul_a^2) * (J + noise_amp * noise); core charge z_core for the
    core-electron attraction and core-core Coulomb terms; short-range
    repulsion a_rep * exp(-(R - r0_rep) / rho_rep).
    """

    eps_s: float = -20.0
    eps_p: float = -10.0
    t0: float = -8.0
    r0_hop: float = 1.4
    lam_hop: float = 0.5
    coul_k: float = 14.4
    coul_a: float = 1.5
    noise_amp: float = 0.1
    z_core: float = 4.0
    a_rep: float = 8.0
    r0_rep: float = 1.4
    rho_rep: float = 0.25
    mass: float = 12.011
    j_pattern: str = "monopole"

    def j55(self) -> np.ndarray:
        """Packed (upper-triangle, row-major) 10 x 10 pattern J of the two-centre
        blocks.  "allones": every entry 1.  "monopole": 1 where both packed
        pairs are on-site densities (mu mu) and (lambda lambda), else 0 -- the
        point-charge limit of NDDO two-centre integrals."""
        diag = np.array([1.0 if a == b else 0.0 for a in range(4) for b in range(a, 4)])
        if self.j_pattern == "allones":
            full = np.ones((10, 10))
        elif self.j_pattern == "monopole":
            full = np.outer(diag, diag)
        else:
            raise ValueError(f"unknown j_pattern {self.j_pattern!r}")
        return full[np.triu_indices(10)].copy()

    def as_array(self) -> np.ndarray:
        """Parameters in the fixed order the C ABI's parameter block uses."""
        return np.array([self.eps_s, self.eps_p, self.t0, self.r0_hop, self.lam_hop,
                         self.coul_k, self.coul_a, self.noise_amp, self.z_core,
                         self.a_rep, self.r0_rep, self.rho_rep, self.mass],
                        dtype=np.float64)


@dataclass(frozen=True)
class OverlapModel:
    """Constants of the synthetic overlap of a non-orthogonal basis: the radial
    factor s(R) = s0 * exp(-(R - r0) / lam) of the off-site blocks (Angstrom).
    At these values the overlap of the seeded clusters has eigenvalues in
    about [0.74, 1.38]."""

    s0: float = 0.08
    r0: float = 1.4
    lam: float = 0.4


@dataclass
class System:
    """One synthetic cluster: everything both sides need as input."""

    n_atoms: int
    seed: int
    R: np.ndarray            # (N, 3) float64, Angstrom
    onecenter: np.ndarray    # (N, 5) float64, eV: Gss, Gsp, Gpp, Gp2, Hsp
    noise: np.ndarray        # (N_pair, 55) float32, packed symmetric 10x10 per pair
    V: np.ndarray            # (N, 3) float64, Angstrom/fs
    params: ModelParams = field(default_factory=ModelParams)

    @property
    def n_orb(self) -> int:
        return 4 * self.n_atoms

    @property
    def n_pair(self) -> int:
        return self.n_atoms * (self.n_atoms - 1) // 2

    @property
    def n_elec(self) -> float:
        return float(4 * self.n_atoms)


def _positions(rng, n_atoms, density, r_min):
    side = (n_atoms / density) ** (1.0 / 3.0)
    pos = np.empty((n_atoms, 3), dtype=np.float64)
    placed = 0
    r2 = r_min * r_min
    while placed < n_atoms:
        c = rng.uniform(0.0, side, size=3)
        if placed == 0 or np.min(np.sum((pos[:placed] - c) ** 2, axis=1)) >= r2:
            pos[placed] = c
            placed += 1
    return pos


def carbon_cluster(n_atoms: int, seed: int, *, density: float = 0.11, r_min: float = 1.3,
                   temp_K: float = 300.0, params: ModelParams | None = None) -> System:
    """Draw one cluster (see the module docstring for the recipe)."""
    if n_atoms < 1:
        raise ValueError("n_atoms must be >= 1")
    params = params or ModelParams()
    rng = np.random.default_rng(seed)
    R = _positions(rng, n_atoms, density, r_min)
    oc = rng.uniform(5.0, 15.0, size=5)
    onecenter = np.tile(oc, (n_atoms, 1))
    n_pair = n_atoms * (n_atoms - 1) // 2
    u = rng.random((n_pair, 55), dtype=np.float32)
    noise = (np.float32(2.0) * u - np.float32(1.0)).astype(np.float32)
    sigma = np.sqrt(_KB_EV_PER_K * temp_K / params.mass * _EV_PER_AMU_TO_A2_PER_FS2)
    V = rng.standard_normal((n_atoms, 3)) * sigma
    if n_atoms > 1:
        V -= V.mean(axis=0, keepdims=True)
    return System(n_atoms=n_atoms, seed=seed, R=R, onecenter=onecenter, noise=noise, V=V,
                  params=params)


def ensemble_sizes(n_traj: int = 64, lo: int = 20, hi: int = 300, seed: int = 4) -> np.ndarray:
    """Atom counts of the ragged ensemble: integers uniform in [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=n_traj)


# The five workloads.  T_e in K, dt in fs.  Low-gap: hopping x0.6, s-p split 4 eV.
WORKLOADS = {
    "c10": dict(n_atoms=10, seed=1, T_e=3000.0, m=3, dt=0.5, steps=10, params=ModelParams()),
    "c100": dict(n_atoms=100, seed=2, T_e=5000.0, m=4, dt=0.5, steps=100, params=ModelParams()),
    "c840": dict(n_atoms=840, seed=3, T_e=5000.0, m=6, dt=0.5, steps=20, params=ModelParams()),
    "c840_lowgap": dict(n_atoms=840, seed=5, T_e=10000.0, m=8, dt=0.5, steps=200,
                        params=replace(ModelParams(), t0=-4.8, eps_s=-14.0)),
}


def workload(name: str) -> tuple[System, dict]:
    """Return (system, settings) for a named single-system workload."""
    w = dict(WORKLOADS[name])
    params = w.pop("params")
    sys_ = carbon_cluster(w["n_atoms"], w["seed"], params=params)
    return sys_, w
