"""Seeded synthetic inputs shared by the HIP path, the oracle and the bench.

This module holds no arithmetic of the method itself: it only draws
initial chain configurations and states the flow fields and sizes of the
workloads.  Random numbers the method itself draws (the Brownian noise) are
generated on each side from the Philox4x64-10 definition, not here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def random_walk(n_beads: int, b: float = 1.0, seed: int = 0, chain: int = 0) -> np.ndarray:
    """A freely-jointed random walk of unit-length bonds scaled by b, r_0 = 0.

    Bond directions are uniform on the sphere (z uniform in [-1, 1], azimuth
    uniform in [0, 2 pi)), drawn from numpy's PCG64 seeded with (seed, chain).
    Returns an (n_beads, 3) float64 array, row-major (bead-major).
    """
    rng = np.random.default_rng([int(seed), int(chain), 0x5EED])
    m = n_beads - 1
    z = rng.uniform(-1.0, 1.0, size=m)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=m)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    u = np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)
    x = np.zeros((n_beads, 3))
    x[1:] = b * np.cumsum(u, axis=0)
    return x


def straight_chain(n_beads: int, b: float = 1.0, axis: int = 0) -> np.ndarray:
    x = np.zeros((n_beads, 3))
    x[:, axis] = b * np.arange(n_beads)
    return x


def relaxation_time(n_beads: int) -> float:
    """Rouse end-to-end relaxation time (N-1)^2 b^2 zeta / (3 pi^2 kT) in
    units zeta = kT = b = 1; used only to turn a Weissenberg number into a
    strain rate."""
    return (n_beads - 1) ** 2 / (3.0 * math.pi ** 2)


def kappa_for(flow: str, rate: float) -> np.ndarray:
    """Row-major 3x3 kappa = (grad v)^T with v = kappa . r."""
    k = np.zeros((3, 3))
    if flow == "none":
        pass
    elif flow == "uniaxial":
        k[0, 0], k[1, 1], k[2, 2] = rate, -0.5 * rate, -0.5 * rate
    elif flow == "planar":
        k[0, 0], k[1, 1] = rate, -rate
    elif flow == "shear":
        k[0, 1] = rate
    else:
        raise ValueError(flow)
    return k


@dataclass(frozen=True)
class Workload:
    name: str
    n_beads: int
    dt: float
    steps: int
    flow: str = "none"
    wi: float = 0.0
    seed: int = 0
    b: float = 1.0
    hstar: float = 0.25
    a: float = 0.5
    chains: int = 1
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return 3 * self.n_beads

    @property
    def rate(self) -> float:
        return 0.0 if self.flow == "none" else self.wi / relaxation_time(self.n_beads)

    @property
    def kappa(self) -> np.ndarray:
        return kappa_for(self.flow, self.rate)

    def initial(self, chain: int = 0) -> np.ndarray:
        return random_walk(self.n_beads, self.b, self.seed, chain)


# The paper's workload family: one chain of unit Kuhn-step rods with RPY HI
# (h* = 0.25, bead radius a = b/2), seeded random-walk start.
SINGLE_SMALL = Workload("single-chain N=32 no flow", 32, 1e-4, 100, "none", 0.0, seed=0)
SINGLE_PLANAR = Workload("single-chain N=512 planar Wi=1", 512, 1e-4, 1000, "planar", 1.0, seed=1)
ENSEMBLE_SHEAR = Workload("ensemble 256 chains N in [64,1024] shear Wi=10", 64, 1e-4, 500, "shear",
                          10.0, seed=3, chains=256)
LONG_UNIAXIAL = Workload("single-chain N=4096 uniaxial Wi=5", 4096, 5e-5, 200, "uniaxial", 5.0, seed=4)
GRAD_PLANAR = Workload("64 chains N=256 planar", 256, 1e-4, 200, "planar", 1.0, seed=5, chains=64)



def ensemble_sizes(count: int, lo: int = 64, hi: int = 1024, seed: int = 3) -> np.ndarray:
    """Bead counts of an ensemble with uneven chains: N_c = lo + floor((hi -
    lo + 1) u_c), u_c uniform on [0, 1) from numpy's PCG64 seeded with
    (seed, 0xC3)."""
    rng = np.random.default_rng([int(seed), 0xC3])
    u = rng.random(count)
    return (lo + np.floor((hi - lo + 1) * u)).astype(np.int64)


def ensemble_chains(w: "Workload", sizes) -> list[dict]:
    """The chains of an ensemble workload with the given bead counts: chain
    c has N_c beads, the workload's flow at Weissenberg number wi with its
    own rate wi / lambda(N_c), a random-walk start drawn with (seed, c), and
    Philox key (seed, c)."""
    out = []
    for c, nb in enumerate(int(v) for v in sizes):
        rate = 0.0 if w.flow == "none" else w.wi / relaxation_time(nb)
        out.append(dict(n_beads=nb, kappa=kappa_for(w.flow, rate), seed=w.seed, chain_id=c,
                        x=random_walk(nb, w.b, w.seed, c)))
    return out


WORKLOADS = {w.name: w for w in (SINGLE_SMALL, SINGLE_PLANAR, ENSEMBLE_SHEAR, LONG_UNIAXIAL, GRAD_PLANAR)}
