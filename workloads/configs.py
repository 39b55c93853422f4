"""Named synthetic workloads.

Each entry stands in for one of the paper's production lattices (whose gauge
ensembles are not available): the lattice shape, fifth-dimension extent,
Mobius parameters, link roughness ``eps``, subdomain tiling, inner iteration
count and precisions are fixed here together with the seeds, so that the
tests, the oracle and the benchmark draw identical inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field


@dataclass(frozen=True)
class Config:
    name: str
    dims: tuple            # (X, Y, Z, T)
    Ls: int
    b: float
    c: float
    M5: float
    mf: float
    eps: float             # link roughness, U = exp(i eps H)
    sub: tuple             # subdomain extents (X, Y, Z, T)
    inner_iters: int
    gauge_seed: int
    src_seed: int
    nrhs: int = 1
    outer_prec: str = "fp32"
    inner_prec: str = "fp16"
    tol: float = 1e-10
    note: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def volume(self) -> int:
        X, Y, Z, T = self.dims
        return X * Y * Z * T

    @property
    def n_subdomains(self) -> int:
        n = 1
        for d, s in zip(self.dims, self.sub):
            n *= d // s
        return n


CONFIGS = {
    # plain FP64 MSPCG on a small lattice; the oracle finishes it in seconds
    "c1": Config("c1", (8, 8, 8, 8), 8, 1.5, 0.5, 1.8, 0.1, 0.3, (4, 4, 4, 4), 5,
                 101, 201, outer_prec="fp64", inner_prec="fp64",
                 note="8^4 x Ls8 FP64 MSPCG, 16 subdomains of 4^4, k=5"),
    # single mixed-precision solve
    "c2": Config("c2", (16, 16, 16, 32), 12, 1.5, 0.5, 1.8, 0.01, 0.5, (4, 4, 4, 8), 6,
                 102, 202, note="16^3x32 x Ls12, FP32 outer + FP64 reliable updates, "
                                "FP16 inner on 256 subdomains of 4^3x8, k=6"),
    # batched multi-RHS on one gauge field
    "c3": Config("c3", (16, 16, 16, 16), 16, 1.5, 0.5, 1.8, 0.005, 0.5, (4, 4, 4, 4), 6,
                 103, 203, nrhs=12, note="16^4 x Ls16, 12 point-smeared sources"),
    # one GPU's share at production shape; k = 3 inner iterations, the
    # cheapest of the paper's values for this lattice (Table 1: k = 3, 4, 6)
    # and the fastest of them on one GPU, where an A_s application costs as
    # much as A and no halo exchange is saved (k = 3, 4, 5, 6: 16.2, 17.1,
    # 18.8, 20.6 s)
    "c4": Config("c4", (32, 32, 32, 64), 12, 1.5, 0.5, 1.8, 0.00078, 0.6, (8, 8, 8, 16), 3,
                 104, 204, note="32^3x64 x Ls12, FP32 outer + FP64 reliable updates, FP16 inner on "
                                "256 subdomains of 8^3x16, k=3"),
}
