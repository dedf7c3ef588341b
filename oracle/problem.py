"""Problem description shared by the oracle's variants.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Parameters follow the paper's problem statement (Sections 2.1-2.2, eq. BLEnergy)
and parameter configuration (Section 4.3: sigma^2 = 1, alpha = 0.0025, s = 2).
The velocity is stationary: a single band-limited field v~ [d, K_1..K_d] used at
every time node; time [0, 1] is split into Nt steps of length dt = 1/Nt.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Tuple

import torch


@dataclass(frozen=True)
class Problem:
    N: Tuple[int, ...]
    K: Tuple[int, ...]
    Nt: int = 10
    alpha: float = 0.0025
    s: int = 2
    sigma2: float = 1.0

    @property
    def d(self) -> int:
        return len(self.N)

    @property
    def dt(self) -> float:
        return 1.0 / self.Nt

    def trapezoid_weights(self):
        """Weights of the trapezoid rule over the Nt+1 time nodes (stationary time integral)."""
        w = [self.dt] * (self.Nt + 1)
        w[0] = w[-1] = 0.5 * self.dt
        return w


def velocity_grid_units(vgrid: torch.Tensor, N) -> torch.Tensor:
    """Velocity samples in unit-torus units -> grid units (multiply component j by N_j)."""
    scale = torch.tensor([float(n) for n in N], dtype=vgrid.dtype).reshape((-1,) + (1,) * len(N))
    return vgrid * scale
