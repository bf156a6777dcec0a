"""Problem description for the oracle: a finite-difference grid and a
material (Methods, "Physics and discretization": structured grid, x-fastest
indexing; per-cell materials): scalar parameters, each of Ms, A, alpha, Ku and
D optionally replaced by an array of one value per cell."""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class Grid:
    n: tuple                 # (nx, ny, nz) cells
    cell: tuple              # (dx, dy, dz) metres
    pbc: tuple = (0, 0, 0)   # 1 = periodic along that axis
    images: tuple = (0, 0, 0)  # periodic image count P per axis (sum p = -P..P)

    @property
    def volume(self) -> float:
        return self.cell[0] * self.cell[1] * self.cell[2]

    @property
    def ncells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def padded(self) -> tuple:
        """FFT size per axis: 2N on open axes with N > 1, N on periodic axes,
        1 when N = 1 (zero padding to 2N, Methods "Physics and discretization")."""
        out = []
        for a in range(3):
            N = self.n[a]
            if N == 1:
                out.append(1)
            elif self.pbc[a]:
                out.append(N)
            else:
                out.append(2 * N)
        return tuple(out)


@dataclass(frozen=True)
class Material:
    Ms: float = 8.0e5        # A/m
    A: float = 1.3e-11       # J/m
    alpha: float = 0.5
    Ku: float = 0.0          # J/m^3
    u: tuple = (0.0, 0.0, 1.0)
    D: float = 0.0           # J/m^2, interfacial
    B: tuple = (0.0, 0.0, 0.0)  # applied field, tesla
    T: float = 0.0           # kelvin
    demag: bool = True
    # Slonczewski spin-transfer torque: current density (A/m^2; a scalar or
    # one value per replica of a batch), fixed-layer direction, polarisation,
    # asymmetry Lambda and secondary (field-like) coefficient eps'
    stt_J: object = 0.0
    stt_p: tuple = (0.0, 0.0, 1.0)
    stt_P: float = 0.0
    stt_lambda: float = 1.0
    stt_eps2: float = 0.0
    # False: damping-only dynamics (the precession term of the LLG equation
    # dropped), the relaxation dynamics
    precess: bool = True
    # cubic anisotropy (J/m^3) along axes c1, c2, c3 = c1 x c2
    Kc1: float = 0.0
    Kc2: float = 0.0
    c1: tuple = (1.0, 0.0, 0.0)
    c2: tuple = (0.0, 1.0, 0.0)
    # bulk DMI (J/m^2)
    Db: float = 0.0
    # RKKY interlayer exchange: surface energy density (J/m^2) coupling
    # cell layers z0 and z1
    rkky: float = 0.0
    rkky_z: tuple = (0, 1)
    # per-cell exchange stiffness (array (nz, ny, nx), J/m) or None: replaces A
    # in the exchange term (harmonic mean per neighbour pair) and in the edge
    # conditions (the edge cell's value)
    A_cells: object = None
    # further per-cell parameters (arrays (nz, ny, nx)) or None: saturation
    # magnetisation (A/m, > 0), damping, uniaxial anisotropy constant (J/m^3)
    # and interfacial DMI constant (J/m^2); each replaces the scalar above
    Ms_cells: object = None
    alpha_cells: object = None
    Ku_cells: object = None
    D_cells: object = None

    @property
    def stt(self) -> bool:
        import numpy as np
        return self.stt_P != 0.0 and bool(np.any(np.asarray(self.stt_J) != 0.0))
