"""FP64 CPU oracle of the micromagnetic effective-field + LLG time step.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct
reference that the HIP library is checked against.  Only ``tests/``, the
``smoke()`` check of the repository entry module and the CPU-baseline leg of the
benchmark may import it; the library and its Python binding never do, and the
two share no code (only the seeded input generators in ``workloads``).

Every function cites the passage of the paper (Claude-SpinDynamics,
arxiv 2608.15253) or the published method it follows.  Where the paper is silent
the reading taken is stated in the docstring.  All arithmetic is float64; numpy's
FFT and linear algebra serve as library primitives.

Pins (``tests/test_oracle_*.py``, run with ``-m "not gpu"``) tie each part to
something other than itself: closed forms (cube self-term 1/3, trace identities,
point-dipole far field, whole-body identity, exact spin-wave dispersion, damped
macrospin, Kittel, Langevin, exact precession of the rotation scheme,
spin-transfer antidamping and precession of a free macrospin, J_c0), brute force (direct O(N^2) convolution, 50-digit
mpmath Newell values, a linear solve of the Gilbert-form spin-transfer torque) and invariants (|m| = 1, m . dm/dt = 0, energy decay).
The Philox generator is pinned by the known-answer vectors published with it
(Salmon et al. 2011).  Parity unpinned: the
interfacial-DMI edge ghosts against another code (closed forms pin the bulk
stencil only), long-horizon thermal trajectories (chaotic; statistical only),
and the behaviour of trained network weights (the network's arithmetic and the
learned-stage attempt are pinned; what training reaches is not).
"""
from .constants import GAMMA0, MU0, KB
from .problem import Grid, Material
from . import newell, demag, fields, llg, philox, integrators, observables, fno, surrogate
from . import rotation

__all__ = ["GAMMA0", "MU0", "KB", "Grid", "Material", "newell", "demag",
           "fields", "llg", "philox", "integrators", "observables", "fno", "surrogate",
           "rotation"]
