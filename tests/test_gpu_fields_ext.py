"""GPU parity of the further field terms (Methods, "Physics and
discretization": bulk DMI, cubic anisotropy, RKKY interlayer exchange)
through the C ABI against the FP64 oracle: fields with every term on (open
3-D block: bulk-DMI ghosts on all axes; periodic film), energies per slot,
and Heun / RK45 steps with the terms on (the FP32 64 x 64 film leaves the
register row kernels for the field kernels).

Bars: fields FP64 1e-11 / FP32 4e-6 of max |H|; energies FP64 1e-12 / FP32
2e-6 of the largest term; states FP64 1e-12 / FP32 1e-5.
"""
import dataclasses

import numpy as np
import pytest

from oracle import fields as ofl
from oracle import integrators as oit
from oracle import observables as oob
from workloads import random_unit, replica_seeds, uniform

from _mmx_case import Case, dev, host, open_ctx

pytestmark = pytest.mark.gpu

EXT = dict(Kc1=4e4, Kc2=-2e4, c1=(0.8, 0.6, 0.0), c2=(-0.6, 0.8, 0.1), Db=1.5e-3)


def _setup(ctx, case, rkky=0.0, rkky_z=(0, 1), ext=EXT):
    import paper_2608_15253_amd as mmx
    mmx.mmx_set_material_ext(ctx, 0, rkky=rkky, rkky_z=rkky_z, **ext)
    mmx.mmx_set_terms(ctx, case.mask() | mmx.MMX_DMI_BULK | mmx.MMX_ANIS_CUBIC | mmx.MMX_RKKY)


def _mat(case, rkky=0.0, rkky_z=(0, 1), ext=EXT):
    return dataclasses.replace(case.material(), rkky=rkky, rkky_z=tuple(rkky_z), **ext)


def _round(m, prec):
    return m.astype(np.float32).astype(np.float64) if prec == 1 else m


CASES = {
    "block-open": (Case((12, 10, 4), (3e-9, 2.5e-9, 2e-9), R=2, Ms=6e5, A=1.2e-11, D=2e-3,
                        Ku=3e5, u=(0.1, 0.2, 0.97), B=(0.01, -0.02, 0.05)), 2e-4, (1, 3)),
    "film-periodic": (Case((16, 12, 1), (2e-9, 2e-9, 1e-9), pbc=(1, 1, 0), images=(1, 1, 0),
                           R=2, Ms=6e5, A=1.2e-11, D=2e-3, Ku=3e5, B=(0.0, 0.0, 0.05)),
                      0.0, (0, 1)),
}


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("name", list(CASES))
def test_fields_and_energies_with_further_terms(name, prec):
    import paper_2608_15253_amd as mmx
    case, rkky, rz = CASES[name]
    m0 = _round(random_unit(case.n, seed=51, replicas=case.R), prec)
    ctx = open_ctx(case, prec)
    try:
        _setup(ctx, case, rkky, rz)
        H = dev(np.zeros_like(m0), prec)
        mmx.mmx_field(ctx, dev(m0, prec), H)
        E = dev(np.zeros((case.R, 6)), 2)
        mmx.mmx_energy(ctx, dev(m0, prec), E)
        got, gE = host(H), host(E)
    finally:
        mmx.mmx_destroy(ctx)
    mat = _mat(case, rkky, rz)
    for r in range(case.R):
        ref = ofl.effective_field(m0[r], case.grid, mat)
        err = np.abs(got[r] - ref).max() / np.abs(ref).max()
        assert err <= (1e-11 if prec == 2 else 4e-6), err
        e = oob.energies(m0[r], case.grid, mat)
        slots = [e["exchange"] + e["rkky"], e["dmi"] + e["dmi_bulk"], e["demag"],
                 e["anisotropy"] + e["cubic"], e["zeeman"], e["total"]]
        scale = max(abs(x) for x in slots[:5])
        assert np.abs(gE[r] - np.array(slots)).max() <= (1e-12 if prec == 2 else 2e-6) * scale
    if rkky:
        parts = ofl.terms(m0[0], case.grid, mat)
        assert np.abs(parts["rkky"]).max() > 1e-3 * np.abs(parts["exchange"]).max()


@pytest.mark.parametrize("prec,n", [(2, (20, 12, 1)), (1, (64, 64, 1))], ids=["f64", "f32-64x64"])
def test_heun_with_further_terms(prec, n):
    import paper_2608_15253_amd as mmx
    R = 2
    case = Case(n, (4e-9, 4e-9, 2e-9), R=R, alpha=0.1, Ku=2e5, A=1.3e-11, B=(0, 0, -0.05), T=300.0,
                seeds=list(replica_seeds(52, R)),
                terms=("exchange", "anisotropy", "zeeman", "demag", "thermal"))
    m0 = _round(uniform(case.n, (0.2, 0.1, 1.0), replicas=R), prec)
    ctx = open_ctx(case, prec)
    try:
        _setup(ctx, case)
        md = dev(m0, prec)
        mmx.mmx_heun(ctx, md, 1e-14, 15, 3)
        got = host(md)
    finally:
        mmx.mmx_destroy(ctx)
    ref = oit.heun_run(m0, case.grid, _mat(case), 1e-14, 15, seed=np.array(case.seeds), step0=3)
    err = np.abs(got - ref).max()
    print(f"[case] heun ext {n} prec={prec}: max |dm| {err:.2e}")
    assert err <= (1e-12 if prec == 2 else 1e-5), err


def test_rk45_block_with_rkky_fp64():
    import paper_2608_15253_amd as mmx
    case = Case((10, 8, 4), (3e-9, 3e-9, 2e-9), R=1, alpha=0.3, Ku=1e5, A=1.3e-11,
                terms=("exchange", "anisotropy", "demag"))
    m0 = random_unit(case.n, seed=53, replicas=1)
    t_end, tol = 5e-12, 1e-6
    ctx = open_ctx(case, 2)
    try:
        _setup(ctx, case, rkky=-3e-4, rkky_z=(0, 3))
        md = dev(m0, 2)
        st = mmx.mmx_rk45(ctx, md, 0.0, t_end, tol, 1e-14)
        got = host(md)
        dts = mmx.mmx_rk45_dts(ctx)
    finally:
        mmx.mmx_destroy(ctx)
    rep = oit.rk45_run(m0[0], case.grid, _mat(case, -3e-4, (0, 3)), 0.0, t_end, tol, dt_replay=dts)
    assert st.t == t_end
    assert np.abs(got[0] - rep.m).max() <= 1e-12


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_per_cell_exchange_fields_and_steps(prec):
    """Per-cell stiffness (two regions and a zero-stiffness cell) with
    interfacial and bulk DMI edges: fields, energies and Heun steps."""
    import paper_2608_15253_amd as mmx
    R = 2
    case = Case((12, 10, 3), (3e-9, 3e-9, 2e-9), R=R, Ms=6e5, A=1.3e-11, D=1.5e-3, alpha=0.2,
                Ku=2e5, B=(0, 0, 0.05), T=200.0, seeds=list(replica_seeds(54, R)),
                terms=("exchange", "dmi", "anisotropy", "zeeman", "demag", "thermal"))
    Ac = np.full((3, 10, 12), 1.3e-11)
    Ac[:, :, 6:] = 0.4e-11
    Ac[1, 4, 3] = 0.0
    ext = dict(EXT, Kc1=0.0, Kc2=0.0)
    m0 = _round(random_unit(case.n, seed=55, replicas=R), prec)
    ctx = open_ctx(case, prec)
    try:
        _setup(ctx, case, ext=ext)
        mmx.mmx_set_exchange_cells(ctx, 0, Ac)
        full = case.mask() | mmx.MMX_DMI_BULK | mmx.MMX_ANIS_CUBIC | mmx.MMX_RKKY
        mmx.mmx_set_terms(ctx, full & ~mmx.MMX_THERMAL)  # fields without the noise
        H = dev(np.zeros_like(m0), prec)
        mmx.mmx_field(ctx, dev(m0, prec), H)
        E = dev(np.zeros((R, 6)), 2)
        mmx.mmx_energy(ctx, dev(m0, prec), E)
        mmx.mmx_set_terms(ctx, full)
        md = dev(m0, prec)
        mmx.mmx_heun(ctx, md, 1e-14, 10, 0)
        got, gE, gm = host(H), host(E), host(md)
    finally:
        mmx.mmx_destroy(ctx)
    mat = dataclasses.replace(_mat(case, ext=ext), A_cells=Ac)
    nothermal = dataclasses.replace(mat, T=0.0)
    for r in range(R):
        ref = ofl.effective_field(m0[r], case.grid, nothermal)
        assert np.abs(got[r] - ref).max() <= (1e-11 if prec == 2 else 4e-6) * np.abs(ref).max()
        e = oob.energies(m0[r], case.grid, nothermal)
        assert abs(gE[r][0] - (e["exchange"] + e["rkky"])) <= \
            (1e-12 if prec == 2 else 2e-6) * max(abs(v) for v in e.values())
    ref_m = oit.heun_run(m0, case.grid, mat, 1e-14, 10, seed=np.array(case.seeds))
    assert np.abs(gm - ref_m).max() <= (1e-12 if prec == 2 else 1e-5)
