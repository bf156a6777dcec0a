"""GPU parity of per-cell materials (mmx_set_material_cells; Methods,
"Physics and discretization": material parameters per cell) through the C ABI
against the FP64 oracle: the effective field and energies with Ms, A, alpha,
Ku and D varying from cell to cell (open 3-D block with its DMI edge ghosts,
periodic film), torque, Heun with the Brown field, the rotation scheme and
RK45 in dt replay; uniform per-cell arrays reproduce the uniform material;
invalid arrays are rejected.

Bars: fields FP64 1e-11 / FP32 4e-6 of max |H|; energies FP64 1e-12 / FP32
2e-6 of the largest term; states FP64 1e-12 / FP32 1e-5.
"""
import dataclasses

import numpy as np
import pytest

from oracle import fields as ofl
from oracle import integrators as oit
from oracle import llg as ollg
from oracle import observables as oob
from oracle import rotation as orot
from workloads import random_unit, replica_seeds, uniform

from _mmx_case import Case, dev, host, open_ctx

pytestmark = pytest.mark.gpu

TOLF = {2: 1e-11, 1: 4e-6}
TOLE = {2: 1e-12, 1: 2e-6}
TOLM = {2: 1e-12, 1: 1e-5}


def _round(a, prec):
    return a.astype(np.float32).astype(np.float64) if prec == 1 else a


def _cells(case, seed, prec, which=("Ms", "A", "alpha", "Ku", "D")):
    rng = np.random.default_rng(seed)
    shape = case.n[::-1]
    lo_hi = {"Ms": (0.6 * case.Ms, 1.3 * case.Ms), "A": (0.7e-11, 1.6e-11),
             "alpha": (0.01, 0.3), "Ku": (-1e5, 5e5), "D": (-1e-3, 3e-3)}
    return {k: _round(rng.uniform(*lo_hi[k], shape), prec) for k in which}


def _apply(ctx, cells, prec):
    import paper_2608_15253_amd as mmx
    arg = {k: (dev(v, prec) if v is not None else None) for k, v in cells.items()}
    mmx.mmx_set_material_cells(ctx, 0, **arg)


def _omat(case, cells):
    mat = case.material()
    kw = {f"{k}_cells": v for k, v in cells.items() if k != "A"}
    if "A" in cells:
        kw["A_cells"] = cells["A"]
    return dataclasses.replace(mat, **kw)


CASES = {
    "block-open": Case((12, 10, 3), (3e-9, 2.5e-9, 2e-9), R=2, Ms=6e5, A=1.2e-11, D=2e-3, Ku=3e5,
                       u=(0.1, 0.2, 0.97), B=(0.01, -0.02, 0.05), alpha=0.1),
    "film-periodic": Case((16, 12, 1), (2e-9, 2e-9, 1e-9), pbc=(1, 1, 0), images=(1, 1, 0), R=2,
                          Ms=6e5, A=1.2e-11, D=2e-3, Ku=3e5, B=(0.0, 0.0, 0.05), alpha=0.1),
}


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("name", list(CASES))
def test_field_torque_and_energy_with_per_cell_materials(name, prec):
    import paper_2608_15253_amd as mmx
    case = CASES[name]
    print(f"[case] material cells {name} prec={prec}", flush=True)
    cells = _cells(case, 3, prec)
    m0 = _round(random_unit(case.n, seed=21, replicas=case.R), prec)
    ctx = open_ctx(case, prec)
    try:
        _apply(ctx, cells, prec)
        H, K = dev(np.zeros_like(m0), prec), dev(np.zeros_like(m0), prec)
        md = dev(m0, prec)
        mmx.mmx_field(ctx, md, H)
        mmx.mmx_torque(ctx, md, K)
        E = dev(np.zeros((case.R, 6)), 2)
        mmx.mmx_energy(ctx, md, E)
        got, gk, gE = host(H), host(K), host(E)
    finally:
        mmx.mmx_destroy(ctx)
    mat = _omat(case, cells)
    for r in range(case.R):
        ref = ofl.effective_field(m0[r], case.grid, mat)
        assert np.abs(got[r] - ref).max() <= TOLF[prec] * np.abs(ref).max()
        kref = ollg.llg_rhs(m0[r], ref, ofl.cell_param(mat, "alpha"))
        assert np.abs(gk[r] - kref).max() <= TOLF[prec] * np.abs(kref).max()
        e = oob.energies(m0[r], case.grid, mat)
        slots = [e["exchange"], e["dmi"], e["demag"], e["anisotropy"], e["zeeman"], e["total"]]
        scale = max(abs(x) for x in slots[:5])
        assert np.abs(gE[r] - np.array(slots)).max() <= TOLE[prec] * scale


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_uniform_arrays_reproduce_uniform_material(prec):
    import paper_2608_15253_amd as mmx
    case = CASES["block-open"]
    shape = case.n[::-1]
    cells = {"Ms": np.full(shape, case.Ms), "A": np.full(shape, case.A),
             "alpha": np.full(shape, case.alpha), "Ku": np.full(shape, case.Ku),
             "D": np.full(shape, case.D)}
    m0 = _round(random_unit(case.n, seed=22, replicas=case.R), prec)
    out = []
    for use in (False, True):
        ctx = open_ctx(case, prec)
        try:
            if use:
                _apply(ctx, cells, prec)
            K = dev(np.zeros_like(m0), prec)
            mmx.mmx_torque(ctx, dev(m0, prec), K)
            out.append(host(K))
        finally:
            mmx.mmx_destroy(ctx)
    assert np.abs(out[0] - out[1]).max() <= TOLF[prec] * np.abs(out[0]).max()


@pytest.mark.parametrize("scheme", ["heun", "depondt"])
@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_thermal_steps_with_per_cell_materials(scheme, prec):
    """Brown field with per-cell alpha and Ms (sigma_i), torque with alpha_i,
    demag of Ms_i m: 20 steps of 2 replicas of a 64 x 32 film (FP32: the
    field kernels take the film instead of the register row kernels)."""
    import paper_2608_15253_amd as mmx
    case = Case((64, 32, 1), (4e-9, 4e-9, 3e-9), R=2, alpha=0.05, Ku=4e5, B=(0, 0, -0.1),
                D=1e-3, T=300.0, seeds=list(replica_seeds(17, 2)),
                terms=("exchange", "dmi", "anisotropy", "zeeman", "demag", "thermal"))
    cells = _cells(case, 5, prec)
    m0 = _round(uniform(case.n, (0.2, 0.0, 1.0), replicas=case.R), prec)
    ctx = open_ctx(case, prec)
    try:
        _apply(ctx, cells, prec)
        md = dev(m0, prec)
        getattr(mmx, "mmx_" + scheme)(ctx, md, 1e-14, 20, 3)
        mmx.mmx_sync(ctx)
        got = host(md)
    finally:
        mmx.mmx_destroy(ctx)
    mat = _omat(case, cells)
    seeds = np.array(case.seeds)
    if scheme == "heun":
        ref = oit.heun_run(m0, case.grid, mat, 1e-14, 20, seed=seeds, step0=3)
    else:
        ref = orot.depondt_run(m0, case.grid, mat, 1e-14, 20, seed=seeds, step0=3)
    assert np.abs(got - ref).max() <= TOLM[prec]


@pytest.mark.parametrize("prec", [2, 1], ids=["f64", "f32"])
def test_rk45_replay_with_per_cell_materials(prec):
    import paper_2608_15253_amd as mmx
    case = Case((24, 20, 1), (3e-9, 3e-9, 2e-9), R=1, alpha=0.3, Ku=2e5, D=1.5e-3,
                B=(0, 0, 0.05), terms=("exchange", "dmi", "anisotropy", "zeeman", "demag"))
    cells = _cells(case, 7, prec)
    m0 = _round(random_unit(case.n, seed=23, replicas=1), prec)
    ctx = open_ctx(case, prec)
    try:
        _apply(ctx, cells, prec)
        md = dev(m0, prec)
        mmx.mmx_rk45(ctx, md, 0.0, 5e-12, 1e-5)
        dts = mmx.mmx_rk45_dts(ctx)
        got = host(md)
    finally:
        mmx.mmx_destroy(ctx)
    assert len(dts) > 5
    ref = oit.rk45_run(m0[0], case.grid, _omat(case, cells), 0.0, sum(dts), 1e-5,
                       dt_replay=dts).m
    assert np.abs(got[0] - ref).max() <= TOLM[prec]


def test_invalid_per_cell_values_are_rejected():
    import torch
    import paper_2608_15253_amd as mmx
    case = CASES["film-periodic"]
    ctx = open_ctx(case, 2)
    try:
        bad = np.full(case.n[::-1], case.Ms)
        bad[0, 3, 4] = 0.0
        with pytest.raises(mmx.MMXError) as e:
            mmx.mmx_set_material_cells(ctx, 0, Ms=dev(bad, 2))
        assert e.value.status == -1
        bad = np.full(case.n[::-1], 0.1)
        bad[0, 1, 1] = np.nan
        with pytest.raises(mmx.MMXError) as e:
            mmx.mmx_set_material_cells(ctx, 0, alpha=dev(bad, 2))
        assert e.value.status == -1
    finally:
        mmx.mmx_destroy(ctx)
