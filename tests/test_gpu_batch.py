"""GPU parity of many-cell batches (form 2).

One system holds cells with different boxes, sphere sizes, band counts,
k-point sets and electron counts (odd ones included); every SCF iteration
runs as single launches over all (cell, k-point) items.  Checks:
  * each cell's SCF trajectory equals the FP64 oracle's (1e-8 Ha/atom) and
    the trajectory of the same cell run as a system of its own;
  * graph replay gives exactly the eager results (same kernels, same order);
  * the 48-cell batched-throughput workload runs in FP32 bulk precision under
    graph replay, and sampled cells equal their own single-cell runs.
"""
import numpy as np
import pytest

import workloads as W
from oracle import energy as oe, scf as oscf
from tests._gpu import Device, log

pytestmark = pytest.mark.gpu
TOL_ATOM = 1e-8


@pytest.fixture(scope="module")
def dev():
    return Device()


def _mixed_cells():
    """Small cells of different shapes: 1 and 4 k-points, 3-5 bands, boxes
    12^3 to 16x15x18, a non-cubic cell, odd and even electron counts, with and
    without projectors, plus the two smallest one-k-point config-4 cells."""
    cells = [
        W.tiny_cell(nat=2, L=6.0, ecut=3.0, S=(12, 12, 12), nb=3, Z=(1, 1), seed=7),
        W.tiny_cell(nat=3, L=7.0, ecut=3.5, S=(16, 15, 18), nb=5, Z=(4, 1, 4), fold=(2, 1, 2),
                    R=np.array([[7.0, 0.5, 0.0], [0.0, 6.6, 0.7], [0.4, 0.0, 7.3]]), seed=31),
        W.tiny_cell(nat=2, L=6.5, ecut=3.0, S=(15, 15, 15), nb=4, Z=(4, 4), fold=(1, 2, 1), seed=13),
    ]
    c4 = [c for c in W.config4() if len(c.kpts) == 1]
    c4.sort(key=lambda c: (c.S[0], c.nb * c.nat))
    return cells + c4[:2]


def _desc(cell):
    return dict(R=cell.R, S=cell.S, ecut=cell.ecut, kpts=cell.kpts, wk=cell.wk, nb=cell.nb,
                n_electrons=cell.n_electrons, tau=cell.tau, Z=cell.Z.astype(float), rc=cell.rc,
                has_proj=cell.has_proj.astype(int), rp=W.PROJ_RP, D=W.PROJ_D)


def _batch(dev, cells, prec=0):
    D = dev.D
    s = D.dpp_batch_create(dev.ctx, [_desc(c) for c in cells], prec)
    off, npw = D.dpp_system_layout(s)
    item0, foff, state0 = D.dpp_system_cells(s)
    blocks = []
    for ci, c in enumerate(cells):
        ks = range(item0[ci], item0[ci + 1])
        blocks += W.initial_wavefunctions(c.y0_seed, [(c.nb, npw[k]) for k in ks])
    Y = dev.tensor(np.concatenate([b.reshape(-1) for b in blocks]))
    return s, Y, (off, npw, item0, foff, state0)


def _run(dev, s, Y, cells, nit, graph=False):
    D = dev.D
    D.dpp_set_graph_mode(s, graph)
    D.dpp_scf_init(s, cells=[dict(tau=c.tau, Z=c.Z, sigma=W.START_SIGMA) for c in cells])
    E, eig = [], None
    for _ in range(nit):
        e, eig = D.dpp_scf_iteration(s, Y)
        E.append([x["E_el"] for x in e])
    return np.array(E), eig


def test_batch_scf_matches_oracle_and_single_cells(dev):
    cells = _mixed_cells()
    nit = 4
    log("batch: " + ", ".join(f"{c.name} S={c.S} nk={len(c.kpts)} nb={c.nb} ne={c.n_electrons}" for c in cells))
    s, Y, _ = _batch(dev, cells)
    Eb, _ = _run(dev, s, Y, cells, nit)
    dev.D.dpp_system_destroy(s)
    for ci, c in enumerate(cells):
        so = oe.build_system(c)
        Ys = W.initial_wavefunctions(c.y0_seed, [(c.nb, b.npw) for b in so.bases])
        res = oscf.scf(so, [y.T.copy() for y in Ys], oe.start_density(c, W.START_SIGMA), nit)
        err = np.max(np.abs(Eb[:, ci] - np.array(res["energies"]))) / c.nat
        log(f"{c.name}: batch {Eb[-1, ci]:.12f} oracle {res['energies'][-1]:.12f} err/atom {err:.2e}")
        assert err < TOL_ATOM
        # the same cell as a system of its own
        s1, Y1, _ = _batch(dev, [c])
        E1, _ = _run(dev, s1, Y1, [c], nit)
        dev.D.dpp_system_destroy(s1)
        assert np.max(np.abs(E1[:, 0] - Eb[:, ci])) / c.nat < 1e-10


def test_graph_replay_equals_eager(dev):
    cells = _mixed_cells()[:3]
    out = {}
    for graph in (False, True):
        s, Y, _ = _batch(dev, cells)
        E, eig = _run(dev, s, Y, cells, 6, graph=graph)
        out[graph] = (E, eig, dev.host(Y))
        dev.D.dpp_system_destroy(s)
    log(f"eager {out[False][0][-1]} graph {out[True][0][-1]}")
    assert np.array_equal(out[False][0], out[True][0])
    assert np.array_equal(out[False][1], out[True][1])
    assert np.array_equal(out[False][2], out[True][2])


def test_graph_replay_config2_mixed(dev):
    """Config 2 in FP32 bulk precision: graph replay equals eager execution."""
    cell = W.config2()
    out = {}
    for graph in (False, True):
        s, Y, _ = _batch(dev, [cell], prec=1)
        E, eig = _run(dev, s, Y, [cell], 4, graph=graph)
        out[graph] = (E, eig)
        dev.D.dpp_system_destroy(s)
    assert np.array_equal(out[False][0], out[True][0])
    assert np.array_equal(out[False][1], out[True][1])


@pytest.mark.parametrize("case", ["full", "partial", "odd"])
def test_fillings_match_oracle_aufbau(dev, case):
    """The device aufbau fillings after one SCF iteration equal the oracle's
    rule applied to the same eigenvalues: every state occupied (2 atoms Z=4,
    4 bands, 2 k-points), empty bands (Z=1 pair, 3 bands) and an odd electron
    count (9 electrons, 5 bands)."""
    D = dev.D
    cell = {
        "full": W.tiny_cell(nat=2, L=6.5, ecut=3.0, S=(15, 15, 15), nb=4, Z=(4, 4), fold=(1, 2, 1), seed=13),
        "partial": W.tiny_cell(nat=2, L=6.0, ecut=3.0, S=(12, 12, 12), nb=3, Z=(1, 1), seed=7),
        "odd": W.tiny_cell(nat=3, L=7.0, ecut=3.5, S=(16, 15, 18), nb=5, Z=(4, 1, 4), fold=(2, 1, 2), seed=31),
    }[case]
    nk = len(cell.kpts)
    s, Y, _ = _batch(dev, [cell])
    D.dpp_scf_init(s, cells=[dict(tau=cell.tau, Z=cell.Z, sigma=W.START_SIGMA)])
    _, eig = D.dpp_scf_iteration(s, Y)
    f = D.dpp_system_fillings(s, nk, cell.nb)
    D.dpp_system_destroy(s)
    eig = np.asarray(eig).reshape(nk, cell.nb)
    ref = oscf.aufbau_fillings([eig[k] for k in range(nk)], np.asarray(cell.wk), cell.n_electrons)
    log(f"fillings {case}: {f.ravel()}")
    assert np.array_equal(f, np.array(ref))
    if case == "full":
        assert np.all(f == 2.0)


def test_config4_batch_fp32_graph(dev):
    """The 48-cell throughput workload: FP32 bulk, graph replay, three SCF
    iterations.  Three sampled cells match the FP64 oracle's three iterations
    from the same start at the mixed-precision bars (1e-6 Ha/atom, 1e-5 Ha on
    every eigenvalue, 1e-5 relative L1 on the output density) and equal their
    own single-cell runs."""
    cells = W.config4()
    s, Y, lay = _batch(dev, cells, prec=1)
    _, _, _, foff, state0 = lay
    nc, nitems, total, nstates, ngrid = dev.D.dpp_system_dims(s)
    log(f"config4: {nc} cells, {nitems} items, {total} coefficients per block, {nstates} states, {ngrid} grid points")
    E, eig = _run(dev, s, Y, cells, 3, graph=True)
    res = dev.D.dpp_scf_cell_residuals(s)
    nall = dev.empty((ngrid,), dev.torch.float64)
    dev.D.dpp_system_copy_field(s, dev.D.DPP_FIELD_NOUT, nall)
    nall = dev.host(nall)
    dev.D.dpp_system_destroy(s)
    assert np.all(np.isfinite(E)) and np.all(np.isfinite(res))
    for ci in (0, 17, 47):
        c = cells[ci]
        so = oe.build_system(c)
        Ys = W.initial_wavefunctions(c.y0_seed, [(c.nb, b.npw) for b in so.bases])
        ro = oscf.scf(so, [y.T.copy() for y in Ys], oe.start_density(c, W.START_SIGMA), 3)
        dE = np.max(np.abs(E[:, ci] - np.array(ro["energies"]))) / c.nat
        de = np.max(np.abs(np.asarray(eig[state0[ci]:state0[ci + 1]]).reshape(len(c.kpts), c.nb) -
                           np.array(ro["eigs"])))
        nc_ = nall[foff[ci]:foff[ci] + int(np.prod(c.S))].reshape(c.S)
        dn = np.sum(np.abs(nc_ - ro["n_out"])) / np.sum(np.abs(ro["n_out"]))
        log(f"cell {ci} ({c.nat} atoms, {len(c.kpts)} k, {c.nb} bands): vs oracle dE/atom {dE:.2e} "
            f"d eig {de:.2e} density L1 {dn:.2e}")
        assert dE < 1e-6 and de < 1e-5 and dn < 1e-5
        s1, Y1, _ = _batch(dev, [c], prec=1)
        E1, _ = _run(dev, s1, Y1, [c], 3, graph=True)
        dev.D.dpp_system_destroy(s1)
        log(f"cell {ci}: batch {E[-1, ci]:.12f} single {E1[-1, 0]:.12f}")
        assert np.max(np.abs(E1[:, 0] - E[:, ci])) / c.nat < 1e-9


def test_tuner_keeps_results(dev):
    """The launch autotuner times the x-pass, rotate and overlap variants on
    the system's items; H Y and the SCF trajectory after tuning agree with an
    untuned system to rounding."""
    D = dev.D
    cells = _mixed_cells()
    sa, Ya, _ = _batch(dev, cells)
    sb, Yb, _ = _batch(dev, cells)
    Ea, _ = _run(dev, sa, Ya, cells, 1)
    Eb, _ = _run(dev, sb, Yb, cells, 1)
    HYa = dev.torch.empty_like(Ya)
    HYb = dev.torch.empty_like(Yb)
    D.dpp_system_apply_H(sa, Ya, HYa)
    D.dpp_system_tune(sb, Yb, HYb, reps=2)
    rep = D.dpp_system_tune_report(sb)
    log("tuning: " + rep)
    assert "x pass" in rep and "overlap blocks" in rep and "->" in rep
    D.dpp_system_apply_H(sb, Yb, HYb)
    a, b = dev.host(HYa), dev.host(HYb)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))
    # two more SCF iterations on each (tuning dropped the band-CG state only)
    Ea2, Eb2 = [], []
    for _ in range(2):
        ea, _ = D.dpp_scf_iteration(sa, Ya)
        eb, _ = D.dpp_scf_iteration(sb, Yb)
        Ea2.append([x["E_el"] for x in ea])
        Eb2.append([x["E_el"] for x in eb])
    nat = np.array([c.nat for c in cells])
    err = np.max(np.abs(np.array(Ea2) - np.array(Eb2)) / nat)
    log(f"SCF after tuning: max difference {err:.2e} Ha/atom")
    assert err < 1e-10
    D.dpp_system_destroy(sa)
    D.dpp_system_destroy(sb)


@pytest.mark.parametrize("which,value", [(0, 1), (0, 2), (0, 3), (1, 2), (1, 4), (2, 1), (2, 2), (2, 3)])
def test_launch_choices_match_default(dev, which, value):
    """Every launch variant the tuner can pick gives the default SCF energies
    to rounding (mixed cells: several boxes, band counts and k-point sets)."""
    D = dev.D
    cells = _mixed_cells()
    sa, Ya, _ = _batch(dev, cells)
    Ea, _ = _run(dev, sa, Ya, cells, 3)
    D.dpp_system_destroy(sa)
    sb, Yb, _ = _batch(dev, cells)
    D.dpp_system_set_launch_choice(sb, which, value)
    Eb, _ = _run(dev, sb, Yb, cells, 3)
    D.dpp_system_destroy(sb)
    nat = np.array([c.nat for c in cells])
    err = np.max(np.abs(Ea - Eb) / nat)
    log(f"choice {which}={value}: max difference {err:.2e} Ha/atom")
    assert err < 1e-10


@pytest.mark.parametrize("S0", [40, 90])
@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_x_pass_variants(dev, prec, S0):
    """At config 2's 40-point and config 3's 90-point x lengths every x-pass
    variant the tuner can pick (one thread per column where it compiles, lane
    pair, LDS) gives the LDS pass's H Y to rounding; the box is S0 x 20 x 18.
    H is applied at the potential of one SCF iteration: the x pass multiplies
    by V_eff, so with no potential set every variant would transform zeros and
    agree trivially.  The test checks that the potential's part of H Y is
    there (at least 1% of max |H Y|; it is about 6%)."""
    D = dev.D
    cell = W.tiny_cell(nat=2, L=10.0, ecut=4.0, S=(S0, 20, 18), nb=4, Z=(4, 4), seed=19)
    s, Y, _ = _batch(dev, [cell], prec=prec)
    Y0 = Y.clone()
    HY = dev.torch.empty_like(Y)
    D.dpp_system_apply_H(s, Y0, HY)  # no potential yet: kinetic and nonlocal terms only
    no_v = dev.host(HY)
    D.dpp_scf_init(s, cells=[dict(tau=cell.tau, Z=cell.Z, sigma=W.START_SIGMA)])
    D.dpp_scf_iteration(s, Y)  # sets V_eff
    out = {}
    variants = (0, 1, 2)
    for v in (3,) + variants:  # LDS first: the reference
        D.dpp_system_set_launch_choice(s, D.DPP_CHOICE_XPASS, v)
        D.dpp_system_apply_H(s, Y0, HY)
        out[v] = dev.host(HY)
    D.dpp_system_destroy(s)
    ref = out[3]
    share = np.max(np.abs(ref - no_v)) / np.max(np.abs(ref))
    log(f"x pass S0={S0} prec={prec}: potential part {share:.2f} of max |H Y|")
    assert share > 0.01
    tol = 1e-12 if prec == 0 else 1e-5
    for v in variants:
        err = np.max(np.abs(out[v] - ref)) / np.max(np.abs(ref))
        log(f"x pass variant {v} at S0={S0} prec={prec}: max rel difference {err:.2e}")
        assert err < tol
