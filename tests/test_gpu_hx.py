"""GPU parity of the Hamiltonian kernels and the Chebyshev filter against the
FP64 oracle, through the C ABI.

Inputs: the 0.55 nm Si35H36 cluster (seed 1001) on its h = 0.7 bohr sphere
(72,455 points, 241 Hilbert blocks -- many tiles and ragged boundary
blocks), random N(0, 1) blocks from seeded generators, V_eff = V_loc plus a
seeded smooth perturbation.

Tolerances (relative to the largest |entry| of the reference):
* FP64: 1e-12 for H X (37 + 1 + KB terms of O(1) magnitude summed in a
  different order: a few ulps times the ~1e2 dynamic range of -1/2 c_k / h^2),
  1e-10 for a degree-10 filter (the recurrence amplifies rounding by at most
  |T_m| growth on [a0, b], bounded here by ~1e2).
* FP32: 2e-6 for H X (eps_32 = 6e-8 times the same ~30 cancellation factor),
  5e-5 for the degree-10 filter.
"""
import math

import numpy as np
import pytest

from oracle import chfsi as OC
from oracle import grid as G
from oracle import hamiltonian as OH
from synth.cluster import make_cluster, random_block

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

H_SPACING = 0.7


@pytest.fixture(scope="module")
def system():
    from paper_2303_00790_amd import binding as B
    c = make_cluster(5.5, 1001)
    radius = c.domain_radius()
    pp = OH.PseudoParams(h_s=2.0, h_p=0.5)   # p channel switched on so every KB column is exercised
    g = G.build_grid(radius, H_SPACING)
    Ho = OH.build_hamiltonian(g, c.pos, c.species, pp)
    rng = np.random.default_rng(77)
    pert = 0.05 * np.sin(g.xyz @ rng.standard_normal(3))
    Ho.veff = Ho.vloc + pert
    Hg = B.Hamiltonian(c.pos, c.species, pp, H_SPACING, radius, B.ORDER_HILBERT, keep_nbr=True)
    rows = torch.from_numpy(g.row_of_rank).cuda()
    veff_rows = torch.zeros(Hg.n_rows, dtype=torch.float64, device="cuda")
    veff_rows[rows] = torch.from_numpy(Ho.veff).cuda()
    Hg.set_veff(veff_rows)
    return dict(B=B, c=c, g=g, Ho=Ho, Hg=Hg, rows=rows, pp=pp, radius=radius)


def to_rows(s, X, dtype, ld=None):
    n, m = X.shape
    ld = ld or m
    out = torch.zeros((s["Hg"].n_rows, ld), dtype=dtype, device="cuda")
    out[s["rows"], :m] = torch.from_numpy(X).to(device="cuda", dtype=dtype)
    return out


def from_rows(s, Y, m):
    return Y[s["rows"], :m].double().cpu().numpy()


def relerr(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_ordering_and_vloc(system):
    s = system
    ijk, rows, nbr = s["Hg"].export_ordering(with_nbr=True)
    assert np.array_equal(ijk, s["g"].ijk) and np.array_equal(rows, s["g"].row_of_rank)
    assert np.array_equal(nbr, G.neighbour_table(s["g"]))
    v = s["Hg"].vloc()[s["rows"]].cpu().numpy()
    assert relerr(v, s["Ho"].vloc) < 1e-13
    pad = torch.ones(s["Hg"].n_rows, dtype=torch.bool, device="cuda")
    pad[s["rows"]] = False
    assert float(s["Hg"].vloc()[pad].abs().max()) == 0.0


@pytest.mark.parametrize("generic", [False, True])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-6)])
@pytest.mark.parametrize("m,ld", [(64, 64), (36, 40), (8, 8), (5, 8), (5, 5), (1, 1)])
def test_apply_parity(system, generic, dtype, tol, m, ld):
    s = system
    X = random_block(s["g"].n, m, 2001 + m)
    ref = s["Ho"].apply(X)
    Xg = to_rows(s, X, dtype, ld)
    Yg = torch.full_like(Xg, float("nan"))
    s["Hg"].apply(Xg[:, :m], Yg[:, :m], generic=generic)
    assert relerr(from_rows(s, Yg, m), ref) < tol
    pad = torch.ones(s["Hg"].n_rows, dtype=torch.bool, device="cuda")
    pad[s["rows"]] = False
    assert float(Yg[pad][:, :m].abs().max()) == 0.0
    if ld > m:   # columns beyond nvec untouched
        assert bool(torch.isnan(Yg[:, m:]).all())


def _bounds(s):
    v0 = random_block(s["g"].n, 1, 3001)[:, 0]
    b, tmin, _ = OC.lanczos_bound(s["Ho"].apply, v0, 10)
    return tmin + 0.1 * (b - tmin), b, tmin


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 5e-5)])
@pytest.mark.parametrize("degree,m", [(10, 32), (3, 36), (2, 8)])
def test_filter_parity(system, dtype, tol, degree, m):
    # degree >= 2 runs the fused KB-coefficient epilogue; m = 36 leaves a
    # ragged vector chunk, m = 8 a single one
    s = system
    a, b, a0 = _bounds(s)
    X = random_block(s["g"].n, m, 2100 + degree)
    ref = OC.chebyshev_filter(s["Ho"].apply, X, degree, a, b, a0)
    Xg = to_rows(s, X, dtype)
    W = torch.full_like(Xg, float("nan"))
    s["Hg"].filter(Xg, W, degree, a, b, a0)
    assert relerr(from_rows(s, Xg, m), ref) < tol
    pad = torch.ones(s["Hg"].n_rows, dtype=torch.bool, device="cuda")
    pad[s["rows"]] = False
    assert float(Xg[pad].abs().max()) == 0.0


def test_filter_tiled_equals_generic_and_is_deterministic(system):
    s = system
    a, b, a0 = _bounds(s)
    X = random_block(s["g"].n, 64, 2200)
    outs = []
    for generic in (False, False, True):
        Xg = to_rows(s, X, torch.float64)
        W = torch.zeros_like(Xg)
        s["Hg"].filter(Xg, W, 8, a, b, a0, generic=generic)
        outs.append(Xg)
    assert torch.equal(outs[0], outs[1])
    assert float((outs[0] - outs[2]).abs().max() / outs[2].abs().max()) < 1e-12


def test_lexicographic_layout_parity(system):
    s = system
    B = s["B"]
    Hl = B.Hamiltonian(s["c"].pos, s["c"].species, s["pp"], H_SPACING, s["radius"], B.ORDER_LEX)
    gl = G.build_grid(s["radius"], H_SPACING, G.ORDER_LEX)
    veff = torch.from_numpy(OH.local_potential(gl, s["c"].pos, s["c"].species, s["pp"])).cuda()
    Hl.set_veff(veff)
    Hol = OH.build_hamiltonian(gl, s["c"].pos, s["c"].species, s["pp"])
    X = random_block(gl.n, 16, 2300)
    Xg = torch.from_numpy(X).cuda()
    Yg = torch.empty_like(Xg)
    Hl.apply(Xg, Yg)
    assert relerr(Yg.cpu().numpy(), Hol.apply(X)) < 1e-12


def test_invalid_arguments_rejected(system):
    s = system
    B = s["B"]
    X = torch.zeros((s["Hg"].n_rows, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(B.ChfError) as e:
        s["Hg"].filter(X, X.clone(), 5, 1.0, 0.5, -1.0)   # a > b
    assert e.value.code == -1
    bad = torch.zeros(s["Hg"].n_rows, dtype=torch.float64, device="cuda")
    bad[s["rows"][5]] = float("nan")
    with pytest.raises(B.ChfError) as e:
        s["Hg"].set_veff(bad)
    assert e.value.code == -6


def test_empty_block_rejected(system):
    # no vectors (nvec = 0) and a leading dimension below nvec are invalid
    s = system
    B = s["B"]
    X = torch.zeros((s["Hg"].n_rows, 8), dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    with pytest.raises(B.ChfError) as e:
        B.call("ham_apply", s["Hg"].handle, B.CHF_F64, B._ptr(X), 8, B._ptr(Y), 8, 0, B._stream())
    assert e.value.code == -1
    with pytest.raises(B.ChfError) as e:
        B.call("ham_apply", s["Hg"].handle, B.CHF_F64, B._ptr(X), 4, B._ptr(Y), 8, 8, B._stream())
    assert e.value.code == -1


@pytest.mark.parametrize("species", ["none", "hydrogen"])
def test_no_projector_atoms(species):
    # degenerate Hamiltonians: no atoms at all (H = -1/2 L) and hydrogen only
    # (local potential, no KB term), both kernels
    from paper_2303_00790_amd import binding as B
    if species == "none":
        pos, spc = np.zeros((0, 3)), np.zeros(0, np.int32)
    else:
        pos, spc = np.array([[0.0, 0.0, 0.7], [0.0, 0.0, -0.7]]), np.ones(2, np.int32)
    pp = OH.PseudoParams(h_s=2.0, h_p=0.5)
    radius = 6.0
    g = G.build_grid(radius, H_SPACING)
    Ho = OH.build_hamiltonian(g, pos, spc, pp)
    Hg = B.Hamiltonian(pos, spc, pp, H_SPACING, radius, B.ORDER_HILBERT, keep_nbr=True)
    rows = torch.from_numpy(g.row_of_rank).cuda()
    X = random_block(g.n, 16, 2400)
    Xg = torch.zeros((Hg.n_rows, 16), dtype=torch.float64, device="cuda")
    Xg[rows] = torch.from_numpy(X).cuda()
    ref = Ho.apply(X)
    for generic in (False, True):
        Yg = torch.full_like(Xg, float("nan"))
        Hg.apply(Xg, Yg, generic=generic)
        assert relerr(Yg[rows].cpu().numpy(), ref) < 1e-12


def test_more_atoms_per_block_than_staged():
    # more than 64 projector atoms touching one 8^3 block: the tiled kernel
    # reads the KB coefficients from global memory instead of staging them
    from paper_2303_00790_amd import binding as B
    rng = np.random.default_rng(31)
    pos = rng.uniform(-3.0, 3.0, size=(90, 3))
    spc = np.zeros(90, np.int32)
    pp = OH.PseudoParams(h_s=2.0, h_p=0.5)
    radius = 9.0
    g = G.build_grid(radius, H_SPACING)
    Ho = OH.build_hamiltonian(g, pos, spc, pp)
    Hg = B.Hamiltonian(pos, spc, pp, H_SPACING, radius, B.ORDER_HILBERT, keep_nbr=True)
    rows = torch.from_numpy(g.row_of_rank).cuda()
    X = random_block(g.n, 8, 2500)
    Xg = torch.zeros((Hg.n_rows, 8), dtype=torch.float64, device="cuda")
    Xg[rows] = torch.from_numpy(X).cuda()
    ref = Ho.apply(X)
    for generic in (False, True):
        Yg = torch.full_like(Xg, float("nan"))
        Hg.apply(Xg, Yg, generic=generic)
        assert relerr(Yg[rows].cpu().numpy(), ref) < 1e-12


def test_rows_with_more_than_16_projector_entries():
    # 24 Si atoms inside 1.5 bohr of the origin: the rows near the centre have
    # 24 projector entries (the in-march KB term takes 16 entries from the
    # broadcast registers and the rest from memory), and every 8^3 block
    # touches at most 24 atoms, so the coefficients are staged in LDS.
    from paper_2303_00790_amd import binding as B
    rng = np.random.default_rng(33)
    d = rng.standard_normal((24, 3))
    pos = 1.5 * d / np.linalg.norm(d, axis=1, keepdims=True) * rng.uniform(0.2, 1.0, (24, 1))
    spc = np.zeros(24, np.int32)
    pp = OH.PseudoParams(h_s=2.0, h_p=0.5)
    radius = 9.0
    g = G.build_grid(radius, H_SPACING)
    Ho = OH.build_hamiltonian(g, pos, spc, pp)
    Hg = B.Hamiltonian(pos, spc, pp, H_SPACING, radius, B.ORDER_HILBERT, keep_nbr=True)
    rows = torch.from_numpy(g.row_of_rank).cuda()
    off, rk, _ = B.projectors_host(H_SPACING, radius, pos, spc, pp)
    per_point = np.bincount(rk, minlength=g.n)
    assert per_point.max() == 24 and (per_point > 16).sum() > 100
    for dtype, tol, m in ((torch.float64, 1e-12, 48), (torch.float32, 2e-6, 64)):
        X = random_block(g.n, m, 2600 + m)
        Xg = torch.zeros((Hg.n_rows, m), dtype=dtype, device="cuda")
        Xg[rows] = torch.from_numpy(X).to(device="cuda", dtype=dtype)
        ref = Ho.apply(X)
        Yg = torch.full_like(Xg, float("nan"))
        Hg.apply(Xg, Yg)
        assert relerr(Yg[rows].double().cpu().numpy(), ref) < tol, dtype


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_filter_narrow_work_equals_full_width(system, dtype):
    # a work block of 32 columns for 96 vectors: the filter runs column block
    # by column block; every vector's arithmetic is the same as in the
    # full-width call, so the results are identical
    s = system
    a, b, a0 = _bounds(s)
    X = random_block(s["g"].n, 96, 2700)
    Xa = to_rows(s, X, dtype)
    Xb = Xa.clone()
    s["Hg"].filter(Xa, torch.zeros_like(Xa), 7, a, b, a0)
    s["Hg"].filter(Xb, torch.zeros((s["Hg"].n_rows, 32), dtype=dtype, device="cuda"), 7, a, b, a0)
    assert torch.equal(Xa, Xb)


def test_filter_rejects_overlapping_work(system):
    s = system
    B = s["B"]
    buf = torch.zeros((s["Hg"].n_rows, 64), dtype=torch.float64, device="cuda")
    a, b, a0 = _bounds(s)
    with pytest.raises(B.ChfError) as e:
        s["Hg"].filter(buf[:, :32], buf[:, 16:48], 3, a, b, a0)
    assert e.value.code == -1
