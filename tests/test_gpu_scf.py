"""GPU parity of the SCF pieces and of whole SCF steps against the FP64
oracle, through the C ABI.

The end-to-end test runs a fixed number of SCF steps from identical inputs
(positions, SAD density, random start block, Lanczos vector) on both sides
and compares every step: the tracked eigenvalues and the Harris-Foulkes
energy within 1e-8 Ha (FP64 path), the SRE within 1e-6 relative.
"""
import math

import numpy as np
import pytest

from oracle import grid as G
from oracle import hamiltonian as OH
from oracle import scf as OS
from synth.cluster import make_cluster, n_states, random_block

from gpu_system import from_rows, relerr, to_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def si35():
    from paper_2303_00790_amd import binding as B
    c = make_cluster(5.5, 1001)
    radius = c.domain_radius()
    pp = OH.PseudoParams()
    g = G.build_grid(radius, 0.7)
    nbr = G.neighbour_table(g)
    Ho = OH.build_hamiltonian(g, c.pos, c.species, pp)
    Hg = B.Hamiltonian(c.pos, c.species, pp, 0.7, radius, B.ORDER_HILBERT)
    rows = torch.from_numpy(g.row_of_rank).cuda()
    return dict(B=B, c=c, g=g, nbr=nbr, Ho=Ho, Hg=Hg, rows=rows, pp=pp, ctx=B.Context(0))


def test_density(si35):
    s = si35
    X, _ = np.linalg.qr(random_block(s["g"].n, 40, 7))
    rho = torch.zeros(s["Hg"].n_rows, dtype=torch.float64, device="cuda")
    s["Hg"].density(to_rows(s, X, torch.float64), 33, rho)
    assert relerr(from_rows(s, rho), OS.density(X, 33, s["g"].h)) < 1e-13
    rho32 = torch.zeros_like(rho)
    s["Hg"].density(to_rows(s, X, torch.float32), 33, rho32)
    assert relerr(from_rows(s, rho32), OS.density(X, 33, s["g"].h)) < 1e-6


def test_lda(si35):
    s = si35
    rng = np.random.default_rng(3)
    rho = np.concatenate([10 ** rng.uniform(-16, 1, s["g"].n - 3), [0.0, 1e-15, 0.5]])
    rg = to_rows(s, rho, torch.float64)
    exc = torch.zeros_like(rg)
    vxc = torch.zeros_like(rg)
    s["Hg"].lda(rg, exc, vxc)
    e_ref, v_ref = OS.lda(rho)
    assert np.allclose(from_rows(s, exc), e_ref, rtol=1e-13, atol=1e-300)
    assert np.allclose(from_rows(s, vxc), v_ref, rtol=1e-13, atol=1e-300)


def test_sad_and_ion_energy(si35):
    s = si35
    ne = s["c"].n_electrons
    rho = s["Hg"].sad_density(s["c"].pos, s["c"].species, ne)
    ref = OS.sad_density(s["g"], s["c"].pos, s["c"].species, ne)
    assert relerr(from_rows(s, rho), ref) < 1e-12
    eii = s["B"].ion_energy(s["c"].pos, s["c"].species, s["pp"])
    assert abs(eii - OS.ion_energy(s["c"].pos, s["pp"].charges(s["c"].species))) < 1e-10 * abs(eii)


@pytest.mark.parametrize("centre", [(0.0, 0.0, 0.0), (1.3, -0.8, 0.6)])
def test_hartree(si35, centre):
    s = si35
    d2 = ((s["g"].xyz - np.array(centre)) ** 2).sum(1)
    rho = 3.0 * (2 * math.pi * 1.5 ** 2) ** -1.5 * np.exp(-d2 / (2 * 1.5 ** 2))
    vref, _ = OS.hartree(s["g"], s["Ho"].lap, s["nbr"], rho)
    vh = torch.zeros(s["Hg"].n_rows, dtype=torch.float64, device="cuda")
    it = s["Hg"].hartree(s["ctx"], to_rows(s, rho, torch.float64), vh, 1e-12)
    assert it > 10
    assert relerr(from_rows(s, vh), vref) < 1e-10


def test_scf_steps_fp64(si35):
    s = si35
    B = s["B"]
    c = s["c"]
    ne = c.n_electrons
    M = n_states(ne)
    X0 = random_block(s["g"].n, M, 2001)
    v0 = random_block(s["g"].n, 1, 3001)[:, 0]
    eii = OS.ion_energy(c.pos, s["pp"].charges(c.species))
    # oracle
    st = OS.ScfState(OS.sad_density(s["g"], c.pos, c.species, ne), X0.copy(), np.zeros(s["g"].n))
    Ho = OH.build_hamiltonian(s["g"], c.pos, c.species, s["pp"])
    ref = [OS.scf_step(Ho, s["nbr"], st, ne, 10, v0, eii) for _ in range(4)]
    # device
    prm = B.ScfParams(ne, M, 10, 4, 1, 10, B.CHF_F64, B.CHF_F64, 6, 0.3, 1e-12, eii)
    rho0 = s["Hg"].sad_density(c.pos, c.species, ne)
    scf = B.Scf(s["Hg"], s["ctx"], prm, rho0, to_rows(s, v0, torch.float64))
    X = to_rows(s, X0, torch.float64)
    W = torch.zeros_like(X)
    for k in range(4):
        rep, eig = scf.step(X, W)
        r = ref[k]
        assert rep.step == k + 1
        assert np.abs(eig - r.eig).max() < 1e-8, (k, np.abs(eig - r.eig).max())
        assert abs(rep.energy - r.energy) < 1e-8, (k, rep.energy, r.energy)
        assert abs(rep.sre_ry - r.sre_ry) < 1e-6 * r.sre_ry
        assert abs(rep.homo - r.homo) < 1e-8 and abs(rep.lumo - r.lumo) < 1e-8
    # the mixed density kept by the state equals the oracle's
    rho_in = torch.zeros(s["Hg"].n_rows, dtype=torch.float64, device="cuda")
    vh = torch.zeros_like(rho_in)
    scf.fields(rho_in, vh)
    assert relerr(from_rows(s, rho_in), st.rho_in) < 1e-8


def test_scf_narrow_work_matches_full_width(si35):
    """scf_step with a work block of 32 columns for 128 states (filter in
    column blocks, Rayleigh-Ritz rotation in row panels) gives the
    full-width step's eigenvalues, energy and SRE within 1e-12 (FP64; the
    two differ only in the summation order of the Gram and rotation
    products)."""
    s = si35
    B = s["B"]
    c = s["c"]
    ne = c.n_electrons
    M = n_states(ne)
    X0 = random_block(s["g"].n, M, 2005)
    v0 = to_rows(s, random_block(s["g"].n, 1, 3005)[:, 0], torch.float64)
    eii = OS.ion_energy(c.pos, s["pp"].charges(c.species))
    prm = B.ScfParams(ne, M, 10, 4, 1, 10, B.CHF_F64, B.CHF_F64, 6, 0.3, 1e-12, eii)
    rho0 = s["Hg"].sad_density(c.pos, c.species, ne)
    runs = []
    for width in (M, 32):
        scf = B.Scf(s["Hg"], s["ctx"], prm, rho0, v0)
        X = to_rows(s, X0, torch.float64)
        W = torch.zeros((s["Hg"].n_rows, width), dtype=torch.float64, device="cuda")
        runs.append([scf.step(X, W) for _ in range(2)] + [X])
    for k in range(2):
        (ra, ea), (rb, eb) = runs[0][k], runs[1][k]
        assert np.abs(ea - eb).max() < 1e-12 * np.abs(ea).max(), k
        assert abs(ra.energy - rb.energy) < 1e-12 * abs(ra.energy), k
        assert abs(ra.sre_ry - rb.sre_ry) < 1e-10 * ra.sre_ry, k
    n_occ = ne // 2
    Xa, Xb = runs[0][2][:, :n_occ], runs[1][2][:, :n_occ]
    # occupied subspaces agree: the projectors X X^T on the occupied columns
    overlap = (Xa.T @ Xb).cpu().numpy()
    assert abs(np.linalg.svd(overlap, compute_uv=False).min() - 1.0) < 1e-10


def test_scf_step_rejects_overlapping_work(si35):
    s = si35
    B = s["B"]
    c = s["c"]
    ne = c.n_electrons
    M = n_states(ne)
    eii = OS.ion_energy(c.pos, s["pp"].charges(c.species))
    prm = B.ScfParams(ne, M, 10, 4, 1, 10, B.CHF_F64, B.CHF_F64, 6, 0.3, 1e-12, eii)
    rho0 = s["Hg"].sad_density(c.pos, c.species, ne)
    v0 = to_rows(s, random_block(s["g"].n, 1, 3005)[:, 0], torch.float64)
    scf = B.Scf(s["Hg"], s["ctx"], prm, rho0, v0)
    buf = torch.zeros((s["Hg"].n_rows, 2 * M), dtype=torch.float64, device="cuda")
    with pytest.raises(B.ChfError) as e:
        scf.step(buf[:, :M], buf[:, M // 2:M // 2 + 32])
    assert e.value.code == -1


def test_mixed_scf_keeps_the_electron_count(si35):
    """The output density of a step is scaled to hold N_e electrons, so
    rho_in, an Anderson combination of such densities and of the normalised
    superposition start, holds N_e after every step of a mixed-precision SCF
    (FP32 filter and Gram).  Without the scaling it would carry the column
    norm error that FP32 Cholesky-QR leaves, ~1e-7 relative."""
    s = si35
    B = s["B"]
    c = s["c"]
    ne = c.n_electrons
    M = n_states(ne)
    eii = OS.ion_energy(c.pos, s["pp"].charges(c.species))
    prm = B.ScfParams(ne, M, 10, 4, 1, 10, B.CHF_F32, B.CHF_F32, 6, 0.3, 1e-12, eii)
    rho0 = s["Hg"].sad_density(c.pos, c.species, ne)
    v0 = to_rows(s, random_block(s["g"].n, 1, 3005)[:, 0], torch.float64)
    scf = B.Scf(s["Hg"], s["ctx"], prm, rho0, v0)
    X = to_rows(s, random_block(s["g"].n, M, 2005), torch.float32)
    W = torch.zeros((s["Hg"].n_rows, M), dtype=torch.float32, device="cuda")
    h3 = 0.7 ** 3
    rho = torch.zeros(s["Hg"].n_rows, dtype=torch.float64, device="cuda")
    for _ in range(3):
        scf.step(X, W)
        scf.fields(rho)
        q = h3 * float(rho.sum())
        assert abs(q - ne) < 1e-11 * ne, (q, ne)


def test_checkpoint_resume_is_bit_exact(si35):
    """Saving the SCF state after three steps and resuming it in a fresh
    handle reproduces the fourth step of the uninterrupted run exactly."""
    s = si35
    B = s["B"]
    c = s["c"]
    ne = c.n_electrons
    M = n_states(ne)
    X0 = random_block(s["g"].n, M, 2002)
    v0 = to_rows(s, random_block(s["g"].n, 1, 3002)[:, 0], torch.float64)
    eii = OS.ion_energy(c.pos, s["pp"].charges(c.species))
    prm = B.ScfParams(ne, M, 10, 4, 1, 10, B.CHF_F64, B.CHF_F64, 6, 0.3, 1e-12, eii)
    rho0 = s["Hg"].sad_density(c.pos, c.species, ne)
    scf = B.Scf(s["Hg"], s["ctx"], prm, rho0, v0)
    X = to_rows(s, X0, torch.float64)
    W = torch.zeros_like(X)
    for _ in range(3):
        scf.step(X, W)
    state = scf.save()
    assert state.size == 8 + (2 + 2 * 3) * s["Hg"].n_rows
    X_saved = X.clone()
    rep, eig = scf.step(X, W)
    rho_a = torch.zeros(s["Hg"].n_rows, dtype=torch.float64, device="cuda")
    scf.fields(rho_a)

    fresh = B.Scf(s["Hg"], s["ctx"], prm, rho0, v0)
    fresh.load(state)
    X2 = X_saved.clone()
    rep2, eig2 = fresh.step(X2, W)
    rho_b = torch.zeros_like(rho_a)
    fresh.fields(rho_b)
    assert rep2.step == rep.step == 4
    assert rep2.energy == rep.energy and rep2.sre_ry == rep.sre_ry
    assert np.array_equal(eig, eig2)
    assert torch.equal(X, X2) and torch.equal(rho_a, rho_b)

    # a state from another mixing history or a truncated buffer is refused
    other = B.Scf(s["Hg"], s["ctx"], B.ScfParams(ne, M, 10, 4, 1, 10, B.CHF_F64, B.CHF_F64, 5, 0.3, 1e-12, eii),
                  rho0, v0)
    with pytest.raises(B.ChfError):
        other.load(state)
    with pytest.raises(B.ChfError):
        fresh.load(state[:-1])


def test_run_writes_one_json_record_per_step(tmp_path):
    """The SCF driver's trace: one JSON object per step with the step report
    and its wall time."""
    import json
    from paper_2303_00790_amd import scf as S
    c = make_cluster(5.5, 1001)
    st = S.setup(c, OH.PseudoParams(), h=0.7, dtype="f64", degree=10)
    rho = st["H"].sad_density(c.pos, c.species, c.n_electrons)
    path = tmp_path / "scf_trace.jsonl"
    res = S.run(st, rho, max_steps=3, sre_tol_ry=0.0, trace=str(path))
    recs = [json.loads(line) for line in path.read_text().splitlines()]
    assert res.steps == 3 and [r["step"] for r in recs] == [1, 2, 3]
    for r in recs:
        assert r["seconds"] > 0 and math.isfinite(r["energy"]) and r["sre_ry"] > 0
        assert r["chfsi_iters"] == (4 if r["step"] == 1 else 1)
        assert r["bound_a0"] < r["bound_a"] < r["bound_b"]
