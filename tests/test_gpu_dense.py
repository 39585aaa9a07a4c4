"""GPU parity of the dense ChFSI steps (Gram products, Lanczos bound,
Cholesky-QR, Rayleigh-Ritz, one full ChFSI iteration) against the FP64
oracle, through the C ABI.

Tolerances: FP64 Gram 1e-13 relative (the products are exact dot products in
a different summation order); FP32 Gram 2e-6 of n (the scale of the diagonal):
FP32 accumulation within row slices of about 4100-5000 rows here,
eps_32 * sqrt(R) ~ 4e-6 random-walk relative error per slice sum, the slice
partials added in FP64 (for the 70000-row case 17 slices, averaging the
slice errors down by ~sqrt(17)).  Eigenvalues from FP64 paths 1e-10 Ha.
"""
import numpy as np
import pytest

from oracle import chfsi as OC
from synth.cluster import random_block

from gpu_system import build, from_rows, relerr, to_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def system():
    s = build()
    s["ctx"] = s["B"].Context(0)
    return s


@pytest.mark.parametrize("n,m,k,same", [(5003, 70, 45, False), (4000, 130, 130, True), (100000, 64, 64, True),
                                        (300, 17, 3, False)])
def test_gram_f64(system, n, m, k, same):
    B = system["B"]
    rng = np.random.default_rng(n + m)
    A = rng.standard_normal((n, m))
    Bm = A if same else rng.standard_normal((n, k))
    At = torch.from_numpy(A).cuda()
    Bt = At if same else torch.from_numpy(Bm).cuda()
    S = torch.zeros((m, Bm.shape[1]), dtype=torch.float64, device="cuda")
    B.gram(system["ctx"], At, Bt, S)
    assert relerr(S.cpu().numpy(), A.T @ Bm) < 1e-13


@pytest.mark.parametrize("n,m", [(70000, 96), (5000, 33)])
def test_gram_f32(system, n, m):
    B = system["B"]
    rng = np.random.default_rng(5)
    A32 = rng.standard_normal((n, m)).astype(np.float32)
    At = torch.from_numpy(A32).cuda()
    S = torch.zeros((m, m), dtype=torch.float64, device="cuda")
    B.gram(system["ctx"], At, At, S)
    ref = A32.astype(np.float64).T @ A32.astype(np.float64)
    assert float(np.abs(S.cpu().numpy() - ref).max() / n) < 2e-6
    assert np.array_equal(S.cpu().numpy(), S.cpu().numpy().T)


def test_gram_f32_wide_block_norms_unbiased(system):
    """FP32 Gram of a wide block over many rows (1,048,576 x 8192, unit
    columns): the diagonal, the columns' squared norms, is what FP32
    Cholesky-QR leaves in the length of every column and so in the charge of
    the SCF density.  The FP32 MFMA sums of the BLAS kernels come out low by
    an amount that grows with the rows one sum runs over (measured on the
    MI355X: -8.6e-6 relative over ~284k-row slices, -3.6e-7 over 8192-row
    slices); the slices are kept short whatever the width, so the mean
    error of the diagonal stays below 1e-6 (a long-slice Gram fails)."""
    B = system["B"]
    n, m = 1 << 20, 8192
    print(f"case: FP32 Gram {n} x {m}", flush=True)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    X = torch.randn((n, m), generator=gen, dtype=torch.float32, device="cuda")
    true = torch.empty(m, dtype=torch.float64, device="cuda")
    for c in range(0, m, 512):
        true[c:c + 512] = (X[:, c:c + 512].double() ** 2).sum(0)
    X /= true.sqrt().float()[None, :]
    for c in range(0, m, 512):
        true[c:c + 512] = (X[:, c:c + 512].double() ** 2).sum(0)
    S = torch.empty((m, m), dtype=torch.float64, device="cuda")
    B.gram(system["ctx"], X, X, S)
    d = (torch.diagonal(S) - true).cpu().numpy()
    del X, S
    torch.cuda.empty_cache()
    print(f"diagonal error: mean {d.mean():.3e}, max |.| {np.abs(d).max():.3e}")
    assert abs(d.mean()) < 1e-6 and np.abs(d).max() < 3e-6


def test_lanczos_bound(system):
    s = system
    v0 = random_block(s["g"].n, 1, 3001)[:, 0]
    ref = OC.lanczos_bound(s["Ho"].apply, v0, 10)
    got = s["Hg"].lanczos_bound(s["ctx"], to_rows(s, v0, torch.float64), 10)
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_orthonormalize_f64(system):
    s = system
    X = random_block(s["g"].n, 96, 2400)
    Q, R = OC.cholesky_qr(X)
    Xg = to_rows(s, X, torch.float64)
    fb = s["B"].orthonormalize(s["ctx"], Xg)
    assert fb == 0
    assert relerr(from_rows(s, Xg, 96), Q) < 1e-11
    G = (Xg.T @ Xg).cpu().numpy()
    assert np.abs(G - np.eye(96)).max() < 1e-12
    pad = torch.ones(s["Hg"].n_rows, dtype=torch.bool, device="cuda")
    pad[s["rows"]] = False
    assert float(Xg[pad].abs().max()) == 0.0


def test_orthonormalize_f32(system):
    s = system
    X = random_block(s["g"].n, 64, 2401)
    Xg = to_rows(s, X, torch.float32)
    s["B"].orthonormalize(s["ctx"], Xg)
    G = (Xg.double().T @ Xg.double()).cpu().numpy()
    assert np.abs(G - np.eye(64)).max() < 5e-5


@pytest.fixture(scope="module")
def filtered_block(system):
    # a block as the SCF filters it: Ritz vectors after two oracle ChFSI
    # iterations, filtered with degree 12 between their own bounds; the
    # columns stay nearly orthogonal but their norms spread by |T_12(t0)|, a
    # condition number of ~1.4e2 (one FP32 Cholesky-QR pass would leave
    # kappa^2 u_32 ~ 1e-3 of orthogonality error)
    s = system
    v0 = random_block(s["g"].n, 1, 3001)[:, 0]
    b, tmin, _ = OC.lanczos_bound(s["Ho"].apply, v0)
    a0, a = tmin, tmin + 0.1 * (b - tmin)
    X = random_block(s["g"].n, 64, 2410)
    for _ in range(2):
        lam, X = OC.chfsi_iteration(s["Ho"].apply, X, 10, a, b, a0)
        a, a0 = lam[-1], lam[0]
    Y = OC.chebyshev_filter(s["Ho"].apply, X, 12, a, b, a0)
    return Y / np.abs(Y).max()


@pytest.mark.parametrize("gram_dtype", ["f32", "f64"])
def test_orthonormalize_f32_filtered_block_matches_oracle(system, filtered_block, gram_dtype):
    # FP32 Cholesky-QR (two passes) of a freshly filtered block against the
    # oracle's one exact pass on the same FP32-rounded block: Q of a full-rank
    # block is unique (positive diagonal of R), and the two-pass product of
    # triangular factors is again such an R.  Q moves by about kappa(X) times
    # the FP32 rounding of the block and of the updates (kappa here ~1.4e2),
    # so 2e-4 of max |Q|; orthonormality to 1e-6; the Ritz values of the FP32
    # Rayleigh-Ritz on the result against the oracle's within 2e-5 of the
    # spectrum's scale (the FP32 H X and Gram products).
    s = system
    B = s["B"]
    X32 = filtered_block.astype(np.float32).astype(np.float64)
    Q, _ = OC.cholesky_qr(X32)
    assert np.linalg.cond(X32) > 100
    Xg = to_rows(s, X32, torch.float32)
    fb = B.orthonormalize(s["ctx"], Xg, gram_dtype=B.CHF_F32 if gram_dtype == "f32" else B.CHF_F64)
    assert fb == 0
    got = from_rows(s, Xg, 64)
    assert relerr(got, Q) < 2e-4
    G = (Xg.double().T @ Xg.double()).cpu().numpy()
    assert np.abs(G - np.eye(64)).max() < 1e-6
    lam, _ = OC.rayleigh_ritz(s["Ho"].apply, Q)
    W = torch.zeros_like(Xg)
    eig = B.rayleigh_ritz(s["Hg"], s["ctx"], Xg, W)
    assert np.abs(eig - lam).max() < 2e-5 * max(1.0, np.abs(lam).max())


def test_orthonormalize_f32_retries_with_fp64_gram(system):
    # a column dependent on the others to ~3e-4 (pivot ratio ~1e-7, below what
    # an FP32 Gram resolves): the first pass is redone with an FP64 Gram
    # (one retry) and the result is orthonormal and spans the same columns
    s = system
    B = s["B"]
    X = random_block(s["g"].n, 32, 2411)
    X = X / np.abs(X).max()
    X[:, 7] = X[:, 3] + 3e-4 * X[:, 7]
    X32 = X.astype(np.float32).astype(np.float64)
    Xg = to_rows(s, X32, torch.float32)
    fb = B.orthonormalize(s["ctx"], Xg)
    assert fb == 1
    got = from_rows(s, Xg, 32)
    assert np.abs(got.T @ got - np.eye(32)).max() < 1e-6
    # span: X32 = got (got^T X32)
    assert relerr(got @ (got.T @ X32), X32) < 1e-5


def test_orthonormalize_rejects_fp64_block_with_fp32_gram(system):
    s = system
    B = s["B"]
    Xg = to_rows(s, random_block(s["g"].n, 8, 2412), torch.float64)
    with pytest.raises(B.ChfError) as e:
        B.orthonormalize(s["ctx"], Xg, gram_dtype=B.CHF_F32)
    assert e.value.code == -1


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_rayleigh_ritz_narrow_work_matches_full_width(system, dtype, tol):
    # W = H X in column blocks and X <- X Q in row panels through a work block
    # of 32 columns for 64 vectors: the same result as a full-width work block
    # up to the summation order of the products
    s = system
    X, _ = OC.cholesky_qr(random_block(s["g"].n, 64, 2413))
    Xa = to_rows(s, X, dtype)
    Xb = Xa.clone()
    ea = s["B"].rayleigh_ritz(s["Hg"], s["ctx"], Xa, torch.zeros_like(Xa))
    eb = s["B"].rayleigh_ritz(s["Hg"], s["ctx"], Xb, torch.zeros((s["Hg"].n_rows, 32), dtype=dtype, device="cuda"))
    assert np.abs(ea - eb).max() < tol * np.abs(ea).max()
    gaps = np.minimum(np.diff(ea, prepend=-np.inf), np.diff(ea, append=np.inf))
    ok = torch.from_numpy(gaps > 1e-6).cuda()
    da = Xa[:, ok].double()
    db = Xb[:, ok].double()
    sign = torch.sign((da * db).sum(0))
    assert float((da - db * sign).abs().max() / da.abs().max()) < (1e-10 if dtype == torch.float64 else 1e-3)


def test_rayleigh_ritz_rejects_more_vectors_than_grid_points():
    # a block wider than the grid cannot be orthonormal; the call refuses it
    # before any device work (it would also not fit the rotation's row panels
    # in a one-column work block)
    from paper_2303_00790_amd import binding as B
    from synth.workloads import MODEL_PP
    H = B.Hamiltonian(np.zeros((1, 3)), np.array([1], np.int32), MODEL_PP, 0.7, 2.5, B.ORDER_HILBERT)
    assert H.n_points < H.n_rows
    ctx = B.Context(0)
    X = torch.zeros((H.n_rows, H.n_points + 1), dtype=torch.float64, device="cuda")
    W = torch.zeros((H.n_rows, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(B.ChfError) as e:
        B.rayleigh_ritz(H, ctx, X, W)
    assert e.value.code == -1 and "grid points" in str(e.value)


def test_orthonormalize_rank_deficient_falls_back(system):
    s = system
    X = random_block(s["g"].n, 32, 2402)
    X[:, 5] = X[:, 4]                     # exactly dependent columns
    Xg = to_rows(s, X, torch.float64)
    try:
        fb = s["B"].orthonormalize(s["ctx"], Xg)
        assert fb == 1
    except s["B"].ChfError as e:
        assert e.code == -4


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 2e-5)])
def test_rayleigh_ritz(system, dtype, tol):
    s = system
    X, _ = OC.cholesky_qr(random_block(s["g"].n, 64, 2403))
    lam, Xr = OC.rayleigh_ritz(s["Ho"].apply, X)
    Xg = to_rows(s, X, dtype)
    W = torch.zeros_like(Xg)
    eig = s["B"].rayleigh_ritz(s["Hg"], s["ctx"], Xg, W)
    assert np.abs(eig - lam).max() < tol * max(1.0, np.abs(lam).max())
    if dtype == torch.float64:
        got = from_rows(s, Xg, 64)
        sign = np.sign((got * Xr).sum(0))
        gaps = np.minimum(np.diff(lam, prepend=-np.inf), np.diff(lam, append=np.inf))
        ok = gaps > 1e-6
        assert relerr((got * sign)[:, ok], Xr[:, ok]) < 1e-8


def test_chfsi_iteration_f64(system):
    s = system
    X = random_block(s["g"].n, 64, 2404)
    v0 = random_block(s["g"].n, 1, 3001)[:, 0]
    b, tmin, _ = OC.lanczos_bound(s["Ho"].apply, v0)
    a0, a = tmin, tmin + 0.1 * (b - tmin)
    Xo = X
    Xg = to_rows(s, X, torch.float64)
    W = torch.zeros_like(Xg)
    for _ in range(3):
        lam, Xo = OC.chfsi_iteration(s["Ho"].apply, Xo, 10, a, b, a0)
        s["Hg"].filter(Xg, W, 10, a, b, a0)
        s["B"].orthonormalize(s["ctx"], Xg)
        eig = s["B"].rayleigh_ritz(s["Hg"], s["ctx"], Xg, W)
        assert np.abs(eig - lam).max() < 1e-9
        a, a0 = lam[-1], lam[0]


def test_reserved_workspace_makes_later_calls_allocation_free(system):
    """After chf_reserve for an operation, calling it at that size allocates
    no device memory in the library (the counter of its allocations stays)."""
    s = system
    B = s["B"]
    H = s["Hg"]
    ctx = B.Context(0)
    X = to_rows(s, random_block(s["g"].n, 48, 2403), torch.float64)
    W = torch.zeros_like(X)
    v0 = to_rows(s, random_block(s["g"].n, 1, 3003)[:, 0], torch.float64)
    # the query is consistent and non-trivial
    hb, cb = B.workspace_bytes(H, B.WS_ORTHONORMALIZE, B.CHF_F64, 48)
    assert hb == 0 and cb >= 48 * 48 * 12
    hb, cb = B.workspace_bytes(H, B.WS_FILTER, B.CHF_F64, 48)
    assert hb >= 4 * H.n_proj * 48 * 8 and cb == 0
    with pytest.raises(B.ChfError):
        B.workspace_bytes(H, 7, B.CHF_F64, 48)
    for op, ldw in ((B.WS_FILTER, 0), (B.WS_ORTHONORMALIZE, 0), (B.WS_RAYLEIGH_RITZ, 48), (B.WS_LANCZOS, 0)):
        B.reserve(H, ctx, op, B.CHF_F64, 48, ldw)
    before = B.device_allocations()
    b, tmin, _ = H.lanczos_bound(ctx, v0, 10)
    H.apply(X, W)
    H.filter(X, W, 4, tmin + 0.1 * (b - tmin), b, tmin - 1.0)
    B.orthonormalize(ctx, X)
    B.rayleigh_ritz(H, ctx, X, W)
    torch.cuda.synchronize()
    assert B.device_allocations() == before


def test_absurd_reservation_reports_out_of_memory(system):
    """A workspace far beyond the device (2^30 FP64 vectors of KB
    coefficients) fails with CHF_ENOMEM and leaves the handle usable."""
    s = system
    B = s["B"]
    with pytest.raises(B.ChfError) as e:
        B.reserve(s["Hg"], None, B.WS_FILTER, B.CHF_F64, 1 << 30)
    assert e.value.code == -2
    X = to_rows(s, random_block(s["g"].n, 8, 2404), torch.float64)
    Y = torch.zeros_like(X)
    s["Hg"].apply(X, Y)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(Y).all())
