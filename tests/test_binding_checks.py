"""The Python binding's argument checks, on the CPU.

The library receives only pointers and leading dimensions, so the binding
checks the extent each call will touch (rows of the Hamiltonian, vector
count, FP64 vector lengths), matching dtypes and device memory before it
calls.  Here the C call, the stream lookup and the device check are replaced
by stand-ins: the shapes the GPU tests use must pass, and every malformed
argument must raise before anything reaches the library."""
import types

import pytest
import torch

B = pytest.importorskip("paper_2303_00790_amd.binding")

N_ROWS = 1024


@pytest.fixture
def fake(monkeypatch):
    calls = []
    monkeypatch.setattr(B, "call", lambda name, *args: calls.append(name))
    monkeypatch.setattr(B, "_on_gpu", lambda t, what: None)
    monkeypatch.setattr(B, "_stream", lambda: None)
    H = B.Hamiltonian.__new__(B.Hamiltonian)
    H.handle = None
    H.n_rows, H.n_points = N_ROWS, 900
    ctx = types.SimpleNamespace(handle=None)
    return H, ctx, calls


def blk(rows=N_ROWS, cols=8, dtype=torch.float64):
    return torch.zeros((rows, cols), dtype=dtype)


def vec(n=N_ROWS, dtype=torch.float64):
    return torch.zeros(n, dtype=dtype)


def test_shapes_the_device_tests_use_are_accepted(fake):
    H, ctx, calls = fake
    X = blk(cols=40)
    H.apply(X, torch.empty_like(X))
    H.apply(X[:, :36], torch.full_like(X, 0.0)[:, :36])      # column views with ld > nvec
    H.filter(X, torch.zeros_like(X), 3, 0.0, 1.0, -1.0)
    H.filter(X, torch.zeros_like(X), 3, 0.0, 1.0, -1.0, nvec=33)
    H.density(X, 33, vec())
    H.hartree(ctx, vec(), vec())
    H.lda(vec(), vec(), vec())
    H.lda(vec(), None, vec())
    H.density_fix(vec(), 8)
    H.lanczos_bound(ctx, vec())
    H.set_veff(vec())
    B.gram(ctx, blk(5003, 70), blk(5003, 45), blk(70, 45))
    B.gram(ctx, blk(300, 17, torch.float32), blk(300, 17, torch.float32), blk(17, 17))
    B.orthonormalize(ctx, X)
    B.rayleigh_ritz(H, ctx, X, torch.zeros_like(X))
    assert calls.count("ham_apply") == 2 and "rayleigh_ritz" in calls and "gram" in calls


@pytest.mark.parametrize("case,err", [
    ("X rows short", ValueError),
    ("Y rows short", ValueError),
    ("Y dtype differs", TypeError),
    ("Y narrower than X", ValueError),
    ("X not 2-D", ValueError),
    ("X columns strided", ValueError),
    ("filter nvec too large", ValueError),
    ("filter work dtype differs", TypeError),
    ("density n_occ too large", ValueError),
    ("rho short", ValueError),
    ("rho FP32", TypeError),
    ("rho strided", ValueError),
    ("veff short", ValueError),
    ("v0 short", ValueError),
    ("gram B rows short", ValueError),
    ("gram S too small", ValueError),
    ("gram S FP32", TypeError),
    ("gram B dtype differs", TypeError),
    ("rayleigh-ritz work rows short", ValueError),
])
def test_malformed_arguments_raise_before_the_call(fake, case, err):
    H, ctx, calls = fake
    X = blk()
    run = {
        "X rows short": lambda: H.apply(blk(N_ROWS - 1), blk()),
        "Y rows short": lambda: H.apply(X, blk(N_ROWS - 1)),
        "Y dtype differs": lambda: H.apply(X, blk(dtype=torch.float32)),
        "Y narrower than X": lambda: H.apply(X, blk(cols=4)),
        "X not 2-D": lambda: H.apply(vec(), vec()),
        "X columns strided": lambda: H.apply(blk(cols=16)[:, ::2], blk()),
        "filter nvec too large": lambda: H.filter(X, blk(), 3, 0.0, 1.0, -1.0, nvec=9),
        "filter work dtype differs": lambda: H.filter(X, blk(dtype=torch.float32), 3, 0.0, 1.0, -1.0),
        "density n_occ too large": lambda: H.density(X, 9, vec()),
        "rho short": lambda: H.hartree(ctx, vec(N_ROWS - 1), vec()),
        "rho FP32": lambda: H.lda(vec(dtype=torch.float32), None, vec()),
        "rho strided": lambda: H.density_fix(vec(2 * N_ROWS)[::2], 8),
        "veff short": lambda: H.set_veff(vec(N_ROWS - 1)),
        "v0 short": lambda: H.lanczos_bound(ctx, vec(10)),
        "gram B rows short": lambda: B.gram(ctx, blk(100, 4), blk(99, 4), blk(4, 4)),
        "gram S too small": lambda: B.gram(ctx, blk(100, 4), blk(100, 5), blk(4, 4)),
        "gram S FP32": lambda: B.gram(ctx, blk(100, 4), blk(100, 4), blk(4, 4, torch.float32)),
        "gram B dtype differs": lambda: B.gram(ctx, blk(100, 4), blk(100, 4, torch.float32), blk(4, 4)),
        "rayleigh-ritz work rows short": lambda: B.rayleigh_ritz(H, ctx, X, blk(N_ROWS - 1)),
    }[case]
    with pytest.raises(err):
        run()
    assert calls == []


def test_scf_step_checks_precision_and_extent(fake):
    H, ctx, calls = fake
    scf = B.Scf.__new__(B.Scf)
    scf.handle = None
    scf.nvec, scf.n_rows, scf.filter_double = 8, N_ROWS, False
    scf.step(blk(dtype=torch.float32), blk(dtype=torch.float32))
    assert calls == ["scf_step"]
    with pytest.raises(TypeError):
        scf.step(blk(), blk())                                   # FP64 block for an FP32 filter
    with pytest.raises(ValueError):
        scf.step(blk(cols=7, dtype=torch.float32), blk(dtype=torch.float32))
    with pytest.raises(TypeError):
        scf.step(blk(dtype=torch.float32), blk())
    assert calls == ["scf_step"]


def test_host_tensors_are_refused(monkeypatch):
    # the real device check: a tensor in host memory never reaches the library
    monkeypatch.setattr(B, "call", lambda name, *args: pytest.fail("reached the library"))
    with pytest.raises(ValueError, match="GPU memory"):
        B._block(blk())
    with pytest.raises(ValueError, match="GPU memory"):
        B._vec(vec(), N_ROWS, "rho")


@pytest.fixture
def fake_net(fake):
    calls = fake[2]            # the stand-ins of `fake` record these calls too
    net = B.DensityNet.__new__(B.DensityNet)
    net.handle = None
    net.n_params = 100
    return net, calls


def f32(n):
    return torch.zeros(n, dtype=torch.float32)


def test_density_net_shapes_accepted(fake_net, fake):
    net, calls = fake_net
    H = fake[0]
    S, D = 16, 24
    import numpy as np
    net.set_params(np.zeros(100, np.float32))
    x = torch.zeros((S, S, S), dtype=torch.float32)
    net.forward(x, torch.zeros_like(x))
    net.mse(x, torch.zeros_like(x), torch.zeros_like(x))
    net.backward(torch.zeros_like(x))
    B.crop(f32(D ** 3), D, S, (1, 2, 3), 5, f32(S ** 3))
    B.highpass(f32(D ** 3), D, 8.0, f32(D ** 3), f32(2 * D ** 3))
    B.rows_to_box(H, vec(), 30.0, f32(D ** 3), D, 3)
    B.box_to_rows(H, f32(D ** 3), D, 3, 30.0, None, vec())
    B.box_to_rows(H, f32(D ** 3), D, 3, 30.0, vec(), vec())
    assert calls[:4] == ["dnet_set_params", "dnet_forward", "dnet_mse", "dnet_backward"]
    # inference and training pass flat boxes and patches; every cube edge up to 256 is recovered
    # from the value count
    for edge in range(1, 257):
        net.forward(f32(edge ** 3), f32(edge ** 3))
        assert net._n_out == edge ** 3


@pytest.mark.parametrize("case", ["params short", "x not a cube", "y short", "dy short", "t short", "crop box short",
                                  "crop patch short", "highpass work short", "rows_to_box rows short",
                                  "box_to_rows box short", "box_to_rows out FP32"])
def test_density_net_malformed_arguments_raise(fake_net, fake, case):
    import numpy as np
    net, calls = fake_net
    H = fake[0]
    S, D = 16, 24
    net._n_out = S ** 3
    run = {
        "params short": lambda: net.set_params(np.zeros(99, np.float32)),
        "x not a cube": lambda: net.forward(f32(S ** 3 + 1), f32(S ** 3 + 1)),
        "y short": lambda: net.forward(f32(S ** 3), f32(S ** 3 - 1)),
        "dy short": lambda: net.backward(f32(S ** 3 - 1)),
        "t short": lambda: net.mse(f32(S ** 3), f32(S ** 3 - 1)),
        "crop box short": lambda: B.crop(f32(D ** 3 - 1), D, S, (0, 0, 0), 0, f32(S ** 3)),
        "crop patch short": lambda: B.crop(f32(D ** 3), D, S, (0, 0, 0), 0, f32(S ** 3 - 1)),
        "highpass work short": lambda: B.highpass(f32(D ** 3), D, 8.0, f32(D ** 3), f32(D ** 3)),
        "rows_to_box rows short": lambda: B.rows_to_box(H, vec(N_ROWS - 1), 1.0, f32(D ** 3), D, 0),
        "box_to_rows box short": lambda: B.box_to_rows(H, f32(D ** 3 - 1), D, 0, 1.0, None, vec()),
        "box_to_rows out FP32": lambda: B.box_to_rows(H, f32(D ** 3), D, 0, 1.0, None, vec(dtype=torch.float32)),
    }[case]
    with pytest.raises((ValueError, TypeError)):
        run()
    assert calls == []


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # no fallback: without the built library every call raises
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "libchfsi.so"))
    monkeypatch.setattr(B, "_stream", lambda: None)     # this host has no GPU to ask for a stream
    with pytest.raises(RuntimeError, match="not built"):
        B.lib()
    with pytest.raises(RuntimeError, match="not built"):
        B.Hamiltonian(torch.zeros((1, 3), dtype=torch.float64).numpy(), [0], types.SimpleNamespace(
            z_si=4.0, z_h=1.0, r_loc=0.7, r_loc_h=0.5, r_c=1.2, r_cut=4.8, h_s=3.0, h_p=0.0), 0.7, 5.0)
