"""GPU parity of the density network against the FP64 oracle.

The device runs BF16 weights and activations into MFMA with FP32
accumulation; the oracle runs FP64 on the same BF16-rounded weights and
input.  Between layers the device rounds activations to BF16 (relative
2^-8 per layer, ~21 layers), so forward outputs and gradients are compared
at 3e-2 relative to their largest magnitude; the Adam update is compared
exactly (same FP32 gradients on both sides, 1e-5).
"""
import numpy as np
import pytest

from oracle import unet as U

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def bf16_round(a):
    a32 = np.asarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def to_oracle(net, flat):
    p = {}
    for name, (info, off) in net.layers.items():
        cin, cout, cin_p, cout_p, k, _ = info
        ntap = k ** 3
        w = flat[off[0]:off[0] + cout_p * ntap * cin_p].reshape(cout_p, ntap, cin_p)[:cout, :, :cin]
        p[name + ".w"] = w.transpose(0, 2, 1).reshape(cout, cin, k, k, k).astype(np.float64)
        p[name + ".b"] = flat[off[1]:off[1] + cout].astype(np.float64)
    return p


def from_oracle_grad(net, g):
    flat = np.zeros(net.n_params, np.float64)
    for name, (info, off) in net.layers.items():
        cin, cout, cin_p, cout_p, k, _ = info
        ntap = k ** 3
        w = np.zeros((cout_p, ntap, cin_p))
        w[:cout, :, :cin] = g[name + ".w"].reshape(cout, cin, ntap).transpose(0, 2, 1)
        flat[off[0]:off[0] + w.size] = w.ravel()
        flat[off[1]:off[1] + cout] = g[name + ".b"]
    return flat


def _net_case(C, S):
    from paper_2303_00790_amd import binding as B
    net = B.DensityNet(C, seed=3)
    flat = net.get_params()
    rng = np.random.default_rng(9)
    info, off = net.layers["out"]
    flat[off[0]:off[0] + info[2] * 1] = rng.standard_normal(info[2]).astype(np.float32) * 0.3   # row 0 of out.w
    flat[off[1]] = 0.1
    # store BF16-exact master weights so both sides see identical values
    flat = bf16_round(flat).astype(np.float32)
    net.set_params(flat)
    x = bf16_round(np.abs(rng.standard_normal((S, S, S))) + 0.2)
    t = rng.standard_normal((S, S, S)) * 0.1
    return B, net, flat, x, t, S


@pytest.fixture(scope="module")
def net_case():
    return _net_case(8, 16)


def _check_forward_and_gradients(case):
    B, net, flat, x, t, S = case
    p = to_oracle(net, flat)
    y_ref, tape = U.forward(p, x[None], keep=True)
    loss_ref, dy_ref = U.mse(y_ref, t[None])
    g_ref = from_oracle_grad(net, U.backward(p, tape, dy_ref))
    xg = torch.from_numpy(x.astype(np.float32)).cuda()
    tg = torch.from_numpy(t.astype(np.float32)).cuda()
    yg = torch.zeros_like(xg)
    dy = torch.zeros_like(xg)
    net.forward(xg, yg)
    loss = net.mse(yg, tg, dy)
    net.backward(dy)
    y = yg.cpu().numpy()
    assert np.abs(y - y_ref[0]).max() < 3e-2 * np.abs(y_ref).max()
    assert abs(loss - loss_ref) < 3e-2 * loss_ref
    g = net.get_grads().astype(np.float64)
    for name, (info, off) in net.layers.items():
        cin, cout, cin_p, cout_p, k, _ = info
        sl = slice(off[0], off[0] + cout_p * k ** 3 * cin_p)
        ref = g_ref[sl]
        assert np.abs(g[sl] - ref).max() < 3e-2 * np.abs(ref).max() + 1e-12, name
        bs = slice(off[1], off[1] + cout)
        assert np.abs(g[bs] - g_ref[bs]).max() < 3e-2 * np.abs(g_ref[bs]).max() + 1e-12, name


def test_forward_and_gradients(net_case):
    _check_forward_and_gradients(net_case)


def test_forward_and_gradients_trained_width():
    # the configuration the network is trained in: 32 channels (the 64-channel
    # concatenations of the decoder go through the multi-row-block paths of
    # the forward, input-gradient and weight-gradient kernels) on a 32^3
    # patch (4^3 bottleneck); every layer's weight and bias gradient is
    # compared, which checks the input gradients of all layers after it
    case = _net_case(32, 32)
    _check_forward_and_gradients(case)


def test_adam_matches_oracle(net_case):
    B, net, flat, x, t, S = net_case
    w0 = net.get_params().astype(np.float64)
    g = net.get_grads().astype(np.float64)
    net.adam(1e-3, 1)
    w1 = net.get_params().astype(np.float64)
    pd, gd = {"w": w0.copy()}, {"w": g}
    U.adam_step(pd, gd, {"w": np.zeros_like(w0)}, {"w": np.zeros_like(w0)}, 1, lr=1e-3)
    assert np.abs(w1 - pd["w"]).max() < 1e-5
    assert not net.get_grads().any()


def test_training_reduces_loss(net_case):
    B, net, flat, x, t, S = net_case
    xg = torch.from_numpy(x.astype(np.float32)).cuda()
    tg = torch.from_numpy((0.05 * x).astype(np.float32)).cuda()
    yg = torch.zeros_like(xg)
    dy = torch.zeros_like(xg)
    losses = []
    for step in range(1, 31):
        net.forward(xg, yg)
        losses.append(net.mse(yg, tg, dy))
        net.backward(dy)
        net.adam(3e-3, step)
    assert losses[-1] < 0.5 * losses[0]


def test_crop_symmetries():
    from paper_2303_00790_amd import binding as B
    D, S = 10, 4
    box = torch.arange(D ** 3, dtype=torch.float32, device="cuda")
    seen = set()
    for sym in range(48):
        patch = torch.zeros(S ** 3, dtype=torch.float32, device="cuda")
        B.crop(box, D, S, (2, 3, 1), sym, patch)
        vals = patch.cpu().numpy().reshape(S, S, S)
        ref = box.cpu().numpy().reshape(D, D, D)[1:1 + S, 3:3 + S, 2:2 + S]
        assert sorted(vals.ravel()) == sorted(ref.ravel())
        seen.add(vals.tobytes())
    assert len(seen) == 48


def test_highpass_matches_oracle():
    from paper_2303_00790_amd import binding as B
    D, sigma = 24, 2.5
    rng = np.random.default_rng(4)
    box = rng.standard_normal((D, D, D)).astype(np.float32)
    ref = U.gaussian_highpass(box.astype(np.float64), sigma)
    bg = torch.from_numpy(box.ravel()).cuda()
    out = torch.zeros_like(bg)
    work = torch.zeros(2 * D ** 3, dtype=torch.float32, device="cuda")
    B.highpass(bg, D, sigma, out, work)
    got = out.cpu().numpy().reshape(D, D, D)   # z, y, x with x fastest: the oracle array's axes in the same order
    assert np.abs(got - ref).max() < 1e-5 * np.abs(ref).max()


@pytest.fixture(scope="module")
def grid_system():
    from gpu_system import build
    return build()


def test_rows_box_round_trip(grid_system):
    # rows -> box places grid point (i, j, k) at cell (i, j, k) + off of a
    # D^3 box, x fastest, scaled; box -> rows reads it back (FP32 box)
    from paper_2303_00790_amd import binding as B
    from paper_2303_00790_amd import density_model as DM
    s = grid_system
    H = s["Hg"]
    D, off = DM.box_geometry(H)
    rng = np.random.default_rng(5)
    vals = rng.uniform(0.0, 0.05, s["g"].n)
    rows = torch.zeros(H.n_rows, dtype=torch.float64, device="cuda")
    rows[s["rows"]] = torch.from_numpy(vals).cuda()
    box = torch.full((D ** 3,), float("nan"), dtype=torch.float32, device="cuda")
    B.rows_to_box(H, rows, 30.0, box, D, off)
    b = box.cpu().numpy().reshape(D, D, D)
    ijk = s["g"].ijk + off
    assert np.allclose(b[ijk[:, 2], ijk[:, 1], ijk[:, 0]], (30.0 * vals).astype(np.float32), rtol=0, atol=0)
    assert np.count_nonzero(b) == np.count_nonzero(vals)
    # with a base, the box holds the scaled difference taken in FP64
    base = torch.zeros_like(rows)
    base[s["rows"]] = torch.from_numpy(vals[::-1].copy()).cuda()
    boxd = torch.full((D ** 3,), float("nan"), dtype=torch.float32, device="cuda")
    B.rows_to_box(H, rows, 30.0, boxd, D, off, base=base)
    bd = boxd.cpu().numpy().reshape(D, D, D)
    assert np.allclose(bd[ijk[:, 2], ijk[:, 1], ijk[:, 0]], (30.0 * (vals - vals[::-1])).astype(np.float32), rtol=0,
                       atol=0)
    back = torch.full_like(rows, float("nan"))
    B.box_to_rows(H, box, D, off, 30.0, None, back)
    got = back.cpu().numpy()
    assert np.abs(got[s["g"].row_of_rank] - vals).max() < 1e-7 * vals.max()
    pad = np.ones(H.n_rows, bool)
    pad[s["g"].row_of_rank] = False
    assert not got[pad].any()


def test_density_fix_clamps_and_renormalises(grid_system):
    # rho <- max(rho, 0) * N_e / (h^3 sum max(rho, 0)) on the inside rows
    s = grid_system
    H = s["Hg"]
    rng = np.random.default_rng(6)
    vals = rng.normal(0.01, 0.02, s["g"].n)
    rows = torch.zeros(H.n_rows, dtype=torch.float64, device="cuda")
    rows[s["rows"]] = torch.from_numpy(vals).cuda()
    ne = 176
    H.density_fix(rows, ne)
    ref = np.maximum(vals, 0.0)
    ref *= ne / (0.7 ** 3 * ref.sum())
    got = rows.cpu().numpy()[s["g"].row_of_rank]
    assert np.abs(got - ref).max() < 1e-13 * ref.max()
