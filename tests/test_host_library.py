"""Host-side checks of the C-ABI library (no GPU): it loads, exports every
symbol the header declares, and its host-built ordering, neighbour and
projector tables equal the oracle's bit for bit."""
import math
import os
import re

import numpy as np
import pytest

from oracle import grid as G
from oracle import hamiltonian as OH
from synth.cluster import make_cluster

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
B = pytest.importorskip("paper_2303_00790_amd.binding")

if not os.path.exists(B.LIB_PATH):
    pytest.skip("libchfsi.so not built", allow_module_level=True)


def _header_symbols():
    text = open(os.path.join(ROOT, "include", "chfsi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    import ctypes
    lib = ctypes.CDLL(B.LIB_PATH)
    names = _header_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares exactly the header's calls
    assert sorted(B.declared_symbols()) == names


def test_error_path_sets_message():
    import ctypes
    g = B.GridDesc(-1.0, 5.0, 0, 0, 3)
    n, nr = ctypes.c_int64(), ctypes.c_int64()
    rc = B.lib().chf_ordering_host(ctypes.byref(g), ctypes.byref(n), ctypes.byref(nr), None, None, None)
    assert rc == -1 and b"bad grid" in B.lib().chf_last_error()


@pytest.mark.parametrize("radius,h,ordering", [(18.0935, 0.7, G.ORDER_HILBERT), (18.0935, 0.7, G.ORDER_LEX),
                                               (9.3, 0.45, G.ORDER_HILBERT), (5.61, 1.0, G.ORDER_HILBERT),
                                               (12.0, 0.6, G.ORDER_LEX)])
def test_ordering_bit_exact(radius, h, ordering):
    ijk, rows, nbr, n_rows = B.ordering_host(h, radius, ordering)
    g = G.build_grid(radius, h, ordering)
    assert np.array_equal(ijk, g.ijk)
    assert np.array_equal(rows, g.row_of_rank)
    assert n_rows == g.n_rows
    assert np.array_equal(nbr, G.neighbour_table(g))


def test_ordering_random_radii():
    rng = np.random.default_rng(11)
    for _ in range(6):
        h = float(rng.uniform(0.5, 1.0))
        radius = float(rng.uniform(3.0, 12.0))
        ijk, rows, _, n_rows = B.ordering_host(h, radius, G.ORDER_HILBERT, with_nbr=False)
        g = G.build_grid(radius, h)
        assert np.array_equal(ijk, g.ijk) and np.array_equal(rows, g.row_of_rank) and n_rows == g.n_rows


def test_projector_tables_match_oracle():
    c = make_cluster(5.5, 1001)
    radius = c.domain_radius()
    pp = OH.PseudoParams()
    off, rank, beta = B.projectors_host(0.7, radius, c.pos, c.species, pp)
    g = G.build_grid(radius, 0.7)
    Bm, _ = OH.projector_matrix(g, c.pos, c.species, pp)
    Bm = Bm.tocsc()
    assert len(off) == Bm.shape[1] // 4 + 1
    for a in range(len(off) - 1):
        col = Bm[:, 4 * a:4 * a + 4].tocoo()
        rows_o = np.unique(col.row)
        assert np.array_equal(rank[off[a]:off[a + 1]], rows_o)
        dense = Bm[rows_o, 4 * a:4 * a + 4].toarray()
        assert np.allclose(beta[off[a]:off[a + 1]], dense, rtol=1e-14, atol=1e-17)


def test_density_net_plan_matches_architecture():
    # every layer's input edge must equal its producer's output edge
    # (stride-2 layers halve, upsampling doubles); the oracle's forward pass
    # gives the reference edges
    import numpy as np
    from oracle import unet as U
    S = 16
    edges = B.dnet_plan(S)
    p = U.init_params(C=4, seed=0)
    _, tape = U.forward(p, np.zeros((1, S, S, S)), keep=True)
    ref = {name: z.shape[1] for name, _, z, _, _ in tape}
    assert edges == [ref[name] for name in B.LAYER_NAMES]


# Calls that accept null handles by design: destroy calls are no-ops on null, the
# timer switch and the allocation counter take no pointer, and chf_last_error reads.
NULL_OK = {"chf_ctx_destroy", "ham_destroy", "chf_scf_destroy", "dnet_destroy", "chf_timer",
           "chf_device_allocations", "chf_last_error"}


def test_every_call_rejects_null_arguments_on_the_host():
    """Every entry point validates its pointers before any device work: with
    null pointers (and unit scalars) it returns CHF_EINVAL and leaves a message
    that names the call.  Runs without a GPU, so a call that reached the
    device first would fail here instead."""
    import ctypes
    lib = B.lib()
    for name in B.declared_symbols():
        if name in NULL_OK:
            continue
        f = getattr(lib, name)
        args = []
        for t in f.argtypes:
            if t in (ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t):
                args.append(t(1))
            elif t in (ctypes.c_double, ctypes.c_float):
                args.append(t(1.0))
            else:
                args.append(None)
        rc = f(*args)
        msg = lib.chf_last_error().decode()
        assert B.STATUS.get(rc) == "CHF_EINVAL", (name, rc, msg)
        assert msg.startswith(name), (name, msg)


def test_ion_energy_matches_oracle_on_the_host():
    # the ion-ion energy is host code: a 3 nm cluster (1,005 atoms) against the oracle's pair sum
    from oracle import scf as OS
    from synth.workloads import MODEL_PP
    c = make_cluster(15.0, 2)
    got = B.ion_energy(c.pos, c.species, MODEL_PP)
    want = OS.ion_energy(c.pos, np.where(c.species == 0, MODEL_PP.z_si, MODEL_PP.z_h).astype(float))
    assert abs(got - want) < 1e-12 * abs(want)


@pytest.mark.parametrize("radius,h", [
    (math.sqrt(50.0) * 0.7, 0.7),    # radius on a lattice shell: the 1e-9 tolerance decides membership
    (math.sqrt(27.0) * 0.9, 0.9),
    (12.0, 1.0), (16.0, 1.0),        # 4 and 5 blocks per edge: Hilbert order 2 then 3
    (28.0, 1.0), (32.0, 1.0),        # 8 and 9 blocks per edge: order 3 then 4
    (1.0001, 1.0),                   # the smallest grid: the centre and its 6 neighbours
])
def test_ordering_edge_radii(radius, h):
    ijk, rows, nbr, n_rows = B.ordering_host(h, radius, G.ORDER_HILBERT)
    g = G.build_grid(radius, h)
    assert np.array_equal(ijk, g.ijk) and np.array_equal(rows, g.row_of_rank) and n_rows == g.n_rows
    assert np.array_equal(nbr, G.neighbour_table(g))
    if radius < 2 * h:
        # the centre sees all six; each outer point sees the centre and the opposite point on its axis
        assert len(ijk) == 7 and (nbr >= 0).sum() == 6 + 6 * 2


def _projector_parity(h, radius, pos, species, pp):
    off, rank, beta = B.projectors_host(h, radius, pos, species, pp)
    g = G.build_grid(radius, h)
    Bm, _ = OH.projector_matrix(g, pos, species, pp)
    Bm = Bm.tocsc()
    assert len(off) == Bm.shape[1] // 4 + 1 and off[-1] == len(rank)
    for a in range(len(off) - 1):
        rows_o = np.unique(Bm[:, 4 * a:4 * a + 4].tocoo().row)
        assert np.array_equal(rank[off[a]:off[a + 1]], rows_o)
        assert np.allclose(beta[off[a]:off[a + 1]], Bm[rows_o, 4 * a:4 * a + 4].toarray(), rtol=1e-14, atol=1e-17)
    return off, rank, beta


def test_projector_tables_edge_cases():
    pp = OH.PseudoParams()
    radius, h = 9.0, 0.7
    # a Si on a grid point (the p channels vanish there), one whose support the sphere cuts,
    # one wholly outside the support of the others, and an H (no projectors)
    pos = np.array([[0.0, 0.0, 0.0], [7.7, 0.3, -0.2], [-3.1, 4.4, 2.0], [0.0, 0.0, 1.5]])
    species = np.array([0, 0, 0, 1], np.int32)
    off, rank, beta = _projector_parity(h, radius, pos, species, pp)
    assert len(off) == 4
    full = off[1] - off[0]
    assert off[2] - off[1] < full          # the cut atom keeps fewer support points
    # H only, and no atoms at all: no projector entries
    off, rank, _ = _projector_parity(h, radius, pos[3:], species[3:], pp)
    assert list(off) == [0] and len(rank) == 0
    off, rank, _ = _projector_parity(h, radius, np.zeros((0, 3)), np.zeros(0, np.int32), pp)
    assert list(off) == [0] and len(rank) == 0
