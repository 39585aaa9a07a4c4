"""ctypes binding of libchfsi.so: argument marshalling only.

Every computation happens inside the HIP library; PyTorch only provides
device memory (tensors) and the current HIP stream.  If the library has not
been built this module raises on first use -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchfsi.so")

CHF_F32, CHF_F64 = 1, 2
ORDER_HILBERT, ORDER_LEX = 0, 1
STATUS = {0: "CHF_OK", -1: "CHF_EINVAL", -2: "CHF_ENOMEM", -3: "CHF_EHIP", -4: "CHF_ENOTPD",
          -5: "CHF_ENOTCONV", -6: "CHF_ENONFINITE", -7: "CHF_EUNSUPPORTED"}


class ChfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [("h", C.c_double), ("radius", C.c_double), ("ordering", C.c_int), ("keep_nbr", C.c_int),
                ("dtypes", C.c_int)]


class Atoms(C.Structure):
    _fields_ = [("n_atoms", C.c_int), ("pos_host", C.POINTER(C.c_double)), ("species_host", C.POINTER(C.c_int))]


class PP(C.Structure):
    _fields_ = [("z_si", C.c_double), ("z_h", C.c_double), ("r_loc_si", C.c_double), ("r_loc_h", C.c_double),
                ("r_c", C.c_double), ("r_cut", C.c_double), ("h_s", C.c_double), ("h_p", C.c_double)]


class ScfParams(C.Structure):
    _fields_ = [("n_electrons", C.c_int), ("nvec", C.c_int), ("degree", C.c_int), ("first_iters", C.c_int),
                ("later_iters", C.c_int), ("lanczos_k", C.c_int), ("filter_dtype", C.c_int),
                ("gram_dtype", C.c_int), ("mix_history", C.c_int), ("mix_beta", C.c_double),
                ("cg_rtol", C.c_double), ("e_ion", C.c_double)]


class ScfReport(C.Structure):
    _fields_ = [("step", C.c_int), ("chfsi_iters", C.c_int), ("cg_iters", C.c_int), ("chol_fallbacks", C.c_int),
                ("sre_ry", C.c_double), ("energy", C.c_double), ("band_energy", C.c_double),
                ("homo", C.c_double), ("lumo", C.c_double), ("bound_a", C.c_double), ("bound_b", C.c_double),
                ("bound_a0", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


P = C.c_void_p
I64 = C.c_int64
D = C.c_double
INT = C.c_int

# name -> argtypes (all return int status except chf_last_error)
_SIGS = {
    "chf_ctx_create": [INT, C.POINTER(P)],
    "chf_ctx_destroy": [P],
    "ham_build": [C.POINTER(GridDesc), C.POINTER(Atoms), C.POINTER(PP), P, C.POINTER(P)],
    "chf_ordering_host": [C.POINTER(GridDesc), C.POINTER(I64), C.POINTER(I64), P, P, P],
    "chf_projectors_host": [C.POINTER(GridDesc), C.POINTER(Atoms), C.POINTER(PP), C.POINTER(I64), P, P, P],
    "ham_destroy": [P],
    "ham_info": [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64), C.POINTER(I64), C.POINTER(I64)],
    "ham_export_ordering": [P, P, P, P],
    "ham_get_vloc": [P, P, P],
    "ham_set_veff": [P, P, P],
    "ham_apply": [P, INT, P, I64, P, I64, INT, P],
    "chf_ham_apply_generic": [P, INT, P, I64, P, I64, INT, P],
    "chebyshev_filter": [P, INT, P, I64, INT, INT, D, D, D, P, I64, P],
    "chf_filter_generic": [P, INT, P, I64, INT, INT, D, D, D, P, I64, P],
    "chebyshev_filter_noalloc": [P, INT, P, I64, INT, INT, D, D, D, P, I64, P],
    "lanczos_bound": [P, P, P, INT, P, P],
    "chf_timer": [INT],
    "chf_timer_read": [P, P],
    "gram": [P, INT, P, I64, P, I64, I64, INT, INT, P, I64, P],
    "orthonormalize": [P, INT, P, I64, I64, INT, INT, P, P],
    "rayleigh_ritz": [P, P, INT, P, I64, INT, P, P, I64, P],
    "chf_density": [P, INT, P, I64, INT, P, P],
    "chf_hartree": [P, P, P, P, D, INT, P, P],
    "chf_lda": [P, P, P, P, P],
    "chf_sad_density": [P, C.POINTER(Atoms), D, D, INT, P, P],
    "chf_ion_energy": [C.POINTER(Atoms), C.POINTER(PP), C.POINTER(D)],
    "chf_density_fix": [P, P, INT, P],
    "chf_scf_create": [P, P, C.POINTER(ScfParams), P, P, C.POINTER(P)],
    "chf_scf_destroy": [P],
    "scf_step": [P, P, I64, P, I64, C.POINTER(ScfReport), P],
    "chf_scf_get_fields": [P, P, P],
    "chf_workspace_bytes": [P, INT, INT, INT, I64, P, P],
    "chf_reserve": [P, P, INT, INT, INT, I64],
    "chf_scf_state_size": [P, P],
    "chf_scf_save": [P, P],
    "chf_scf_load": [P, P, I64],
    "dnet_create": [INT, C.c_uint64, C.POINTER(P)],
    "dnet_destroy": [P],
    "dnet_param_count": [P, C.POINTER(I64)],
    "dnet_layer_info": [P, INT, P, P],
    "dnet_plan": [INT, P],
    "dnet_get_params": [P, P],
    "dnet_set_params": [P, P],
    "dnet_get_grads": [P, P],
    "dnet_forward": [P, P, INT, P, P],
    "dnet_backward": [P, P, P],
    "dnet_adam": [P, C.c_float, INT, P],
    "dnet_mse": [P, P, P, I64, C.POINTER(D), P, P],
    "dnet_crop": [P, INT, INT, INT, INT, INT, INT, P, P],
    "dnet_highpass": [P, INT, D, P, P, P],
    "chf_rows_to_box": [P, P, P, D, P, INT, INT, P],
    "chf_box_to_rows": [P, P, INT, INT, D, P, P, P],
}

_lib = None


def lib():
    """Load libchfsi.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        # torch brings its own HIP runtime, which the library then shares
        # (same soname); initialise torch's device state first, so that a
        # library call that touches the device before any tensor does (for
        # example creating the density network) cannot leave torch unable
        # to see the GPU
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
        L = C.CDLL(LIB_PATH)
        L.chf_last_error.restype = C.c_char_p
        L.chf_last_error.argtypes = []
        L.chf_device_allocations.restype = C.c_int64
        L.chf_device_allocations.argtypes = []
        for name, args in _SIGS.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.restype = C.c_int
            f.argtypes = args
        _lib = L
    return _lib


def declared_symbols() -> list[str]:
    return ["chf_last_error", "chf_device_allocations", *_SIGS.keys()]


def check(rc: int) -> None:
    if rc != 0:
        raise ChfError(rc, lib().chf_last_error().decode())


def call(name: str, *args) -> None:
    check(getattr(lib(), name)(*args))


# ---------------------------------------------------------------------------
# tensor helpers (torch imported lazily so host-only use needs no GPU)
# ---------------------------------------------------------------------------
def _stream():
    import torch
    return P(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> P:
    return P(t.data_ptr())


def _torch_f64():
    import torch
    return torch.float64


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return CHF_F64
    if t.dtype == torch.float32:
        return CHF_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _on_gpu(t, what: str) -> None:
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{what}: expected a tensor in GPU memory")


def _block(t, rows: int | None = None, like=None, nvec: int | None = None, what: str = "vector block"):
    """(pointer, ld) of a row-major block.  The library sees only the pointer and
    ld, so the extent it will touch is checked here: at least `rows` rows, at
    least `nvec` columns, the dtype of `like`, device memory."""
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("vector blocks must be 2-D with contiguous rows")
    if rows is not None and t.shape[0] < rows:
        raise ValueError(f"{what}: {t.shape[0]} rows, the Hamiltonian has {rows}")
    if nvec is not None and not 1 <= nvec <= t.shape[1]:
        raise ValueError(f"{what}: nvec {nvec} outside 1..{t.shape[1]}")
    if like is not None and t.dtype != like.dtype:
        raise TypeError(f"{what}: dtype {t.dtype} differs from {like.dtype}")
    _on_gpu(t, what)
    return _ptr(t), t.stride(0)


def _vec(t, n: int, what: str, double: bool = True):
    """Pointer to a contiguous device vector of at least n FP64 (or FP32) values."""
    import torch
    want = torch.float64 if double else torch.float32
    if t.dtype != want:
        raise TypeError(f"{what}: dtype {t.dtype}, expected {want}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: must be contiguous")
    if t.numel() < n:
        raise ValueError(f"{what}: {t.numel()} values, needs {n}")
    _on_gpu(t, what)
    return _ptr(t)


def make_pp(pp) -> PP:
    return PP(pp.z_si, pp.z_h, pp.r_loc, pp.r_loc_h, pp.r_c, pp.r_cut, pp.h_s, pp.h_p)


def _atoms(pos: np.ndarray, species: np.ndarray):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    species = np.ascontiguousarray(species, dtype=np.int32)
    a = Atoms(len(species), pos.ctypes.data_as(C.POINTER(C.c_double)), species.ctypes.data_as(C.POINTER(C.c_int)))
    return a, (pos, species)


def ordering_host(h: float, radius: float, ordering: int = ORDER_HILBERT, with_nbr: bool = True):
    g = GridDesc(h, radius, ordering, 0, 3)
    n, nr = I64(), I64()
    call("chf_ordering_host", C.byref(g), C.byref(n), C.byref(nr), None, None, None)
    ijk = np.zeros((n.value, 3), np.int32)
    rows = np.zeros(n.value, np.int64)
    nbr = np.zeros((n.value, 36), np.int32) if with_nbr else None
    call("chf_ordering_host", C.byref(g), C.byref(n), C.byref(nr), P(ijk.ctypes.data), P(rows.ctypes.data),
         P(nbr.ctypes.data) if with_nbr else None)
    return ijk, rows, nbr, nr.value


def projectors_host(h: float, radius: float, pos, species, pp, ordering: int = ORDER_HILBERT):
    g = GridDesc(h, radius, ordering, 0, 3)
    a, keep = _atoms(pos, species)
    cp = make_pp(pp)
    npairs = I64()
    call("chf_projectors_host", C.byref(g), C.byref(a), C.byref(cp), C.byref(npairs), None, None, None)
    n_si = int((np.asarray(species) == 0).sum())
    off = np.zeros(n_si + 1, np.int64)
    rk = np.zeros(npairs.value, np.int32)
    beta = np.zeros((npairs.value, 4), np.float64)
    call("chf_projectors_host", C.byref(g), C.byref(a), C.byref(cp), C.byref(npairs), P(off.ctypes.data),
         P(rk.ctypes.data), P(beta.ctypes.data))
    return off, rk, beta


def timer(enable: bool) -> None:
    call("chf_timer", int(enable))


def timer_read() -> dict:
    ms = (C.c_double * 2)()
    n = (C.c_int64 * 2)()
    call("chf_timer_read", C.cast(ms, P), C.cast(n, P))
    return {"hx_ms": ms[0], "hx_launches": n[0], "gather_ms": ms[1], "gather_launches": n[1]}


class Context:
    def __init__(self, device: int = 0):
        self.handle = P()
        call("chf_ctx_create", device, C.byref(self.handle))

    def close(self):
        if self.handle:
            call("chf_ctx_destroy", self.handle)
            self.handle = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hamiltonian:
    """Device Hamiltonian handle (ham_build / ham_* calls)."""

    def __init__(self, pos, species, pp, h: float, radius: float, ordering: int = ORDER_HILBERT,
                 keep_nbr: bool = False, dtypes: int = 3):
        g = GridDesc(h, radius, ordering, int(keep_nbr), dtypes)
        a, keep = _atoms(pos, species)
        cp = make_pp(pp)
        self.handle = P()
        call("ham_build", C.byref(g), C.byref(a), C.byref(cp), _stream(), C.byref(self.handle))
        vals = [I64() for _ in range(5)]
        call("ham_info", self.handle, *[C.byref(v) for v in vals])
        self.n_points, self.n_rows, self.n_blocks, self.n_proj, self.n_pairs = [v.value for v in vals]
        self.h = h
        self.ordering = ordering

    def close(self):
        if self.handle:
            call("ham_destroy", self.handle)
            self.handle = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def export_ordering(self, with_nbr: bool = False):
        ijk = np.zeros((self.n_points, 3), np.int32)
        rows = np.zeros(self.n_points, np.int64)
        nbr = np.zeros((self.n_points, 36), np.int32) if with_nbr else None
        call("ham_export_ordering", self.handle, P(ijk.ctypes.data), P(rows.ctypes.data),
             P(nbr.ctypes.data) if with_nbr else None)
        return ijk, rows, nbr

    def vloc(self):
        import torch
        out = torch.empty(self.n_rows, dtype=torch.float64, device="cuda")
        call("ham_get_vloc", self.handle, _ptr(out), _stream())
        return out

    def set_veff(self, veff):
        call("ham_set_veff", self.handle, _vec(veff.contiguous(), self.n_rows, "veff"), _stream())

    def apply(self, X, Y, generic: bool = False):
        px, ldx = _block(X, self.n_rows, what="X")
        py, ldy = _block(Y, self.n_rows, like=X, nvec=X.shape[1], what="Y")
        call("chf_ham_apply_generic" if generic else "ham_apply", self.handle, _dtype_code(X), px, ldx, py, ldy,
             X.shape[1], _stream())

    def filter(self, X, work, degree: int, a: float, b: float, a0: float, generic: bool = False, nvec=None):
        """X <- p_m(H) X in place; work may be narrower than X (column blocks)."""
        px, ldx = _block(X, self.n_rows, nvec=nvec or X.shape[1], what="X")
        pw, ldw = _block(work, self.n_rows, like=X, what="work")
        call("chf_filter_generic" if generic else "chebyshev_filter", self.handle, _dtype_code(X), px, ldx,
             nvec or X.shape[1], degree, a, b, a0, pw, ldw, _stream())

    def lanczos_bound(self, ctx: Context, v0, k: int = 10):
        out = (C.c_double * 3)()
        call("lanczos_bound", self.handle, ctx.handle, _vec(v0, self.n_rows, "v0"), k, C.cast(out, P), _stream())
        return tuple(out)

    def density(self, X, n_occ: int, rho):
        px, ldx = _block(X, self.n_rows, nvec=n_occ, what="X")
        call("chf_density", self.handle, _dtype_code(X), px, ldx, n_occ, _vec(rho, self.n_rows, "rho"), _stream())

    def hartree(self, ctx: Context, rho, vh, rtol: float = 1e-12, max_iter: int = 20000) -> int:
        it = C.c_int()
        call("chf_hartree", self.handle, ctx.handle, _vec(rho, self.n_rows, "rho"), _vec(vh, self.n_rows, "vh"), rtol,
             max_iter, C.byref(it), _stream())
        return it.value

    def lda(self, rho, exc, vxc):
        call("chf_lda", self.handle, _vec(rho, self.n_rows, "rho"),
             _vec(exc, self.n_rows, "exc") if exc is not None else None, _vec(vxc, self.n_rows, "vxc"), _stream())

    def density_fix(self, rho, n_electrons: int):
        call("chf_density_fix", self.handle, _vec(rho, self.n_rows, "rho"), n_electrons, _stream())

    def sad_density(self, pos, species, n_electrons: int, alpha_si: float = 0.074, alpha_h: float = 0.21):
        import torch
        a, keep = _atoms(pos, species)
        rho = torch.zeros(self.n_rows, dtype=torch.float64, device="cuda")
        call("chf_sad_density", self.handle, C.byref(a), alpha_si, alpha_h, n_electrons, _ptr(rho), _stream())
        return rho


def ion_energy(pos, species, pp) -> float:
    a, keep = _atoms(pos, species)
    cp = make_pp(pp)
    out = C.c_double()
    call("chf_ion_energy", C.byref(a), C.byref(cp), C.byref(out))
    return out.value


def gram(ctx: Context, A, B, S) -> None:
    pa, lda = _block(A, what="A")
    pb, ldb = _block(B, A.shape[0], like=A, what="B")
    ps, lds = _block(S, A.shape[1], nvec=B.shape[1], what="S")
    if S.dtype != _torch_f64():
        raise TypeError("S: must be FP64")
    call("gram", ctx.handle, _dtype_code(A), pa, lda, pb, ldb, A.shape[0], A.shape[1], B.shape[1], ps, lds, _stream())


def orthonormalize(ctx: Context, X, nvec=None, gram_dtype=None) -> int:
    """Cholesky-QR of X in place; gram_dtype (CHF_F32 / CHF_F64) defaults to the
    block's precision.  Returns the number of breakdown retries."""
    px, ldx = _block(X, nvec=nvec or X.shape[1], what="X")
    fb = C.c_int()
    code = _dtype_code(X)
    call("orthonormalize", ctx.handle, code, px, ldx, X.shape[0], nvec or X.shape[1],
         code if gram_dtype is None else gram_dtype, C.byref(fb), _stream())
    return fb.value


def rayleigh_ritz(H: Hamiltonian, ctx: Context, X, work, nvec=None) -> np.ndarray:
    n = nvec or X.shape[1]
    px, ldx = _block(X, H.n_rows, nvec=n, what="X")
    pw, ldw = _block(work, H.n_rows, like=X, what="work")
    eig = np.zeros(n, np.float64)
    call("rayleigh_ritz", H.handle, ctx.handle, _dtype_code(X), px, ldx, n, P(eig.ctypes.data), pw, ldw, _stream())
    return eig


WS_FILTER, WS_ORTHONORMALIZE, WS_RAYLEIGH_RITZ, WS_LANCZOS = 0, 1, 2, 3


def workspace_bytes(H, op: int, dtype: int, nvec: int, ldw: int = 0):
    """(bytes on the Hamiltonian, bytes on the context) of one operation."""
    hb, cb = I64(), I64()
    call("chf_workspace_bytes", H.handle, op, dtype, nvec, ldw, C.byref(hb), C.byref(cb))
    return hb.value, cb.value


def reserve(H, ctx, op: int, dtype: int, nvec: int, ldw: int = 0) -> None:
    call("chf_reserve", H.handle, ctx.handle if ctx is not None else None, op, dtype, nvec, ldw)


def device_allocations() -> int:
    return int(lib().chf_device_allocations())


class Scf:
    """SCF state handle (chf_scf_create / scf_step)."""

    def __init__(self, H: Hamiltonian, ctx: Context, params: ScfParams, rho0, v_lanczos):
        self.handle = P()
        self._keep = (H, ctx)
        call("chf_scf_create", H.handle, ctx.handle, C.byref(params), _vec(rho0, H.n_rows, "rho0"),
             _vec(v_lanczos, H.n_rows, "v_lanczos"), C.byref(self.handle))
        self.nvec = params.nvec
        self.n_rows = H.n_rows
        self.filter_double = params.filter_dtype == CHF_F64

    def step(self, X, work):
        if (X.dtype == _torch_f64()) != self.filter_double:
            raise TypeError(f"X: dtype {X.dtype} is not the SCF's filter precision")
        px, ldx = _block(X, self.n_rows, nvec=self.nvec, what="X")
        pw, ldw = _block(work, self.n_rows, like=X, what="work")
        rep = ScfReport()
        eig = np.zeros(self.nvec, np.float64)
        call("scf_step", self.handle, px, ldx, pw, ldw, C.byref(rep), P(eig.ctypes.data))
        return rep, eig

    def save(self) -> np.ndarray:
        """Checkpoint of the SCF state (host array; X is saved by the caller)."""
        n = I64()
        call("chf_scf_state_size", self.handle, C.byref(n))
        out = np.zeros(n.value, np.float64)
        call("chf_scf_save", self.handle, P(out.ctypes.data))
        return out

    def load(self, state: np.ndarray) -> None:
        state = np.ascontiguousarray(state, dtype=np.float64)
        call("chf_scf_load", self.handle, P(state.ctypes.data), int(state.size))

    def fields(self, rho_in, vh=None):
        call("chf_scf_get_fields", self.handle, _vec(rho_in, self.n_rows, "rho_in") if rho_in is not None else None,
             _vec(vh, self.n_rows, "vh") if vh is not None else None)

    def close(self):
        if self.handle:
            call("chf_scf_destroy", self.handle)
            self.handle = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


LAYER_NAMES = ["c1a", "c1b", "d1", "c2a", "c2b", "d2", "c3a", "c3b", "d3", "c4a", "c4b", "u3", "c5a", "c5b", "u2",
               "c6a", "c6b", "u1", "c7a", "c7b", "out"]


class DensityNet:
    """Device U-Net for the initial-density correction (dnet_* calls)."""

    def __init__(self, channels: int = 32, seed: int = 0):
        self.handle = P()
        call("dnet_create", channels, seed, C.byref(self.handle))
        n = I64()
        call("dnet_param_count", self.handle, C.byref(n))
        self.n_params = n.value
        self.layers = {}
        for i, name in enumerate(LAYER_NAMES):
            info = (C.c_int * 6)()
            off = (C.c_int64 * 2)()
            call("dnet_layer_info", self.handle, i, C.cast(info, P), C.cast(off, P))
            self.layers[name] = (tuple(info), tuple(off))

    def close(self):
        if self.handle:
            call("dnet_destroy", self.handle)
            self.handle = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        call("dnet_get_params", self.handle, P(out.ctypes.data))
        return out

    def set_params(self, flat: np.ndarray) -> None:
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        if flat.size != self.n_params:
            raise ValueError(f"set_params: {flat.size} values, the network has {self.n_params}")
        call("dnet_set_params", self.handle, P(flat.ctypes.data))

    def get_grads(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        call("dnet_get_grads", self.handle, P(out.ctypes.data))
        return out

    def forward(self, x, y):
        S = int(round(x.numel() ** (1 / 3)))
        if S ** 3 != x.numel():
            raise ValueError(f"forward: x holds {x.numel()} values, not an S^3 patch")
        call("dnet_forward", self.handle, _vec(x, S ** 3, "x", double=False), S, _vec(y, S ** 3, "y", double=False),
             _stream())
        self._n_out = S ** 3

    def backward(self, dy):
        call("dnet_backward", self.handle, _vec(dy, getattr(self, "_n_out", 0), "dy", double=False), _stream())

    def adam(self, lr: float, step: int):
        call("dnet_adam", self.handle, lr, step, _stream())

    def mse(self, y, t, dy=None) -> float:
        loss = C.c_double()
        n = y.numel()
        call("dnet_mse", self.handle, _vec(y, n, "y", double=False), _vec(t, n, "t", double=False), n, C.byref(loss),
             _vec(dy, n, "dy", double=False) if dy is not None else None, _stream())
        return loss.value


def dnet_plan(S: int) -> list[int]:
    edges = (C.c_int * len(LAYER_NAMES))()
    call("dnet_plan", S, C.cast(edges, P))
    return list(edges)


def crop(box, D: int, S: int, origin, sym: int, patch) -> None:
    call("dnet_crop", _vec(box, D ** 3, "box", double=False), D, S, int(origin[0]), int(origin[1]), int(origin[2]), sym,
         _vec(patch, S ** 3, "patch", double=False), _stream())


def highpass(box, D: int, sigma: float, out, work) -> None:
    call("dnet_highpass", _vec(box, D ** 3, "box", double=False), D, float(sigma),
         _vec(out, D ** 3, "out", double=False), _vec(work, 2 * D ** 3, "work", double=False), _stream())


def rows_to_box(H: "Hamiltonian", rows, scale: float, box, D: int, off: int, base=None) -> None:
    """box = scale * (rows - base) on the cells of the grid points (base None: 0)."""
    call("chf_rows_to_box", H.handle, _vec(rows, H.n_rows, "rows"),
         _vec(base, H.n_rows, "base") if base is not None else None, scale, _vec(box, D ** 3, "box", double=False), D,
         off, _stream())


def box_to_rows(H: "Hamiltonian", box, D: int, off: int, scale: float, base, out) -> None:
    call("chf_box_to_rows", H.handle, _vec(box, D ** 3, "box", double=False), D, off, scale,
         _vec(base, H.n_rows, "base") if base is not None else None, _vec(out, H.n_rows, "out"), _stream())
