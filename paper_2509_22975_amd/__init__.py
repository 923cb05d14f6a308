"""MI355X-native Monte Carlo diagonalization hot path (Python binding).

Thin ctypes marshalling over ``libmcd.so`` (C ABI in ``include/mcd.h``).
Every step of the path runs in the library's HIP kernels; PyTorch only
provides device memory (tensors) and the current HIP stream.  The library
must be built (``python -m paper_2509_22975_amd.build``); importing this
package without it raises, there is no fallback.

Keys are passed as torch.int64 tensors holding the uint64 bit pattern
(up << 32) | down.

Device memory: the library allocates none; every call that needs device
memory takes a workspace (``Workspace``: a torch.uint8 tensor wrapped by
mcd_ws_create).  An ``Operator`` owns a workspace of exactly the size
mcd_op_workspace_size reports; a kept band run (``BandKeep``) one of the size
mcd_band_workspace_size reports; solver calls take their scratch from a
workspace per (device, stream) that this module keeps and grows when a call
reports MCD_E_WORKSPACE (``release_scratch()`` hands it back to torch).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcd.so")

MCD_OK, MCD_NOCONV = 0, 1
MCD_E_WORKSPACE = -5
STORAGE = {"auto": 0, "on_the_fly": 1, "otf": 1, "csr": 2}
STORAGE_NAME = {0: "auto", 1: "on_the_fly", 2: "csr"}
DTYPE = {"f64": 0, "f32": 1}
KERNEL_NAME = {1: "stream", 2: "merge", 3: "stream_xcd", 4: "rowchunk", 5: "stream_small",
               6: "stream_small_xcd", 7: "grouped", 8: "grouped_xcd"}

P = ctypes.POINTER
c_i32, c_i64, c_u64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p


class McdModel(ctypes.Structure):
    _fields_ = [("n_orb", c_i32), ("n_bonds", c_i32), ("bond_i", P(c_i32)), ("bond_j", P(c_i32)),
                ("bond_t", P(c_dbl)), ("U", P(c_dbl)), ("eps", P(c_dbl))]


class McdBasisCfg(ctypes.Structure):
    _fields_ = [("mode", c_i32), ("n_up", c_i32), ("n_dn", c_i32), ("start_key", c_u64),
                ("seed", c_u64), ("beta_s", c_dbl), ("burn_in", c_i64), ("max_steps", c_i64),
                ("n_f", c_i64), ("pre_level", c_i32)]


class McdOpInfo(ctypes.Structure):
    _fields_ = [("n", c_i64), ("nnz", c_i64), ("storage", c_i32), ("n_classes", c_i32),
                ("rows_per_block", c_i32), ("kernel", c_i32), ("device_bytes", c_i64),
                ("build_ms", c_dbl), ("grouped_blocks", c_i64),
                ("grouped_groups", c_i64), ("rows_per_block_l", c_i32), ("reserved", c_i32)]


class McdLanczosCfg(ctypes.Structure):
    _fields_ = [("max_iter", c_i32), ("check_every", c_i32), ("tol", c_dbl), ("seed", c_u64),
                ("store_vectors", c_i32), ("min_iter", c_i32), ("precision", c_i32)]


class McdSolveInfo(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("converged", c_i32), ("e0", c_dbl), ("residual", c_dbl),
                ("solve_ms", c_dbl), ("apply_ms", c_dbl), ("n_apply", c_i32),
                ("krylov_dim", c_i32), ("n_plus", c_i64), ("n_minus", c_i64),
                ("n_truncated", c_i64)]


class McdBandCfg(ctypes.Structure):
    _fields_ = [("max_blocks", c_i32), ("precision", c_i32), ("w_t", c_dbl), ("dtol", c_dbl),
                ("storage", c_i32), ("reorth", c_i32), ("per_column", c_i32), ("eta", c_dbl),
                ("g_tol", c_dbl), ("vjp_freq_batch", c_i32), ("vjp_chunk", c_i32)]


_lib = None


def lib():
    """The loaded libmcd.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2509_22975_amd.build` (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    L.mcd_last_error.restype = ctypes.c_char_p
    L.mcd_version.restype = ctypes.c_int
    c_sz = ctypes.c_size_t
    L.mcd_ws_create.argtypes = [c_vp, c_sz, P(c_vp)]
    L.mcd_ws_destroy.argtypes = [c_vp]
    L.mcd_ws_destroy.restype = None
    L.mcd_ws_stats.argtypes = [c_vp, P(c_sz), P(c_sz), P(c_sz), P(c_sz)]
    L.mcd_ws_set_debug.argtypes = [c_vp, c_i32]
    L.mcd_basis_build.argtypes = [P(McdModel), P(McdBasisCfg), c_vp, c_i64, P(c_i64), P(c_i64),
                                  c_vp, c_vp]
    L.mcd_op_create.argtypes = [P(McdModel), c_vp, c_i64, c_i32, c_i32, c_vp, c_vp, P(c_vp)]
    L.mcd_op_workspace_size.argtypes = [P(McdModel), c_vp, c_i64, c_i32, c_vp, c_vp, P(c_sz),
                                        P(c_sz)]
    L.mcd_op_destroy.argtypes = [c_vp]
    L.mcd_op_destroy.restype = None
    L.mcd_op_info.argtypes = [c_vp, P(McdOpInfo)]
    L.mcd_op_set_kernel.argtypes = [c_vp, c_i32]
    L.mcd_hamiltonian_apply.argtypes = [c_vp, c_i32, c_i32, c_vp, c_vp, c_vp]
    L.mcd_hamiltonian_diagonal.argtypes = [c_vp, c_vp, c_vp]
    L.mcd_hamiltonian_connectivity.argtypes = [c_vp, c_i64, c_i64, c_vp, c_vp, c_vp, c_i64,
                                               P(c_i64), c_vp, c_vp]
    L.mcd_lanczos_ground.argtypes = [c_vp, P(McdLanczosCfg), c_vp, P(c_dbl), c_vp, P(c_dbl),
                                     P(c_dbl), P(McdSolveInfo), c_vp, c_vp]
    L.mcd_lanczos_workspace_size.argtypes = [c_vp, P(McdLanczosCfg), P(c_sz)]
    L.mcd_hamiltonian_contract.argtypes = [c_vp, P(McdModel), c_vp, c_vp, P(c_dbl), P(c_dbl),
                                           P(c_dbl), c_vp, c_vp]
    L.mcd_hamiltonian_contract_noalloc.argtypes = [c_vp, P(McdModel), c_vp, c_vp, P(c_dbl),
                                                   P(c_dbl), P(c_dbl), c_vp]
    L.mcd_batch_lanczos_ground.argtypes = [P(c_vp), c_i32, P(McdLanczosCfg), P(c_dbl), P(c_vp),
                                           P(c_i32), P(McdSolveInfo), c_vp, c_vp]
    band = [P(McdModel), c_vp, c_i64, c_vp, c_dbl, c_i32, P(c_i32), P(c_i32), c_i32, P(c_dbl),
            P(McdBandCfg)]
    L.mcd_band_lanczos_green.argtypes = band + [P(c_dbl), P(c_dbl), P(c_dbl), P(McdSolveInfo),
                                                c_vp, c_vp]
    L.mcd_band_workspace_size.argtypes = band + [c_i32, c_vp, c_vp, P(c_sz)]
    L.mcd_batch_band_green.argtypes = [P(c_vp), P(c_vp), P(c_i64), P(c_vp), P(c_dbl), c_i32,
                                       c_i32, P(c_i32), P(c_i32), c_i32, P(c_dbl),
                                       P(McdBandCfg), P(c_vp), P(McdSolveInfo), c_vp, c_vp]
    vjp = band + [P(c_dbl), c_dbl, c_dbl, c_i32, P(c_dbl), P(c_dbl), P(c_dbl), P(McdSolveInfo),
                  c_vp, c_vp]
    L.mcd_band_green_vjp.argtypes = vjp
    L.mcd_band_lanczos_green_keep.argtypes = L.mcd_band_lanczos_green.argtypes + [P(c_vp)]
    L.mcd_band_green_vjp_keep.argtypes = vjp + [c_vp]
    L.mcd_band_keep_destroy.argtypes = [c_vp]
    L.mcd_band_keep_destroy.restype = None
    for name in ("mcd_basis_build", "mcd_op_create", "mcd_op_info", "mcd_op_set_kernel",
                 "mcd_hamiltonian_apply", "mcd_hamiltonian_diagonal",
                 "mcd_hamiltonian_connectivity", "mcd_lanczos_ground", "mcd_band_lanczos_green",
                 "mcd_batch_lanczos_ground", "mcd_hamiltonian_contract", "mcd_band_green_vjp",
                 "mcd_batch_band_green", "mcd_band_lanczos_green_keep", "mcd_band_green_vjp_keep",
                 "mcd_ws_create", "mcd_ws_stats", "mcd_ws_set_debug", "mcd_op_workspace_size",
                 "mcd_lanczos_workspace_size", "mcd_band_workspace_size",
                 "mcd_hamiltonian_contract_noalloc"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class McdError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().mcd_last_error().decode(errors="replace")
        super().__init__(f"{where}: status {code}: {msg}")
        self.code = code


def _check(code, where, allow_noconv=True):
    if code < 0 or (code > 0 and not allow_noconv):
        raise McdError(code, where)
    return code


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


WS_POISON = 1          # mcd_ws_set_debug: NaN-fill floating-point pieces on take
_WS_DEBUG = 0


class Workspace:
    """A caller-owned device buffer handed to the library (mcd_ws): a
    torch.uint8 tensor of `nbytes` bytes on `device` and its handle.  New
    workspaces take the flags set by ``workspace_debug``."""

    def __init__(self, nbytes, device="cuda"):
        torch = _torch()
        self.nbytes = int(max(nbytes, 256) + 255) // 256 * 256
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        if self.buf.data_ptr() % 256:
            raise RuntimeError("workspace buffer is not 256-byte aligned")
        h = c_vp(0)
        _check(lib().mcd_ws_create(c_vp(self.buf.data_ptr()), self.nbytes, ctypes.byref(h)),
               "mcd_ws_create")
        self._h = h
        if _WS_DEBUG:
            self.set_debug(_WS_DEBUG)

    def set_debug(self, flags: int):
        _check(lib().mcd_ws_set_debug(self._h, int(flags)), "mcd_ws_set_debug")

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        sz, used, high, need = (ctypes.c_size_t(0) for _ in range(4))
        _check(lib().mcd_ws_stats(self._h, ctypes.byref(sz), ctypes.byref(used),
                                  ctypes.byref(high), ctypes.byref(need)), "mcd_ws_stats")
        return dict(size=sz.value, in_use=used.value, high_water=high.value, need=need.value)

    def close(self):
        if self._h:
            lib().mcd_ws_destroy(self._h)
            self._h = c_vp(0)
            self.buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_SCRATCH = {}


def workspace_debug(flags: int):
    """Debug flags (WS_POISON or 0) for every workspace created from now on
    and for the current scratch workspaces; returns the previous flags."""
    global _WS_DEBUG
    old, _WS_DEBUG = _WS_DEBUG, int(flags)
    for ws in _SCRATCH.values():
        ws.set_debug(_WS_DEBUG)
    return old


def _scratch_key():
    torch = _torch()
    return (torch.cuda.current_device(), torch.cuda.current_stream().cuda_stream)


def scratch(min_bytes=0) -> Workspace:
    """The solver scratch workspace of the current device and stream (kept
    between calls, grown on demand; calls on one stream are ordered, so its
    pieces are reused safely)."""
    key = _scratch_key()
    ws = _SCRATCH.get(key)
    if ws is None or ws.nbytes < min_bytes:
        if ws is not None:
            ws.close()
        ws = Workspace(max(min_bytes, 64 << 20), device=f"cuda:{key[0]}")
        _SCRATCH[key] = ws
    return ws


def release_scratch():
    """Hands every scratch workspace of this module back to torch."""
    _torch().cuda.synchronize()
    for ws in _SCRATCH.values():
        ws.close()
    _SCRATCH.clear()


def _with_scratch(call, where, min_bytes=0, tries=8):
    """call(ws_handle) on the scratch workspace; on MCD_E_WORKSPACE the scratch
    grows to the size the failed request needed (at least doubling) and the
    call is made again."""
    need = min_bytes
    for _ in range(tries):
        ws = scratch(need)
        code = call(ws.handle)
        if code != MCD_E_WORKSPACE:
            return _check(code, where)
        need = max(ws.stats()["need"], 2 * ws.nbytes)
        need = (need + (1 << 20) - 1) // (1 << 20) * (1 << 20)
    raise McdError(MCD_E_WORKSPACE, where)


class _ModelBuf:
    """Keeps the host arrays of an mcd_model alive while the struct is used."""

    def __init__(self, model):
        bonds = list(model.bonds)
        self.bi = np.ascontiguousarray([b[0] for b in bonds], dtype=np.int32)
        self.bj = np.ascontiguousarray([b[1] for b in bonds], dtype=np.int32)
        self.bt = np.ascontiguousarray([b[2] for b in bonds], dtype=np.float64)
        self.U = np.ascontiguousarray(model.U, dtype=np.float64)
        self.eps = np.ascontiguousarray(model.eps, dtype=np.float64)
        self.s = McdModel(int(model.n_orb), len(bonds),
                          self.bi.ctypes.data_as(P(c_i32)), self.bj.ctypes.data_as(P(c_i32)),
                          self.bt.ctypes.data_as(P(c_dbl)), self.U.ctypes.data_as(P(c_dbl)),
                          self.eps.ctypes.data_as(P(c_dbl)))


def keys_to_numpy(keys) -> np.ndarray:
    return keys.detach().cpu().numpy().view(np.uint64)


def keys_from_numpy(keys: np.ndarray, device="cuda"):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(keys, dtype=np.uint64).view(np.int64)).to(device)


def basis_build(model, mode="full", n_up=None, n_dn=None, start_key=0, seed=0, beta_s=0.5,
                burn_in=0, max_steps=0, n_f=0, cap=None, device="cuda", pre_level=0):
    """Basis keys (torch.int64 on device) and the number of chain steps."""
    torch = _torch()
    n_up = model.n_up if n_up is None else n_up
    n_dn = model.n_dn if n_dn is None else n_dn
    mb = _ModelBuf(model)
    m = {"full": 0, "chain": 1, "steps": 2}[mode]
    if cap is None:
        import math
        cap = math.comb(model.n_orb, n_up) * math.comb(model.n_orb, n_dn) if m == 0 else int(n_f)
    cfg = McdBasisCfg(m, n_up, n_dn, int(start_key), int(seed), float(beta_s), int(burn_in),
                      int(max_steps), int(n_f), int(pre_level))
    out = torch.empty(max(int(cap), 1), dtype=torch.int64, device=device)
    n_out, steps = c_i64(0), c_i64(0)
    _with_scratch(lambda ws: lib().mcd_basis_build(ctypes.byref(mb.s), ctypes.byref(cfg),
                                                   c_vp(out.data_ptr()), int(cap),
                                                   ctypes.byref(n_out), ctypes.byref(steps), ws,
                                                   _stream()),
                  "mcd_basis_build")
    return out[: n_out.value], steps.value


class Operator:
    """H~ on a basis (mcd_op_create / mcd_hamiltonian_apply)."""

    def __init__(self, model, keys, storage="auto", validate=True):
        torch = _torch()
        assert keys.dtype == torch.int64 and keys.is_cuda
        self.model = model
        self._mb = _ModelBuf(model)
        self.keys = keys.contiguous()
        self.n = int(keys.numel())
        self.device = keys.device
        self.ws_bytes = operator_workspace_size(model, self.keys, storage, mb=self._mb)
        self._ws = Workspace(self.ws_bytes, device=self.device)
        h = c_vp(0)
        _check(lib().mcd_op_create(ctypes.byref(self._mb.s), c_vp(self.keys.data_ptr()), self.n,
                                   STORAGE[storage], 1 if validate else 0, self._ws.handle,
                                   _stream(), ctypes.byref(h)), "mcd_op_create")
        self._h = h

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("operator is closed")
        return self._h

    def info(self) -> dict:
        i = McdOpInfo()
        _check(lib().mcd_op_info(self.handle, ctypes.byref(i)), "mcd_op_info")
        return dict(n=i.n, nnz=i.nnz, storage=STORAGE_NAME[i.storage], n_classes=i.n_classes,
                    rows_per_block=i.rows_per_block, kernel=KERNEL_NAME.get(i.kernel, "none"),
                    device_bytes=i.device_bytes, build_ms=i.build_ms,
                    grouped_blocks=i.grouped_blocks, grouped_groups=i.grouped_groups,
                    rows_per_block_l=i.rows_per_block_l)

    def kernels(self) -> list:
        """One-vector CSR kernels this operator can run (grouped ones only when
        its grouped layout was built)."""
        if self.info()["storage"] != "csr":
            return []
        g = self.info()["grouped_blocks"] > 0
        return [v for k, v in sorted(KERNEL_NAME.items()) if g or k < 7]

    def set_kernel(self, name: str):
        """Force the one-vector CSR kernel: 'stream', 'merge', 'stream_xcd', 'rowchunk',
        'stream_small', 'stream_small_xcd', 'grouped' or 'grouped_xcd'."""
        _check(lib().mcd_op_set_kernel(self.handle, {v: k for k, v in KERNEL_NAME.items()}[name]),
               "mcd_op_set_kernel")

    def apply(self, x, out=None):
        """y = H~ x; x is (n,) or (n, nvec) float64/float32 on the device."""
        torch = _torch()
        x = x.contiguous()
        nvec = 1 if x.dim() == 1 else x.shape[1]
        dt = {torch.float64: 0, torch.float32: 1}[x.dtype]
        y = torch.empty_like(x) if out is None else out
        _check(lib().mcd_hamiltonian_apply(self.handle, dt, nvec, c_vp(x.data_ptr()),
                                           c_vp(y.data_ptr()), _stream()), "mcd_hamiltonian_apply")
        return y

    def apply_raw(self, dtype_code: int, nvec: int, x_ptr: int, y_ptr: int, stream=None):
        return lib().mcd_hamiltonian_apply(self.handle, dtype_code, nvec, c_vp(x_ptr), c_vp(y_ptr),
                                           _stream() if stream is None else stream)

    def diagonal(self):
        torch = _torch()
        d = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(lib().mcd_hamiltonian_diagonal(self.handle, c_vp(d.data_ptr()), _stream()),
               "mcd_hamiltonian_diagonal")
        return d

    def connectivity(self, row0=0, row1=None):
        """(rows, cols, vals) numpy arrays of the off-diagonal elements."""
        torch = _torch()
        row1 = self.n if row1 is None else row1
        cnt = c_i64(0)
        ws = scratch(8 * max(row1 - row0, 1) + 4096)
        code = lib().mcd_hamiltonian_connectivity(self.handle, row0, row1, None, None, None, 0,
                                                  ctypes.byref(cnt), ws.handle, _stream())
        if code not in (0, -4):
            _check(code, "mcd_hamiltonian_connectivity")
        m = max(cnt.value, 1)
        r = torch.empty(m, dtype=torch.int64, device=self.device)
        c = torch.empty(m, dtype=torch.int64, device=self.device)
        v = torch.empty(m, dtype=torch.float64, device=self.device)
        _check(lib().mcd_hamiltonian_connectivity(self.handle, row0, row1, c_vp(r.data_ptr()),
                                                  c_vp(c.data_ptr()), c_vp(v.data_ptr()), m,
                                                  ctypes.byref(cnt), ws.handle, _stream()),
               "mcd_hamiltonian_connectivity")
        k = cnt.value
        return r[:k].cpu().numpy(), c[:k].cpu().numpy(), v[:k].cpu().numpy()

    def contract(self, a, b=None):
        """(d_t [n_bonds], d_U [n_orb], d_eps [n_orb]) = <a| dH~/dtheta |b> (numpy)."""
        b = a if b is None else b
        m = self.model
        dt = np.zeros(len(m.bonds))
        dU = np.zeros(m.n_orb)
        de = np.zeros(m.n_orb)
        _with_scratch(lambda ws: lib().mcd_hamiltonian_contract(
            self.handle, ctypes.byref(self._mb.s), c_vp(a.data_ptr()), c_vp(b.data_ptr()),
            dt.ctypes.data_as(P(c_dbl)), dU.ctypes.data_as(P(c_dbl)),
            de.ctypes.data_as(P(c_dbl)), ws, _stream()), "mcd_hamiltonian_contract")
        return dt, dU, de

    def contract_noalloc(self, a, b=None):
        """contract() through mcd_hamiltonian_contract_noalloc (no workspace:
        the library's fixed device scratch)."""
        b = a if b is None else b
        m = self.model
        dt = np.zeros(len(m.bonds))
        dU = np.zeros(m.n_orb)
        de = np.zeros(m.n_orb)
        _check(lib().mcd_hamiltonian_contract_noalloc(
            self.handle, ctypes.byref(self._mb.s), c_vp(a.data_ptr()), c_vp(b.data_ptr()),
            dt.ctypes.data_as(P(c_dbl)), dU.ctypes.data_as(P(c_dbl)),
            de.ctypes.data_as(P(c_dbl)), _stream()), "mcd_hamiltonian_contract_noalloc")
        return dt, dU, de

    def close(self):
        if self._h:
            lib().mcd_op_destroy(self._h)
            self._h = c_vp(0)
            self._ws.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


@dataclass
class SolveInfo:
    iters: int
    converged: bool
    e0: float
    residual: float
    solve_ms: float
    apply_ms: float
    n_apply: int
    krylov_dim: int
    n_plus: int
    n_minus: int
    n_truncated: int

    @staticmethod
    def of(i: McdSolveInfo) -> "SolveInfo":
        return SolveInfo(i.iters, bool(i.converged), i.e0, i.residual, i.solve_ms, i.apply_ms,
                         i.n_apply, i.krylov_dim, i.n_plus, i.n_minus, i.n_truncated)


def operator_workspace_size(model, keys, storage="auto", grouped=None, mb=None) -> int:
    """Bytes mcd_op_create takes for this model, basis and storage
    (mcd_op_workspace_size; the nonzeros are counted in a probe workspace).
    grouped: include room for the grouped one-vector layout (None: when that
    room, an upper bound, is under half the free device memory)."""
    mb = _ModelBuf(model) if mb is None else mb
    n = int(keys.numel())
    b, bg = ctypes.c_size_t(0), ctypes.c_size_t(0)
    code = lib().mcd_op_workspace_size(ctypes.byref(mb.s), c_vp(keys.data_ptr()), n,
                                       STORAGE[storage], None, _stream(), ctypes.byref(b),
                                       ctypes.byref(bg))
    if code == MCD_E_WORKSPACE:   # the CSR count needs a probe workspace of b bytes
        probe = Workspace(b.value, device=keys.device)
        try:
            code = lib().mcd_op_workspace_size(ctypes.byref(mb.s), c_vp(keys.data_ptr()), n,
                                               STORAGE[storage], probe.handle, _stream(),
                                               ctypes.byref(b), ctypes.byref(bg))
        finally:
            probe.close()
    _check(code, "mcd_op_workspace_size")
    if grouped is None:
        free, _ = _torch().cuda.mem_get_info(keys.device)
        grouped = bg.value < 0.5 * free
    return bg.value if grouped else b.value


def _lanczos_cfg(max_iter, check_every, tol, seed, store_vectors, min_iter, precision):
    return McdLanczosCfg(int(max_iter), int(check_every), float(tol), int(seed),
                         1 if store_vectors else 0, int(min_iter), DTYPE[precision])


def lanczos_ground(op: Operator, max_iter=300, tol=1e-12, seed=0, check_every=10,
                   store_vectors=None, min_iter=1, phi0=None, want_psi=True, precision="f64"):
    """(E0, psi0 tensor or None, alpha, beta, SolveInfo) via mcd_lanczos_ground.
    precision "f32": float32 Krylov vectors, E0 refined by a float64 Rayleigh
    quotient (info.residual = its float64 residual norm).  store_vectors None:
    keep every Krylov vector when that store takes under half the free device
    memory, else run the recurrence a second time for psi0."""
    torch = _torch()
    if store_vectors is None:
        cfg = _lanczos_cfg(max_iter, check_every, tol, seed, True, min_iter, precision)
        need = ctypes.c_size_t(0)
        _check(lib().mcd_lanczos_workspace_size(op.handle, ctypes.byref(cfg), ctypes.byref(need)),
               "mcd_lanczos_workspace_size")
        free, _ = torch.cuda.mem_get_info(op.device)
        store_vectors = need.value < 0.5 * free
    cfg = _lanczos_cfg(max_iter, check_every, tol, seed, store_vectors, min_iter, precision)
    psi = torch.empty(op.n, dtype=torch.float64, device=op.device) if want_psi else None
    e0 = c_dbl(0)
    a = np.zeros(max_iter)
    b = np.zeros(max_iter)
    info = McdSolveInfo()
    need = ctypes.c_size_t(0)
    _check(lib().mcd_lanczos_workspace_size(op.handle, ctypes.byref(cfg), ctypes.byref(need)),
           "mcd_lanczos_workspace_size")
    _with_scratch(lambda ws: lib().mcd_lanczos_ground(
        op.handle, ctypes.byref(cfg), c_vp(phi0.data_ptr()) if phi0 is not None else None,
        ctypes.byref(e0), c_vp(psi.data_ptr()) if want_psi else None,
        a.ctypes.data_as(P(c_dbl)), b.ctypes.data_as(P(c_dbl)), ctypes.byref(info), ws,
        _stream()), "mcd_lanczos_ground", min_bytes=need.value)
    si = SolveInfo.of(info)
    return e0.value, psi, a[: si.iters], b[: si.iters], si


def batch_lanczos_ground(ops, max_iter=400, tol=1e-12, seed=0, check_every=10, min_iter=1,
                         want_psi=True):
    """Ground states of several operators at once (mcd_batch_lanczos_ground).

    Returns (e0 list, psi list or None, iterations list, SolveInfo)."""
    torch = _torch()
    K = len(ops)
    cfg = _lanczos_cfg(max_iter, check_every, tol, seed, True, min_iter, "f64")
    hs = (c_vp * K)(*[op.handle for op in ops])
    psis = [torch.empty(op.n, dtype=torch.float64, device=op.device) for op in ops] if want_psi else None
    pp = (c_vp * K)(*[c_vp(p.data_ptr()) for p in psis]) if want_psi else None
    e0 = (c_dbl * K)()
    it = (c_i32 * K)()
    info = McdSolveInfo()
    ntot = sum(op.n for op in ops)
    est = 8 * (ntot * (min(max_iter, max(op.n for op in ops)) + 3) + K * (2 * max_iter + 8)) + (4 << 20)
    code = _with_scratch(lambda ws: lib().mcd_batch_lanczos_ground(
        hs, K, ctypes.byref(cfg), e0, pp, it, ctypes.byref(info), ws, _stream()),
        "mcd_batch_lanczos_ground", min_bytes=est)
    return list(e0), psis, list(it), SolveInfo.of(info)


def _band_cfg(max_blocks, precision, w_t, dtol, storage, reorth, per_column, eta, g_tol=0.0,
              vjp_freq_batch=0, vjp_chunk=0):
    return McdBandCfg(int(max_blocks), DTYPE[precision], float(w_t), float(dtol),
                      STORAGE[storage], (2 if reorth is True else int(reorth)),
                      1 if per_column else 0, float(eta), float(g_tol), int(vjp_freq_batch),
                      int(vjp_chunk))


class BandKeep:
    """The two sector runs of a forward band_lanczos_green(..., keep=True)
    call (mcd_band_keep: Krylov blocks, T, operators on F~+-), held in their
    own workspace until close() for band_green_vjp(..., keep=...)."""

    def __init__(self, handle, ws):
        self._h = handle
        self._ws = ws

    def close(self):
        if self._h:
            lib().mcd_band_keep_destroy(self._h)
            self._h = None
        if self._ws is not None:
            self._ws.close()
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _band_args(model, keys, psi0, e0, orbitals, spins, omega, cfg):
    mb = _ModelBuf(model)
    orb = np.ascontiguousarray(orbitals, dtype=np.int32)
    sp = np.ascontiguousarray(spins, dtype=np.int32)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    keepalive = (mb, orb, sp, om, cfg)
    args = [ctypes.byref(mb.s), c_vp(keys.data_ptr()), int(keys.numel()), c_vp(psi0.data_ptr()),
            float(e0), len(orb), orb.ctypes.data_as(P(c_i32)), sp.ctypes.data_as(P(c_i32)),
            len(om), om.ctypes.data_as(P(c_dbl)), ctypes.byref(cfg)]
    return args, keepalive, len(orb), len(om)


def band_workspace_size(model, keys, psi0, e0, orbitals, spins, omega, keep=False, **kw) -> int:
    """Bytes mcd_band_lanczos_green(_keep) takes with these arguments
    (mcd_band_workspace_size; the preparation runs in the scratch workspace)."""
    cfg = _band_cfg(kw.get("max_blocks", 50), kw.get("precision", "f64"), kw.get("w_t", 1.0),
                    kw.get("dtol", 1e-10), kw.get("storage", "auto"), kw.get("reorth", 2),
                    kw.get("per_column", False), kw.get("eta", 0.0), kw.get("g_tol", 0.0))
    args, keepalive, _, _ = _band_args(model, keys, psi0, e0, orbitals, spins, omega, cfg)
    out = ctypes.c_size_t(0)
    _with_scratch(lambda ws: lib().mcd_band_workspace_size(*args, 1 if keep else 0, ws, _stream(),
                                                           ctypes.byref(out)),
                  "mcd_band_workspace_size")
    return out.value


def band_lanczos_green(model, keys, psi0, e0, orbitals, spins, omega, max_blocks=50,
                       precision="f64", w_t=1.0, dtol=1e-10, storage="auto", reorth=2,
                       parts=False, per_column=False, eta=0.0, g_tol=0.0, keep=False, ws=None):
    """G [n_freq, n_sel, n_sel] complex128 via mcd_band_lanczos_green.

    eta == 0: omega are Matsubara frequencies (z = i w); eta > 0: real
    frequencies broadened by eta (z = w + i eta).  keep=True calls
    mcd_band_lanczos_green_keep (in a workspace of its own, sized by
    mcd_band_workspace_size) and appends a BandKeep to the returned tuple.
    ws: a Workspace to use instead of the scratch one (no retry)."""
    cfg = _band_cfg(max_blocks, precision, w_t, dtol, storage, reorth, per_column, eta, g_tol)
    args, keepalive, ns, nf = _band_args(model, keys, psi0, e0, orbitals, spins, omega, cfg)
    G = np.zeros((nf, ns, ns), dtype=np.complex128)
    Gp = np.zeros_like(G)
    Gm = np.zeros_like(G)
    info = McdSolveInfo()
    dp = lambda a: a.view(np.float64).ctypes.data_as(P(c_dbl))
    outs = [dp(G), dp(Gp), dp(Gm), ctypes.byref(info)]
    kept = None
    if keep:
        nbytes = band_workspace_size(model, keys, psi0, e0, orbitals, spins, omega, keep=True,
                                     max_blocks=max_blocks, precision=precision, w_t=w_t,
                                     dtol=dtol, storage=storage, reorth=reorth, eta=eta,
                                     g_tol=g_tol)
        kws = Workspace(nbytes, device=keys.device)
        h = c_vp()
        code = lib().mcd_band_lanczos_green_keep(*args, *outs, kws.handle, _stream(),
                                                 ctypes.byref(h))
        if code < 0:
            kws.close()
        _check(code, "mcd_band_lanczos_green_keep")
        kept = BandKeep(h.value, kws)
    elif ws is not None:
        _check(lib().mcd_band_lanczos_green(*args, *outs, ws.handle, _stream()),
               "mcd_band_lanczos_green")
    else:
        _with_scratch(lambda w: lib().mcd_band_lanczos_green(*args, *outs, w, _stream()),
                      "mcd_band_lanczos_green")
    out = (G, Gp, Gm, SolveInfo.of(info)) if parts else (G, SolveInfo.of(info))
    return out + (kept,) if keep else out


def band_green_vjp(model, keys, psi0, e0, orbitals, spins, omega, G_bar, e0_bar=0.0,
                   max_blocks=50, precision="f64", dtol=1e-10, storage="auto", reorth=2, eta=0.0,
                   cg_tol=1e-12, cg_max_iter=20000, g_tol=0.0, keep=None, vjp_freq_batch=0,
                   vjp_chunk=0):
    """(d_t [n_bonds], d_U [n_orb], d_eps [n_orb], SolveInfo) = Re sum conj(G_bar) dG/dtheta
    + e0_bar dE0/dtheta via mcd_band_green_vjp (same arguments as band_lanczos_green), or
    via mcd_band_green_vjp_keep on the runs of a BandKeep.  Without keep and with
    reorth=0 the Krylov blocks are regenerated rather than stored; vjp_freq_batch
    (frequencies per contraction pass, 0 = all) and vjp_chunk (blocks per
    accumulation, 0 = 16) bound the work matrices."""
    cfg = _band_cfg(max_blocks, precision, 1.0, dtol, storage, reorth, False, eta, g_tol,
                    vjp_freq_batch, vjp_chunk)
    args, keepalive, ns, nf = _band_args(model, keys, psi0, e0, orbitals, spins, omega, cfg)
    gb = np.ascontiguousarray(np.asarray(G_bar, dtype=np.complex128).reshape(nf, ns, ns))
    dt = np.zeros(len(model.bonds))
    dU = np.zeros(model.n_orb)
    de = np.zeros(model.n_orb)
    info = McdSolveInfo()
    dp = lambda a: a.ctypes.data_as(P(c_dbl))
    rest = [gb.view(np.float64).ctypes.data_as(P(c_dbl)), float(e0_bar), float(cg_tol),
            int(cg_max_iter), dp(dt), dp(dU), dp(de), ctypes.byref(info)]
    if keep is not None:
        if not keep._h:
            raise ValueError("the BandKeep is closed")
        _with_scratch(lambda w: lib().mcd_band_green_vjp_keep(*args, *rest, w, _stream(),
                                                             c_vp(keep._h)),
                      "mcd_band_green_vjp_keep")
    else:
        _with_scratch(lambda w: lib().mcd_band_green_vjp(*args, *rest, w, _stream()),
                      "mcd_band_green_vjp")
    return dt, dU, de, SolveInfo.of(info)


def batch_band_green(models, keys_list, psi_list, e0_list, orbitals, spins, omega,
                     max_blocks=50, precision="f64", w_t=1.0, dtol=1e-10, storage="auto",
                     reorth=2, eta=0.0, g_tol=0.0, ws=None):
    """[G_i] for many instances at once (mcd_batch_band_green): every run of
    every instance in lockstep; each G_i as band_lanczos_green would return it.
    Returns (list of G, SolveInfo).  ws: a Workspace to use instead of the
    scratch one (no retry; instances then run in groups that fit it)."""
    K = len(models)
    bufs = [_ModelBuf(m) for m in models]
    orb = np.ascontiguousarray(orbitals, dtype=np.int32)
    sp = np.ascontiguousarray(spins, dtype=np.int32)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    ns, nf = len(orb), len(om)
    Gs = [np.zeros((nf, ns, ns), dtype=np.complex128) for _ in range(K)]
    mp = (c_vp * K)(*[ctypes.cast(ctypes.byref(b.s), c_vp) for b in bufs])
    kp = (c_vp * K)(*[c_vp(k.data_ptr()) for k in keys_list])
    nn = (c_i64 * K)(*[int(k.numel()) for k in keys_list])
    pp = (c_vp * K)(*[c_vp(p.data_ptr()) for p in psi_list])
    ee = (c_dbl * K)(*[float(e) for e in e0_list])
    gp = (c_vp * K)(*[c_vp(G.ctypes.data) for G in Gs])
    cfg = _band_cfg(max_blocks, precision, w_t, dtol, storage, reorth, False, eta, g_tol)
    info = McdSolveInfo()
    call = lambda w: lib().mcd_batch_band_green(mp, kp, nn, pp, ee, K, ns,
                                                orb.ctypes.data_as(P(c_i32)),
                                                sp.ctypes.data_as(P(c_i32)), nf,
                                                om.ctypes.data_as(P(c_dbl)), ctypes.byref(cfg),
                                                gp, ctypes.byref(info), w, _stream())
    if ws is not None:
        _check(call(ws.handle), "mcd_batch_band_green")
    else:
        _with_scratch(call, "mcd_batch_band_green")
    return Gs, SolveInfo.of(info)
