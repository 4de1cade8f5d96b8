"""Python handles over the C ABI.  Argument marshalling only: no numerics here."""
from __future__ import annotations

import ctypes as C
import weakref

import numpy as np

from . import _lib as L


class QrvieError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qrvie status {status}: {msg}")
        self.status = status


def _torch():
    import torch
    return torch


class Context:
    """A device, a stream (torch's current stream by default) and an HBM budget."""

    def __init__(self, device: int = 0, stream=None, hbm_budget: int = 0):
        torch = _torch()
        self.lib = L.load()
        self.device = device
        if stream is None:
            stream = torch.cuda.Stream(device)      # default priority
        self.stream = stream
        self._children = []                      # weak references to geometries and operators
        h = C.c_void_p()
        st = self.lib.qrvie_ctx_create(device, C.c_void_p(stream.cuda_stream), hbm_budget, C.byref(h))
        if st != L.OK:
            raise QrvieError(st, "ctx_create failed")
        self.h = h

    def order(self):
        """Make the library stream wait for work queued on torch's current stream."""
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def probe_read(self, buf, reps: int = 5) -> float:
        """Best streaming-read rate (GB/s) of the library's read probe over a device tensor."""
        _device_tensor(buf, self.device, "probe read")
        nbytes = buf.numel() * buf.element_size() // 16 * 16
        out = C.c_double()
        self.order()
        self.check(self.lib.qrvie_probe_read(self.h, C.c_void_p(buf.data_ptr()), nbytes, reps, C.byref(out)),
                   "probe read")
        return out.value

    def probe_mfma(self, f64: bool = True) -> float:
        """Measured 16x16x4 matrix-core rate (TFLOP/s), FP64 or FP32."""
        out = C.c_double()
        self.order()
        self.check(self.lib.qrvie_probe_mfma(self.h, 1 if f64 else 0, C.byref(out)), "probe mfma")
        return out.value

    def check(self, st: int, what: str = "") -> int:
        if st not in (L.OK, L.NOT_CONVERGED):
            msg = self.lib.qrvie_last_error(self.h).decode()
            raise QrvieError(st, f"{what}: {msg}")
        return st

    def bytes_in_use(self) -> int:
        return int(self.lib.qrvie_ctx_bytes_in_use(self.h))

    def peak_bytes(self, reset: bool = False) -> int:
        """High-water mark of the library's device bytes on this context (then reset it)."""
        return int(self.lib.qrvie_ctx_peak_bytes(self.h, 1 if reset else 0))

    def _adopt(self, obj):
        if len(self._children) >= 64:
            self._children = [r for r in self._children if r() is not None]
        self._children.append(weakref.ref(obj))

    def close(self):
        """Destroy the context; operators and geometries still open on it are closed first
        (operators before geometries), since the library frees them through the context."""
        if getattr(self, "h", None):
            alive = [r() for r in getattr(self, "_children", [])]
            for o in alive:
                if isinstance(o, Operator):
                    o.close()
            for o in alive:
                if o is not None and not isinstance(o, Operator):
                    o.close()
            self._children = []
            self.lib.qrvie_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def array_desc(array):
    """qrvie_array_desc of an array object, and the numpy buffers it points into (keep them)."""
    keep = dict(
        centers=np.ascontiguousarray(array.centers, dtype=np.float64),
        radius=np.ascontiguousarray(array.radius, dtype=np.float64),
        height=np.ascontiguousarray(array.height, dtype=np.float64),
        eps=np.ascontiguousarray(np.asarray(array.eps_r, dtype=np.complex128).reshape(-1)),
        ij=np.ascontiguousarray(array.lattice_ij if getattr(array, "lattice_ij", None) is not None
                                else np.zeros((len(array.centers), 2)), dtype=np.int32),
    )
    # the library reads n entries of each (n_eps = 1 or n): refuse mismatched lengths here
    n = int(keep["centers"].shape[0]) if keep["centers"].ndim == 2 else -1
    if (keep["centers"].shape != (n, 3) or keep["radius"].shape != (n,) or keep["height"].shape != (n,)
            or keep["ij"].shape != (n, 2) or keep["eps"].shape[0] not in (1, n)):
        raise ValueError("array: expected centers (n, 3), radius (n,), height (n,), lattice_ij (n, 2) and "
                         f"eps_r (1,) or (n,); got {keep['centers'].shape}, {keep['radius'].shape}, "
                         f"{keep['height'].shape}, {keep['ij'].shape}, {keep['eps'].shape}")
    d = L.ArrayDescC()
    d.n = n
    d.centers = _dptr(keep["centers"], C.c_double)
    d.radius = _dptr(keep["radius"], C.c_double)
    d.height = _dptr(keep["height"], C.c_double)
    d.eps_r = keep["eps"].ctypes.data_as(C.POINTER(L.C128))
    d.n_eps = int(keep["eps"].shape[0])
    d.lattice_ij = _dptr(keep["ij"], C.c_int32)
    d.pitch = float(getattr(array, "pitch", 0.0))
    d.wavelength = float(getattr(array, "wavelength", 1.0))
    d.cells_per_particle = int(getattr(array, "cells_per_particle", 48))
    shape = getattr(array, "shape", "disk")
    grid = getattr(array, "grid", "lattice")
    if shape not in ("disk", "sphere") or grid not in ("lattice", "paper"):
        raise ValueError(f"array: shape must be 'disk' or 'sphere' and grid 'lattice' or 'paper', got {shape!r}, {grid!r}")
    d.shape = 0 if shape == "disk" else 1
    d.grid = 0 if grid == "lattice" else 1
    return d, keep


class Geometry:
    """An array of disks: any object with centers, radius, height, eps_r, lattice_ij,
    pitch, wavelength and cells_per_particle attributes (numpy arrays)."""

    def __init__(self, ctx: Context, array):
        self.ctx = ctx
        lib = ctx.lib
        d, self._keep = array_desc(array)
        h = C.c_void_p()
        ctx.check(lib.qrvie_geom_create(ctx.h, C.byref(d), C.byref(h)), "geom_create")
        self.h = h
        ctx._adopt(self)
        self.n_particles = d.n
        self.ndof = int(lib.qrvie_geom_ndof(h))
        self.n_levels = int(lib.qrvie_geom_nlevels(h))

    def order(self) -> np.ndarray:
        out = np.zeros(self.n_particles, dtype=np.int32)
        self.ctx.check(self.ctx.lib.qrvie_geom_order(self.h, _dptr(out, C.c_int32)), "geom_order")
        return out

    def blocks(self) -> np.ndarray:
        """Finest-level grid block (i, j) of each caller particle."""
        out = np.zeros((self.n_particles, 2), dtype=np.int32)
        self.ctx.check(self.ctx.lib.qrvie_geom_blocks(self.h, _dptr(out, C.c_int32)), "geom_blocks")
        return out

    def cells(self):
        c = np.zeros((self.n_particles * 48, 3))
        v = np.zeros(self.n_particles * 48)
        self.ctx.check(self.ctx.lib.qrvie_geom_cells(self.h, _dptr(c, C.c_double), _dptr(v, C.c_double)), "cells")
        return c, v

    def close(self):
        if getattr(self, "h", None):
            if getattr(self.ctx, "h", None):
                self.ctx.lib.qrvie_geom_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _device_tensor(t, device: int, what: str):
    """Refuse anything but a contiguous tensor on cuda:`device`: the library takes its
    address as a raw device pointer."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor, got {type(t).__name__}")
    if not t.is_cuda or t.device.index != device:
        raise ValueError(f"{what}: tensor is on {t.device}, the context on cuda:{device}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")


def _cols(t, n: int, device: int, what: str):
    """(nrhs, n) or (n,) contiguous complex128 tensor on cuda:`device` -> (ptr, ld, nrhs)."""
    torch = _torch()
    _device_tensor(t, device, what)
    if t.dtype != torch.complex128:
        raise TypeError(f"{what}: expected complex128, got {t.dtype}")
    if t.dim() not in (1, 2) or t.shape[-1] != n:
        raise ValueError(f"{what}: expected shape (nrhs, {n}) or ({n},), got {tuple(t.shape)}")
    nrhs = 1 if t.dim() == 1 else t.shape[0]
    return C.c_void_p(t.data_ptr()), n, nrhs


def assemble(ctx: Context, geom: Geometry, rows, cols):
    """Dense block of Z for caller particle lists rows x cols -> (144*len(rows)) x (144*len(cols))
    device tensor (returned transposed view of the column-major buffer)."""
    torch = _torch()
    r = np.ascontiguousarray(rows, dtype=np.int32)
    c = np.ascontiguousarray(cols, dtype=np.int32)
    m, n = 144 * r.size, 144 * c.size
    buf = torch.empty((n, m), dtype=torch.complex128, device=f"cuda:{ctx.device}")
    ctx.order()
    ctx.check(ctx.lib.qrvie_assemble(ctx.h, geom.h, r.size, _dptr(r, C.c_int32), c.size, _dptr(c, C.c_int32),
                                     C.c_void_p(buf.data_ptr()), m), "assemble")
    return buf.t()


def rhs_plane_waves(ctx: Context, geom: Geometry, theta_deg, phi_deg, pol):
    torch = _torch()
    th = np.ascontiguousarray(np.atleast_1d(theta_deg), dtype=np.float64)
    ph = np.ascontiguousarray(np.atleast_1d(phi_deg), dtype=np.float64)
    po = np.ascontiguousarray(np.atleast_1d(pol), dtype=np.int32)
    v = torch.empty((th.size, geom.ndof), dtype=torch.complex128, device=f"cuda:{ctx.device}")
    ctx.order()
    ctx.check(ctx.lib.qrvie_rhs_plane_waves(ctx.h, geom.h, th.size, _dptr(th, C.c_double), _dptr(ph, C.c_double),
                                            _dptr(po, C.c_int32), C.c_void_p(v.data_ptr()), geom.ndof), "rhs")
    return v


def _compression(name: str) -> int:
    """'aca' (cross approximation, the default) or 'sketch' (assembled blocks, randomised sketch)."""
    try:
        return {"aca": 0, "sketch": 1}[name]
    except KeyError:
        raise ValueError(f"compression must be 'sketch' or 'aca', not {name!r}") from None


class Operator:
    """The compressed interaction operator Z_QR with its block-diagonal preconditioner."""

    def __init__(self, ctx: Context, geom: Geometry, eps: float = 1e-6, max_block_rows: int = 0, seed: int = 0,
                 far_prec: int = L.PREC_C128, verbose: bool = False, chunk_bytes: int = 0,
                 share_transpose: bool = False, compression: str = "aca", aca_start: int = 0,
                 aca_stop: float = 0.0):
        self.ctx, self.geom, self.far_prec = ctx, geom, far_prec
        self.shared = bool(share_transpose)
        o = L.CompressOpts(eps=eps, far_prec=far_prec, near_prec=L.PREC_C128, max_block_rows=max_block_rows,
                           share_transpose=1 if share_transpose else 0, seed=seed, verbose=1 if verbose else 0,
                           chunk_bytes=chunk_bytes, compression=_compression(compression), aca_start=aca_start,
                           aca_stop=aca_stop)
        self.opts = o
        h = C.c_void_p()
        ctx.check(ctx.lib.qrvie_op_create(ctx.h, geom.h, C.byref(o), C.byref(h)), "op_create")
        self.h = h
        ctx._adopt(self)

    @staticmethod
    def footprint_estimate(geom: Geometry, eps: float = 1e-6, max_block_rows: int = 0, far_prec: int = L.PREC_C128,
                           chunk_bytes: int = 0, share_transpose: bool = False, compression: str = "aca",
                           aca_start: int = 0) -> int:
        o = L.CompressOpts(eps=eps, far_prec=far_prec, max_block_rows=max_block_rows, chunk_bytes=chunk_bytes,
                           share_transpose=1 if share_transpose else 0, compression=_compression(compression),
                           aca_start=aca_start)
        out = C.c_size_t()
        st = geom.ctx.lib.qrvie_op_footprint_estimate(geom.h, C.byref(o), C.byref(out))
        geom.ctx.check(st, "footprint")
        return int(out.value)

    @staticmethod
    def solve_footprint_estimate(geom: Geometry, nrhs: int, restart: int, max_iter: int, op=None,
                                 mode: int = L.SOLVE_FP64) -> int:
        o = L.SolveOpts(restart=restart, max_iter=max_iter, mode=mode, tol=1e-6, use_x0=0)
        out = C.c_size_t()
        st = geom.ctx.lib.qrvie_solve_footprint_estimate(geom.h, op.h if op is not None else None, nrhs,
                                                         C.byref(o), C.byref(out))
        geom.ctx.check(st, "solve footprint")
        return int(out.value)

    def stats(self) -> dict:
        s = L.OpStats()
        self.ctx.check(self.ctx.lib.qrvie_op_stats_get(self.h, C.byref(s)), "stats")
        nl = s.n_levels + 1
        return dict(n_levels=s.n_levels, n_blocks=s.n_blocks, n_blocks_level=list(s.n_blocks_level[:nl]),
                    min_rank_level=list(s.min_rank_level[:nl]), max_rank_level=list(s.max_rank_level[:nl]),
                    mean_rank_level=list(s.mean_rank_level[:nl]), n_self_types=s.n_self_types,
                    n_qr_entries=s.n_qr_entries, gain=s.gain, max_block_rel_err=s.max_block_rel_err,
                    apply_bytes=s.apply_bytes, apply_bytes_c64=s.apply_bytes_c64, device_bytes=s.device_bytes,
                    t_compression_s=s.t_compression_s, t_precond_setup_s=s.t_precond_setup_s,
                    n_aca=s.n_aca, n_aca_resumed=s.n_aca_resumed, n_aca_retried=s.n_aca_retried,
                    n_aca_sketch=s.n_aca_sketch)

    def num_blocks(self) -> int:
        return int(self.ctx.lib.qrvie_op_num_blocks(self.h))

    def export_block(self, b: int, factors: bool = True):
        info = L.BlockInfo()
        self.ctx.check(self.ctx.lib.qrvie_op_export_block(self.h, b, C.byref(info), None, None), "export")
        Q = R = None
        if factors and info.rank > 0:
            Qb = np.zeros(info.m * info.rank, dtype=np.complex128)
            Rb = np.zeros(info.rank * info.n, dtype=np.complex128)
            self.ctx.check(self.ctx.lib.qrvie_op_export_block(self.h, b, C.byref(info), C.c_void_p(Qb.ctypes.data),
                                                              C.c_void_p(Rb.ctypes.data)), "export")
            Q = Qb.reshape(info.rank, info.m).T
            R = Rb.reshape(info.n, info.rank).T
        d = {f: getattr(info, f) for f, _ in L.BlockInfo._fields_}
        return d, Q, R

    def export_self(self, p: int):
        Z = np.zeros(144 * 144, dtype=np.complex128)
        Zi = np.zeros(144 * 144, dtype=np.complex128)
        self.ctx.check(self.ctx.lib.qrvie_op_export_self(self.h, p, C.c_void_p(Z.ctypes.data),
                                                         C.c_void_p(Zi.ctypes.data)), "export_self")
        return Z.reshape(144, 144).T, Zi.reshape(144, 144).T

    def apply(self, x, prec=None):
        """y = Z_QR x with the operator's own far factors, or those of precision `prec`."""
        torch = _torch()
        px, ld, nrhs = _cols(x, self.geom.ndof, self.ctx.device, "apply")
        y = torch.empty_like(x)
        self.ctx.order()
        if prec is None:
            st = self.ctx.lib.qrvie_apply(self.ctx.h, self.h, nrhs, px, ld, C.c_void_p(y.data_ptr()), ld)
        else:
            st = self.ctx.lib.qrvie_apply_prec(self.ctx.h, self.h, prec, nrhs, px, ld, C.c_void_p(y.data_ptr()), ld)
        self.ctx.check(st, "apply")
        return y

    def apply_noalloc(self, x, y):
        """y = Z_QR x for one vector into the caller's y, with the library's fixed scratch
        (no device allocation, asynchronous on the context stream)."""
        px, _, nrhs = _cols(x, self.geom.ndof, self.ctx.device, "apply_noalloc x")
        py, _, nry = _cols(y, self.geom.ndof, self.ctx.device, "apply_noalloc y")
        if nrhs != 1 or nry != 1:
            raise ValueError("apply_noalloc: one vector of shape (n,) or (1, n)")
        self.ctx.order()
        self.ctx.check(self.ctx.lib.qrvie_apply_noalloc(self.ctx.h, self.h, px, py), "apply_noalloc")
        return y

    def profile_apply(self, reps: int = 10, prec: int = L.PREC_C128) -> dict:
        """Per-stage device time (ms) and algorithmic bytes of one single-RHS product."""
        ms = (C.c_double * 6)()
        by = (C.c_int64 * 6)()
        self.ctx.order()
        self.ctx.check(self.ctx.lib.qrvie_op_profile_apply(self.ctx.h, self.h, prec, reps, ms, by), "profile")
        names = ("rphase", "qphase", "final", "product", "qtphase")
        return {k: dict(ms=ms[i], bytes=by[i]) for i, k in enumerate(names)}

    def profile_block(self, nrhs: int = 64, reps: int = 5) -> dict:
        """Per-stage device time (ms) and flops of one block product of nrhs right-hand sides."""
        ms = (C.c_double * 4)()
        fl = (C.c_int64 * 4)()
        self.ctx.order()
        self.ctx.check(self.ctx.lib.qrvie_op_profile_block(self.ctx.h, self.h, nrhs, reps, ms, fl), "profile block")
        names = ("rphase", "qphase", "self", "precond")
        return {k: dict(ms=ms[i], flops=fl[i]) for i, k in enumerate(names)}

    def tune_block(self, nrhs: int = 64, reps: int = 5, prec: int = None) -> dict:
        """Autotune the block product's tile shape per strip group (R panels, Q panels, self
        blocks) for nrhs right-hand sides; the operator keeps the fastest bitwise-identical
        shape.  Returns the per-variant timings, mismatch counts and the choices."""
        if prec is None:
            prec = L.PREC_C128 if self.far_prec != L.PREC_C64_ONLY else L.PREC_C64
        t = L.BlockTune()
        self.ctx.order()
        self.ctx.check(self.ctx.lib.qrvie_op_tune_block(self.ctx.h, self.h, prec, nrhs, reps, C.byref(t)),
                       "tune block")
        nv = t.n_variants
        groups = ("rphase", "qphase", "self")
        return {
            "nrhs_tile": t.nrhs_tile,
            "variants": [dict(u=t.u[v], rows_per_wave=t.rows_per_wave[v]) for v in range(nv)],
            "ms": {g: [t.ms[i][v] for v in range(nv)] for i, g in enumerate(groups)},
            "mismatches": {g: [t.mismatches[i][v] for v in range(nv)] for i, g in enumerate(groups)},
            "chosen": {g: t.chosen[i] for i, g in enumerate(groups)},
        }

    def precondition(self, y):
        torch = _torch()
        py, ld, nrhs = _cols(y, self.geom.ndof, self.ctx.device, "precondition")
        z = torch.empty_like(y)
        self.ctx.order()
        self.ctx.check(self.ctx.lib.qrvie_precondition(self.ctx.h, self.h, nrhs, py, ld, C.c_void_p(z.data_ptr()), ld),
                       "precondition")
        return z

    def solve(self, v, restart: int = 30, tol: float = 1e-8, max_iter: int = 10000, x0=None,
              mode: int = L.SOLVE_FP64, inner_tol: float = 0.0, verbose: bool = False, block_width: int = 0,
              inner_fp32: bool = False):
        torch = _torch()
        pv, ld, nrhs = _cols(v, self.geom.ndof, self.ctx.device, "solve")
        if x0 is not None:
            _cols(x0, self.geom.ndof, self.ctx.device, "solve x0")
            if x0.shape != v.shape:
                raise ValueError(f"solve: x0 has shape {tuple(x0.shape)}, v {tuple(v.shape)}")
        x = torch.zeros_like(v) if x0 is None else x0.clone()
        o = L.SolveOpts(restart=restart, max_iter=max_iter, mode=mode, tol=tol, use_x0=0 if x0 is None else 1,
                        inner_tol=inner_tol, verbose=1 if verbose else 0, block_width=block_width,
                        inner_fp32=1 if inner_fp32 else 0)
        infos = (L.SolveInfo * nrhs)()
        self.ctx.order()
        st = self.ctx.check(self.ctx.lib.qrvie_solve(self.ctx.h, self.h, nrhs, pv, ld, C.c_void_p(x.data_ptr()), ld,
                                                     C.byref(o), infos), "solve")
        out = [{f: getattr(i, f) for f, _ in L.SolveInfo._fields_} for i in infos]
        return x, out, st

    def close(self):
        if getattr(self, "h", None):
            if getattr(self.ctx, "h", None):
                self.ctx.lib.qrvie_op_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
