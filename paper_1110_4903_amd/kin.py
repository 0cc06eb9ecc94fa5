"""ctypes binding of libkin.so (include/kin.h).  Argument marshalling only: every step of the
kinetics update runs in the library's HIP kernels.

Device arrays may be passed as torch tensors (their data_ptr() is handed over with
KIN_MEM_DEVICE, pinned CPU tensors with KIN_MEM_PINNED), host arrays as numpy arrays; stream
arguments take a torch.cuda.Stream or a raw handle.  Importing this
module loads the shared library and raises ImportError if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libkin.so")

OK, EINVAL, ENOMEM, EBUSY, ENOTFOUND, EDEVICE, ECOMPILE = range(7)
FP64, FP32_LU = 0, 1
MEM_HOST, MEM_DEVICE, MEM_PINNED = 0, 1, 2
LAYOUT_AUTO, LAYOUT_LANE, LAYOUT_WAVE, LAYOUT_GLOBAL = 0, 1, 2, 3
CELL_OK, CELL_OK_HALVED, CELL_FAILED, CELL_BAD_INPUT = 0, 1, 2, 3
Q_BYTES_IN_USE, Q_LAYOUT, Q_BLOCK, Q_NUM_CU, Q_DEVICE_PTRS, Q_JIT_SECONDS, Q_LARGEST_FREE, Q_TUNED = range(8)
# size classes of a launch's cell count (the autotuner's key): below these bounds, and the rest
SIZE_CLASS_BOUNDS = (4096, 16384, 65536, 262144)


def size_class(cells: int) -> int:
    return sum(cells >= b for b in SIZE_CLASS_BOUNDS)

EXPORTS = ("kin_default_solver_opts", "kin_last_error", "kin_create", "kin_destroy",
           "kin_mech_upload", "kin_mech_release", "kin_state_upload", "kin_state_reset",
           "kin_advance", "kin_download", "kin_sync", "kin_instance_release", "kin_footprint",
           "kin_query", "kin_set_layout", "kin_jit_check", "kin_download_schedule", "kin_autotune",
           "kin_stream_create", "kin_stream_destroy", "kin_state_upload_conserved",
           "kin_download_conserved", "kin_state_reset_conserved", "kin_advance_noalloc",
           "kin_advance_trace", "kin_kernel_times", "kin_fluid_create", "kin_fluid_release",
           "kin_fluid_upload", "kin_fluid_download", "kin_fluid_max_dt", "kin_fluid_step",
           "kin_split_step")
BC_PERIODIC, BC_OUTFLOW = 0, 1

if not os.path.exists(SO):
    raise ImportError(f"{SO} is not built: run `python -m paper_1110_4903_amd.build`")
# torch's wheel carries its own HIP runtime under the same soname as the system one.  A process
# must hold only one, so torch is loaded first and the library binds to the runtime it brought.
try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - the library also works without torch
    pass
_lib = C.CDLL(SO)


class KinError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libkin status {status}: {msg}")
        self.status = status


class CtxOpts(C.Structure):
    _fields_ = [("device", C.c_int32), ("hbm_budget", C.c_uint64), ("tune_cache", C.c_char_p),
                ("flags", C.c_uint32)]


CTX_TIME_KERNELS = 1


class MechDesc(C.Structure):
    _fields_ = [("ns", C.c_int32), ("ne", C.c_int32), ("nr", C.c_int32), ("ntb", C.c_int32),
                ("M", C.c_void_p), ("elem", C.c_void_p), ("nasa", C.c_void_p), ("T_mid", C.c_void_p),
                ("reac_idx", C.c_void_p), ("reac_nu", C.c_void_p), ("prod_idx", C.c_void_p),
                ("prod_nu", C.c_void_p), ("A", C.c_void_p), ("b", C.c_void_p), ("Ta", C.c_void_p),
                ("reversible", C.c_void_p), ("tb", C.c_void_p), ("eff", C.c_void_p)]


class SolverOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol_Y", C.c_double), ("atol_T", C.c_double),
                ("y_neg", C.c_double), ("k_max", C.c_int32), ("L_max", C.c_int32),
                ("layout", C.c_int32), ("L_forced", C.c_int32), ("max_iters", C.c_int32),
                ("point_implicit", C.c_int32), ("diverge_ratio", C.c_double)]


_vp, _i32, _i64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
_lib.kin_default_solver_opts.argtypes = [_vp]
_lib.kin_default_solver_opts.restype = None
_lib.kin_last_error.restype = C.c_char_p
_lib.kin_create.argtypes = [_vp, _vp]
_lib.kin_destroy.argtypes = [_vp]
_lib.kin_destroy.restype = None
_lib.kin_mech_upload.argtypes = [_vp, _vp, _vp]
_lib.kin_mech_release.argtypes = [_vp, _i32]
_lib.kin_state_upload.argtypes = [_vp, _i32, _i64, _vp, _vp, _vp, _vp, C.c_int, _vp, _vp]
_lib.kin_state_reset.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, C.c_int, _vp]
_lib.kin_advance.argtypes = [_vp, _vp, _vp, _i32, C.c_int, _vp, _vp]
_lib.kin_advance_noalloc.argtypes = [_vp, _vp, _vp, _i32, C.c_int, _vp, _vp]
_lib.kin_advance_trace.argtypes = [_vp, _i32, C.c_double, C.c_int, _vp, _i32, _vp, _vp]
_lib.kin_kernel_times.argtypes = [_vp, _vp, _i32, _vp]
_lib.kin_fluid_create.argtypes = [_vp, _i32, _i32, _i32, C.c_double, C.c_double, _i32, _vp]
_lib.kin_fluid_release.argtypes = [_vp, _i32]
_lib.kin_fluid_upload.argtypes = [_vp, _i32, _vp, C.c_int, _vp]
_lib.kin_fluid_download.argtypes = [_vp, _i32, _vp, C.c_int, _vp]
_lib.kin_fluid_max_dt.argtypes = [_vp, _i32, C.c_double, _vp, _vp]
_lib.kin_fluid_step.argtypes = [_vp, _i32, C.c_double, _i32, _vp]
_lib.kin_split_step.argtypes = [_vp, _i32, _i32, C.c_double, _i32, C.c_int, _vp, _vp]
_lib.kin_download.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int, _vp]
_lib.kin_sync.argtypes = [_vp, _vp]
_lib.kin_download_schedule.argtypes = [_vp, _i32, _vp, C.c_int, _vp]
_lib.kin_autotune.argtypes = [_vp, _i32, _i32, C.c_double, C.c_int, _vp, _vp, _vp]
_lib.kin_state_upload_conserved.argtypes = [_vp, _i32, _i64, _vp, _vp, _vp, C.c_int, _vp, _vp]
_lib.kin_download_conserved.argtypes = [_vp, _i32, _vp, _vp, C.c_int, _vp]
_lib.kin_state_reset_conserved.argtypes = [_vp, _i32, _vp, _vp, _vp, C.c_int, _vp]
_lib.kin_stream_create.argtypes = [_vp, _i32, _i32, _vp]
_lib.kin_stream_destroy.argtypes = [_vp, _vp]
_lib.kin_instance_release.argtypes = [_vp, _i32]
_lib.kin_footprint.argtypes = [_vp, _i32, _i64, C.c_int, _vp]
_lib.kin_query.argtypes = [_vp, _i32, _i64, _vp]
_lib.kin_set_layout.argtypes = [_vp, _i32, _i32, _i32]
_lib.kin_jit_check.argtypes = [_vp, C.c_char_p, _sz]
for _f in EXPORTS:
    if _f not in ("kin_default_solver_opts", "kin_last_error", "kin_destroy"):
        getattr(_lib, _f).restype = C.c_int


def _check(status: int):
    if status != OK:
        raise KinError(status, _lib.kin_last_error().decode(errors="replace"))


def solver_opts(**kw) -> SolverOpts:
    o = SolverOpts()
    _lib.kin_default_solver_opts(C.byref(o))
    for k, v in kw.items():
        if v is not None:
            setattr(o, k, v)
    return o


class _MechArrays:
    """Contiguous, correctly typed copies of a synth.Mechanism and the descriptor over them."""

    def __init__(self, mech):
        f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
        self.keep = dict(M=f64(mech.M), elem=np.ascontiguousarray(mech.comp, dtype=np.int8),
                         nasa=f64(mech.nasa), T_mid=f64(mech.T_mid),
                         reac_idx=i32(mech.reac_idx), reac_nu=i32(mech.reac_nu),
                         prod_idx=i32(mech.prod_idx), prod_nu=i32(mech.prod_nu),
                         A=f64(mech.A), b=f64(mech.b), Ta=f64(mech.Ta),
                         reversible=i32(mech.reversible), tb=i32(mech.tb),
                         eff=f64(mech.eff if mech.eff.size else np.zeros((1, mech.ns))))
        d = MechDesc()
        d.ns, d.ne, d.nr, d.ntb = mech.ns, mech.ne, mech.nr, mech.ntb
        for k, v in self.keep.items():
            setattr(d, k, v.ctypes.data)
        self.desc = d


def jit_check(mech) -> str:
    """Generate and compile a mechanism's lane-layout kernels with hipRTC (no device needed)."""
    arr = _MechArrays(mech)
    buf = C.create_string_buffer(1 << 16)
    _check(_lib.kin_jit_check(C.byref(arr.desc), buf, len(buf)))
    return buf.value.decode(errors="replace")


def _ptr(x):
    """(address, memory kind) of a numpy array (host) or torch tensor (device, or pinned host)."""
    if x is None:
        return None, None
    if isinstance(x, np.ndarray):
        if not x.flags.c_contiguous or x.dtype not in (np.float64, np.int32):
            raise ValueError("host arrays must be C-contiguous float64/int32")
        return x.ctypes.data, MEM_HOST
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("device tensors must be contiguous")
        if x.is_cuda:
            return x.data_ptr(), MEM_DEVICE
        return x.data_ptr(), (MEM_PINNED if x.is_pinned() else MEM_HOST)
    raise TypeError(f"unsupported array type {type(x)}")


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream  # torch.cuda.Stream


class Context:
    """A libkin context on one GPU."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, tune_cache: Optional[str] = None,
                 time_kernels: bool = False):
        self._h = C.c_void_p()
        o = CtxOpts(device, hbm_budget, tune_cache.encode() if tune_cache else None,
                    CTX_TIME_KERNELS if time_kernels else 0)
        _check(_lib.kin_create(C.byref(self._h), C.byref(o)))
        self.mech_ns = {}
        self.inst_info = {}

    def close(self):
        if self._h:
            _lib.kin_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- mechanisms -------------------------------------------------------------------------
    def mech_upload(self, mech) -> int:
        arr = _MechArrays(mech)
        mid = C.c_int32()
        _check(_lib.kin_mech_upload(self._h, C.byref(arr.desc), C.byref(mid)))
        self.mech_ns[mid.value] = mech.ns
        return mid.value

    def mech_release(self, mech_id: int):
        _check(_lib.kin_mech_release(self._h, mech_id))

    def set_layout(self, mech_id: int, layout: int, block: int):
        _check(_lib.kin_set_layout(self._h, mech_id, layout, block))

    def autotune(self, mech_id: int, inst_id: int, dt: float, prec: int = FP64):
        """Time every admissible (layout, block) on an instance and keep the fastest."""
        lay, blk, ms = C.c_int32(), C.c_int32(), C.c_double()
        _check(_lib.kin_autotune(self._h, mech_id, inst_id, float(dt), prec, C.byref(lay), C.byref(blk),
                                 C.byref(ms)))
        return lay.value, blk.value, ms.value

    # -- instances --------------------------------------------------------------------------
    def state_upload(self, mech_id: int, rho, T, Y, e0=None, stream=None) -> int:
        ns = self.mech_ns[mech_id]
        n = int(rho.shape[0])
        if tuple(Y.shape) != (ns, n) or T.shape[0] != n:
            raise ValueError(f"expected rho[{n}], T[{n}], Y[{ns}][{n}]")
        (pr, kind), (pt, k2), (py, k3) = _ptr(rho), _ptr(T), _ptr(Y)
        pe, k4 = _ptr(e0)
        if len({kind, k2, k3} | ({k4} if e0 is not None else set())) != 1:
            raise ValueError("all state arrays must live in the same memory")
        iid = C.c_int32()
        _check(_lib.kin_state_upload(self._h, mech_id, n, pr, pt, py, pe, kind,
                                     _stream_handle(stream), C.byref(iid)))
        self.inst_info[iid.value] = (mech_id, n, ns)
        return iid.value

    def state_upload_conserved(self, mech_id: int, rho_s, E_sens, T_guess=None, stream=None) -> int:
        """Instance from partial densities rho_s[Ns][n] (kg/m^3) and sensible energy E_sens[n]
        (J/m^3, formation energies at 298.15 K left out); see kin_state_upload_conserved."""
        ns = self.mech_ns[mech_id]
        n = int(E_sens.shape[0])
        if tuple(rho_s.shape) != (ns, n) or (T_guess is not None and T_guess.shape[0] != n):
            raise ValueError(f"expected rho_s[{ns}][{n}], E_sens[{n}], T_guess[{n}]")
        (pr, kind), (pe, k2) = _ptr(rho_s), _ptr(E_sens)
        pt, k3 = _ptr(T_guess)
        if len({kind, k2} | ({k3} if T_guess is not None else set())) != 1:
            raise ValueError("all arrays must live in the same memory")
        iid = C.c_int32()
        _check(_lib.kin_state_upload_conserved(self._h, mech_id, n, pr, pe, pt, kind,
                                               _stream_handle(stream), C.byref(iid)))
        self.inst_info[iid.value] = (mech_id, n, ns)
        return iid.value

    def state_reset_conserved(self, inst_id: int, rho_s, E_sens, T_guess=None, stream=None):
        (pr, kind), (pe, k2) = _ptr(rho_s), _ptr(E_sens)
        pt, k3 = _ptr(T_guess)
        if len({kind, k2} | ({k3} if T_guess is not None else set())) != 1:
            raise ValueError("all arrays must live in the same memory")
        _check(_lib.kin_state_reset_conserved(self._h, inst_id, pr, pe, pt, kind, _stream_handle(stream)))

    def download_conserved(self, inst_id: int):
        """Host copies (rho_s[Ns][n], E_sens[n]) of an instance's state."""
        _, n, ns = self.inst_info[inst_id]
        rho_s = np.empty((ns, n))
        E = np.empty(n)
        _check(_lib.kin_download_conserved(self._h, inst_id, rho_s.ctypes.data, E.ctypes.data, MEM_HOST, None))
        return rho_s, E

    def download_conserved_device(self, inst_id: int, rho_s, E_sens, stream=None):
        """Stream-ordered conversion into torch tensors, both on the device or both pinned."""
        (pr, kind), (pe, k2) = _ptr(rho_s), _ptr(E_sens)
        if kind != k2 or kind == MEM_HOST:
            raise ValueError("destinations must both be device tensors or both pinned host tensors")
        _check(_lib.kin_download_conserved(self._h, inst_id, pr, pe, kind, _stream_handle(stream)))

    def state_reset(self, inst_id: int, rho, T, Y, e0=None, stream=None):
        (pr, kind), (pt, _), (py, _) = _ptr(rho), _ptr(T), _ptr(Y)
        pe, _ = _ptr(e0)
        _check(_lib.kin_state_reset(self._h, inst_id, pr, pt, py, pe, kind, _stream_handle(stream)))

    def advance(self, inst_ids: Sequence[int], dts: Sequence[float], prec: int = FP64,
                opts: Optional[SolverOpts] = None, stream=None):
        ids = np.ascontiguousarray(inst_ids, dtype=np.int32)
        dd = np.ascontiguousarray(dts, dtype=np.float64)
        if ids.shape != dd.shape:
            raise ValueError("one dt per instance")
        _check(_lib.kin_advance(self._h, ids.ctypes.data, dd.ctypes.data, int(ids.shape[0]), prec,
                                C.byref(opts) if opts is not None else None, _stream_handle(stream)))

    def advance_noalloc(self, inst_ids: Sequence[int], dts: Sequence[float], prec: int = FP64,
                        opts: Optional[SolverOpts] = None, stream=None):
        """kin_advance_noalloc: the same step with no device allocation (fixed device memory)."""
        ids = np.ascontiguousarray(inst_ids, dtype=np.int32)
        dd = np.ascontiguousarray(dts, dtype=np.float64)
        if ids.shape != dd.shape:
            raise ValueError("one dt per instance")
        _check(_lib.kin_advance_noalloc(self._h, ids.ctypes.data, dd.ctypes.data, int(ids.shape[0]), prec,
                                        C.byref(opts) if opts is not None else None, _stream_handle(stream)))

    # -- fluid step and operator-split step ---------------------------------------------------
    def fluid_create(self, mech_id: int, nx: int, ny: int, dx: float, dy: float, bc: int = BC_PERIODIC) -> int:
        fid = C.c_int32()
        _check(_lib.kin_fluid_create(self._h, mech_id, nx, ny, float(dx), float(dy), bc, C.byref(fid)))
        self.fluid_info = getattr(self, "fluid_info", {})
        self.fluid_info[fid.value] = (self.mech_ns[mech_id] + 3, ny, nx)
        return fid.value

    def fluid_release(self, fluid_id: int):
        _check(_lib.kin_fluid_release(self._h, fluid_id))

    def fluid_upload(self, fluid_id: int, Q, stream=None):
        p, kind = _ptr(Q)
        _check(_lib.kin_fluid_upload(self._h, fluid_id, p, kind, _stream_handle(stream)))

    def fluid_download(self, fluid_id: int):
        Q = np.empty(self.fluid_info[fluid_id])
        _check(_lib.kin_fluid_download(self._h, fluid_id, Q.ctypes.data, MEM_HOST, None))
        return Q

    def fluid_max_dt(self, fluid_id: int, cfl: float, stream=None) -> float:
        dt = C.c_double()
        _check(_lib.kin_fluid_max_dt(self._h, fluid_id, float(cfl), C.byref(dt), _stream_handle(stream)))
        return dt.value

    def fluid_step(self, fluid_id: int, dt: float, y_first: bool = False, stream=None):
        _check(_lib.kin_fluid_step(self._h, fluid_id, float(dt), int(bool(y_first)), _stream_handle(stream)))

    def split_step(self, fluid_id: int, inst_id: int, dt: float, y_first: bool = False, prec: int = FP64,
                   opts: Optional[SolverOpts] = None, stream=None):
        _check(_lib.kin_split_step(self._h, fluid_id, inst_id, float(dt), int(bool(y_first)), prec,
                                   C.byref(opts) if opts is not None else None, _stream_handle(stream)))

    def kernel_times(self):
        """Durations (ms) of the advance kernels since the last call (kin_kernel_times)."""
        cnt = C.c_int32()
        buf = np.zeros(4096, np.float64)
        _check(_lib.kin_kernel_times(self._h, buf.ctypes.data, buf.shape[0], C.byref(cnt)))
        return buf[:min(cnt.value, buf.shape[0])].tolist()

    def advance_trace(self, inst_id: int, dt: float, prec: int = FP64, opts: Optional[SolverOpts] = None,
                      words: int = 16):
        """kin_advance_trace on the current stream; returns the schedule record as a host array
        [n][words] of uint64 (word 0: attempts, words 1..: accept bits)."""
        import torch
        _, n, _ = self.inst_info[inst_id]
        buf = torch.empty((n, words), dtype=torch.int64, device="cuda")
        _check(_lib.kin_advance_trace(self._h, inst_id, float(dt), prec, C.byref(opts) if opts is not None else None,
                                      int(words), buf.data_ptr(), _stream_handle(torch.cuda.current_stream())))
        torch.cuda.synchronize()
        return buf.cpu().numpy().view(np.uint64)

    def download(self, inst_id: int):
        """Host copies (T, Y, status, level, iters) of an instance."""
        _, n, ns = self.inst_info[inst_id]
        T = np.empty(n)
        Y = np.empty((ns, n))
        st, lv, it = (np.empty(n, np.int32) for _ in range(3))
        _check(_lib.kin_download(self._h, inst_id, T.ctypes.data, Y.ctypes.data, None, st.ctypes.data,
                                 lv.ctypes.data, it.ctypes.data, MEM_HOST, None))
        return T, Y, st, lv, it

    def download_schedule(self, inst_id: int):
        """Host copy of the per-cell sub-step schedule hashes of the last advance."""
        _, n, _ = self.inst_info[inst_id]
        h = np.empty(n, np.uint64)
        _check(_lib.kin_download_schedule(self._h, inst_id, h.ctypes.data, MEM_HOST, None))
        return h

    def download_e0(self, inst_id: int):
        """Host copy of the per-cell internal energy the instance conserves."""
        _, n, ns = self.inst_info[inst_id]
        e0 = np.empty(n)
        _check(_lib.kin_download(self._h, inst_id, None, None, e0.ctypes.data, None, None, None,
                                 MEM_HOST, None))
        return e0

    def download_device(self, inst_id: int, T, Y, e0=None, status=None, level=None, iters=None,
                        stream=None):
        """Stream-ordered copy of an instance's state into torch tensors, all on the device or
        all in pinned host memory; nothing waits for it."""
        arrs = [a for a in (T, Y, e0, status, level, iters) if a is not None]
        kinds = {_ptr(a)[1] for a in arrs}
        if len(kinds) != 1 or kinds == {MEM_HOST}:
            raise ValueError("destinations must all be device tensors or all pinned host tensors")
        ptrs = [(_ptr(a)[0] if a is not None else None) for a in (T, Y, e0, status, level, iters)]
        _check(_lib.kin_download(self._h, inst_id, *ptrs, kinds.pop(), _stream_handle(stream)))

    def stream_create(self, cu_begin: int, cu_end: int) -> int:
        """A raw stream handle whose kernels run on compute units [cu_begin, cu_end)."""
        h = C.c_void_p()
        _check(_lib.kin_stream_create(self._h, cu_begin, cu_end, C.byref(h)))
        return h.value

    def stream_destroy(self, handle: int):
        _check(_lib.kin_stream_destroy(self._h, handle))

    def sync(self, stream=None):
        _check(_lib.kin_sync(self._h, _stream_handle(stream)))

    def instance_release(self, inst_id: int):
        _check(_lib.kin_instance_release(self._h, inst_id))
        self.inst_info.pop(inst_id, None)

    def footprint(self, mech_id: int, n_cells: int, prec: int = FP64) -> int:
        b = C.c_uint64()
        _check(_lib.kin_footprint(self._h, mech_id, n_cells, prec, C.byref(b)))
        return b.value

    # -- queries ----------------------------------------------------------------------------
    def query_int(self, what: int, arg: int = 0) -> int:
        v = C.c_int32()
        _check(_lib.kin_query(self._h, what, arg, C.byref(v)))
        return v.value

    def largest_free(self) -> int:
        v = C.c_uint64()
        _check(_lib.kin_query(self._h, Q_LARGEST_FREE, 0, C.byref(v)))
        return v.value

    def bytes_in_use(self) -> int:
        v = C.c_uint64()
        _check(_lib.kin_query(self._h, Q_BYTES_IN_USE, 0, C.byref(v)))
        return v.value

    def jit_seconds(self, mech_id: int) -> float:
        v = C.c_double()
        _check(_lib.kin_query(self._h, Q_JIT_SECONDS, mech_id, C.byref(v)))
        return v.value

    def tuned(self, mech_id: int):
        """{(precision, size class): (layout, block)} of the autotuned choices of a mechanism."""
        out = np.zeros(20, np.int32)
        _check(_lib.kin_query(self._h, Q_TUNED, mech_id, out.ctypes.data))
        return {(p, c): (int(out[2 * (5 * p + c)]), int(out[2 * (5 * p + c) + 1]))
                for p in range(2) for c in range(5) if out[2 * (5 * p + c)] >= 0}

    def device_ptrs(self, inst_id: int):
        v = (C.c_uint64 * 7)()
        _check(_lib.kin_query(self._h, Q_DEVICE_PTRS, inst_id, v))
        return dict(zip(("rho", "e0", "T", "Y", "status", "level", "iters"), list(v)))
