"""Thin ctypes binding of the HIP library (include/rve.h); argument marshalling only.

Every step of the solve runs in the library's HIP kernels.  Device buffers are
passed as torch CUDA (HIP) tensors through their data_ptr(); PyTorch is used only
for device memory and streams.  Importing this module fails loudly when the
built library is missing.
"""
import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librve.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "rve.h")

RVE_OK, RVE_EPARTIAL, RVE_EINVAL, RVE_ENOMEM, RVE_EHIP, RVE_EUNSUPPORTED = 0, 1, -1, -2, -3, -4
S_CONVERGED, S_NOCONV, S_DETF, S_SINGULAR, S_NONFINITE = 0, 1, 2, 3, 4
PREC_FP64, PREC_FP32_IR = 0, 1
LAW_NEOHOOKE, LAW_SVK, LAW_LINEAR = 0, 1, 2
BC_PERIODIC, BC_LINEAR = 0, 1
ELEM_Q1, ELEM_P1 = 0, 1
FLAG_OUTPUTS_AT_CAP, FLAG_DIRECT_TANGENT = 1, 2


class RveError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class MeshDesc(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32), ("nphase", C.c_int32), ("lame", C.c_void_p),
                ("phase", C.c_void_p), ("incl_center", C.c_double * 3), ("incl_radius", C.c_double),
                ("incl_phase", C.c_int32), ("law", C.c_int32), ("bc", C.c_int32),
                ("elem", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32),
                ("det_backtrack", C.c_int32), ("flags", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("leaf", C.c_int32), ("wave_max_m", C.c_int32), ("slots", C.c_int32), ("threads", C.c_int32),
                ("ms", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        # torch ships its own HIP/HSA runtime; loading it first makes the
        # library's libamdhip64 dependency resolve to that same runtime, so the
        # process holds one HIP runtime whichever module touches the GPU first
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.rve_lame.argtypes = [dp, dp, C.POINTER(dp), C.POINTER(dp)]
        L.rve_mesh_create.argtypes = [C.POINTER(MeshDesc), C.POINTER(vp)]
        L.rve_mesh_destroy.argtypes = [vp]
        L.rve_mesh_get_phase.argtypes = [vp, vp]
        L.rve_batch_create.argtypes = [vp, i64, C.POINTER(vp)]
        L.rve_batch_destroy.argtypes = [vp]
        L.rve_batch_state_offsets.argtypes = [vp, vp]
        L.rve_opts_default.argtypes = [C.POINTER(Opts)]
        L.rve_opts_default.restype = None
        L.rve_solve_batch.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.POINTER(Opts), vp]
        L.rve_solve_batch_sync.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.POINTER(Opts), vp]
        L.rve_solve_batch_subset.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(Opts), vp]
        L.rve_solve_batch_static.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.POINTER(Opts), vp]
        L.rve_probe_peaks.argtypes = [C.POINTER(dp), C.POINTER(dp), C.POINTER(dp), vp]
        L.rve_assemble_batch.argtypes = [vp, vp, vp, vp, vp]
        L.rve_plan_info.argtypes = [i32, i32, C.POINTER(dp), C.POINTER(i64), C.POINTER(i32), C.POINTER(i32)]
        L.rve_plan_export.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp, vp]
        L.rve_plan_schedule.argtypes = [i32, i32, vp, vp, vp]
        L.rve_strerror.argtypes = [C.c_int]
        L.rve_strerror.restype = C.c_char_p
        L.rve_last_error.argtypes = [C.c_char_p, C.c_size_t]
        L.rve_autotune.argtypes = [vp, vp, i64, C.POINTER(Opts), C.POINTER(Tuning), vp]
        L.rve_tuning_get.argtypes = [i32, i32, C.POINTER(Tuning)]
        L.rve_tuning_set.argtypes = [i32, i32, C.POINTER(Tuning)]
        L.rve_tuning_reset.argtypes = [i32, i32]
        _lib = L
    return _lib


def declared_functions():
    """Names of the functions declared in include/rve.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?(?:int|void|char|int64_t|double)\s*\*?\s*(rve_\w+)\s*\(",
                                 txt, flags=re.M)))


def last_error():
    buf = C.create_string_buffer(1024)
    lib().rve_last_error(buf, 1024)
    return buf.value.decode()


def check(code, what=""):
    if code < 0:
        raise RveError(code, f"{what}: {lib().rve_strerror(code).decode()}: {last_error()}")
    return code


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data_as(C.c_void_p)
    return C.c_void_p(t.data_ptr())


def lame(E, nu):
    la, mu = C.c_double(), C.c_double()
    check(lib().rve_lame(E, nu, C.byref(la), C.byref(mu)), "rve_lame")
    return la.value, mu.value


def two_phase_lame(ratio, E=1.0, nu=0.3):
    return np.array([lame(E, nu), lame(ratio * E, nu)], dtype=np.float64)


def _tuning_dict(t):
    return dict(leaf=t.leaf, wave_max_m=t.wave_max_m, slots=t.slots, threads=t.threads, ms=t.ms)


def tuning_get(d, n):
    t = Tuning()
    check(lib().rve_tuning_get(d, n, C.byref(t)), "rve_tuning_get")
    return _tuning_dict(t)


def tuning_set(d, n, leaf=0, wave_max_m=64, slots=0, threads=0):
    t = Tuning(leaf, wave_max_m, slots, threads, 0.0)
    check(lib().rve_tuning_set(d, n, C.byref(t)), "rve_tuning_set")


def tuning_reset(d=0, n=0):
    check(lib().rve_tuning_reset(d, n), "rve_tuning_reset")


def autotune(mesh, F, opts=None, stream=None):
    """Times the candidate plans / launch shapes on F (device float64 [nF, d^2])
    and keeps the fastest for (mesh.d, mesh.n); returns the choice."""
    import torch
    if not isinstance(F, torch.Tensor) or not F.is_cuda or F.dtype != torch.float64 or not F.is_contiguous():
        raise ValueError("F: expected a contiguous float64 GPU tensor")
    nF = F.numel() // (mesh.d * mesh.d)
    t = Tuning()
    o = opts if opts is not None else default_opts()
    check(lib().rve_autotune(mesh.h, _ptr(F), nF, C.byref(o), C.byref(t), C.c_void_p(stream) if stream else None),
          "rve_autotune")
    return _tuning_dict(t)


def probe_peaks(stream=None):
    """Measured FP64 / FP32 MFMA TFLOP/s and HBM copy GB/s of the current device."""
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    check(lib().rve_probe_peaks(C.byref(a), C.byref(b), C.byref(c), C.c_void_p(stream) if stream else None),
          "rve_probe_peaks")
    return dict(fp64_mfma_tflops=a.value, fp32_mfma_tflops=b.value, hbm_copy_gbs=c.value)


def plan_info(d, n):
    f, nnz, nf, mf = C.c_double(), C.c_int64(), C.c_int32(), C.c_int32()
    check(lib().rve_plan_info(d, n, C.byref(f), C.byref(nnz), C.byref(nf), C.byref(mf)), "rve_plan_info")
    return dict(factor_flops=f.value, nnz_L=nnz.value, nfronts=nf.value, max_front=mf.value)


def plan_schedule(d, n):
    """Workgroup-front steps [nsteps, 4] (1, 2 or 4 fronts side by side, -1
    padded) and the per-front wave-phase flags of the (d, n) plan."""
    ns = np.zeros(1, np.int64)
    check(lib().rve_plan_schedule(d, n, _ptr(ns), None, None), "rve_plan_schedule")
    nf = plan_info(d, n)["nfronts"]
    steps = np.zeros((int(ns[0]), 4), np.int32)
    wave = np.zeros(nf, np.int32)
    check(lib().rve_plan_schedule(d, n, _ptr(ns), _ptr(steps), _ptr(wave)), "rve_plan_schedule")
    return dict(steps=steps, wave=wave)


def plan_export(d, n):
    sizes = np.zeros(6, np.int64)
    check(lib().rve_plan_export(d, n, _ptr(sizes), None, None, None, None, None, None), "rve_plan_export")
    fr = np.zeros((sizes[0], 8), np.int32)
    rows = np.zeros(sizes[1], np.int32)
    rel = np.zeros(sizes[2], np.int32)
    ch = np.zeros(sizes[3], np.int32)
    kp = np.zeros((sizes[4], 4), np.int32)
    kc = np.zeros((sizes[5], 3), np.int32)
    check(lib().rve_plan_export(d, n, _ptr(sizes), _ptr(fr), _ptr(rows), _ptr(rel), _ptr(ch), _ptr(kp), _ptr(kc)),
          "rve_plan_export")
    return dict(fronts=fr, rows=rows, relind=rel, children=ch, kpair=kp, kcontrib=kc)


class Mesh:
    """rve_mesh handle: phase field by explicit array or centred inclusion."""

    def __init__(self, d, n, lame_tab, phase=None, radius=0.0, center=None, incl_phase=1, law=LAW_NEOHOOKE,
                 bc=BC_PERIODIC, elem=ELEM_Q1):
        self._lame = np.ascontiguousarray(lame_tab, np.float64)
        self._phase = None if phase is None else np.ascontiguousarray(phase, np.uint8)
        c = center if center is not None else [0.5, 0.5, 0.5]
        desc = MeshDesc(d, n, self._lame.shape[0], self._lame.ctypes.data_as(C.c_void_p),
                        None if self._phase is None else self._phase.ctypes.data_as(C.c_void_p),
                        (C.c_double * 3)(*[float(x) for x in list(c) + [0.5] * (3 - len(c))]), float(radius),
                        incl_phase, int(law), int(bc), int(elem))
        h = C.c_void_p()
        check(lib().rve_mesh_create(C.byref(desc), C.byref(h)), "rve_mesh_create")
        self.h, self.d, self.n, self.law, self.bc, self.elem = h, d, n, law, bc, elem

    def phase(self):
        out = np.zeros(self.n ** self.d, np.uint8)
        check(lib().rve_mesh_get_phase(self.h, _ptr(out)), "rve_mesh_get_phase")
        return out

    def destroy(self):
        if self.h is not None:
            check(lib().rve_mesh_destroy(self.h), "rve_mesh_destroy")
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def default_opts(**kw):
    o = Opts()
    lib().rve_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Batch:
    """rve_batch handle over a list of Mesh objects (kept alive by the batch)."""

    def __init__(self, meshes):
        self.meshes = list(meshes)
        arr = (C.c_void_p * len(self.meshes))(*[m.h.value for m in self.meshes])
        h = C.c_void_p()
        check(lib().rve_batch_create(arr, len(self.meshes), C.byref(h)), "rve_batch_create")
        self.h = h
        self.B = len(self.meshes)
        self.d = self.meshes[0].d
        off = np.zeros(self.B + 1, np.int64)
        check(lib().rve_batch_state_offsets(self.h, _ptr(off)), "rve_batch_state_offsets")
        self.state_offsets = off

    def _check(self, t, numel, dtype, name):
        import torch
        if t is None:
            return
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError(f"{name}: expected a GPU tensor")
        if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
            raise ValueError(f"{name}: expected contiguous {dtype} with {numel} elements, got "
                             f"{t.dtype} {tuple(t.shape)} contiguous={t.is_contiguous()}")

    def solve(self, F, P, A=None, w_state=None, status=None, iters=None, opts=None, stream=None, sync=False,
              static=False):
        """All tensors on the GPU (float64 / int32), contiguous; sizes are checked
        here because the C ABI receives bare device pointers.  static=True calls
        rve_solve_batch_static (workspace in the library's static device array)."""
        import torch
        d2 = self.d * self.d
        self._check(F, self.B * d2, torch.float64, "F")
        self._check(P, self.B * d2, torch.float64, "P")
        self._check(A, self.B * d2 * d2, torch.float64, "A")
        self._check(w_state, int(self.state_offsets[-1]), torch.float64, "w_state")
        self._check(status, self.B, torch.int32, "status")
        self._check(iters, self.B, torch.int32, "iters")
        if F is None or P is None:
            raise ValueError("F and P are required")
        o = opts if opts is not None else default_opts()
        s = C.c_void_p(stream) if stream is not None else None
        if static and sync:
            raise ValueError("static and sync are exclusive")
        fn = lib().rve_solve_batch_static if static else (lib().rve_solve_batch_sync if sync else lib().rve_solve_batch)
        return check(fn(self.h, _ptr(F), _ptr(P), _ptr(A), _ptr(w_state), _ptr(status), _ptr(iters),
                        C.byref(o), s), "rve_solve_batch_static" if static else "rve_solve_batch")

    def assemble(self, F, w_state=None, status=None, stream=None):
        """One assembly (element pass + residual gather) of every RVE, alone
        (rve_assemble_batch)."""
        import torch
        d2 = self.d * self.d
        self._check(F, self.B * d2, torch.float64, "F")
        self._check(w_state, int(self.state_offsets[-1]), torch.float64, "w_state")
        self._check(status, self.B, torch.int32, "status")
        s = C.c_void_p(stream) if stream is not None else None
        return check(lib().rve_assemble_batch(self.h, _ptr(F), _ptr(w_state), _ptr(status), s), "rve_assemble_batch")

    def solve_subset(self, idx, count, F, P, A=None, w_state=None, status=None, iters=None, opts=None, stream=None):
        """Solves only the RVEs idx[0 .. count[0]) (device int32 tensors)."""
        import torch
        d2 = self.d * self.d
        self._check(idx, idx.numel(), torch.int32, "idx")
        self._check(count, 1, torch.int32, "count")
        if idx.numel() > self.B:
            raise ValueError("idx: more entries than RVEs")
        self._check(F, self.B * d2, torch.float64, "F")
        self._check(P, self.B * d2, torch.float64, "P")
        self._check(A, self.B * d2 * d2, torch.float64, "A")
        self._check(w_state, int(self.state_offsets[-1]), torch.float64, "w_state")
        self._check(status, self.B, torch.int32, "status")
        self._check(iters, self.B, torch.int32, "iters")
        o = opts if opts is not None else default_opts()
        s = C.c_void_p(stream) if stream is not None else None
        return check(lib().rve_solve_batch_subset(self.h, _ptr(idx), _ptr(count), _ptr(F), _ptr(P), _ptr(A),
                                                  _ptr(w_state), _ptr(status), _ptr(iters), C.byref(o), s),
                     "rve_solve_batch_subset")

    def destroy(self):
        if self.h is not None:
            check(lib().rve_batch_destroy(self.h), "rve_batch_destroy")
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
