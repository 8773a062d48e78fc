"""ctypes binding of the two-scale driver (include/fehmm.h); marshalling only."""
import ctypes as C
import os
import re

import numpy as np

from . import rve

HEADER = os.path.join(os.path.dirname(rve.HERE), "include", "fehmm.h")
BC_CLAMPED_PULL, BC_UNIAXIAL = 0, 1
NESTED, ALTERNATING = 0, 1
ELEM_Q1, ELEM_P1 = 0, 1
STEP_CONVERGED, STEP_NOCONV, STEP_RVE_FAILED = 0, 1, 2
MAX_HIST = 64


class Desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("Lx", C.c_double), ("Ly", C.c_double),
                ("hole_r", C.c_double), ("bc", C.c_int32), ("stretch", C.c_double), ("nsteps", C.c_int32),
                ("rtol_macro", C.c_double), ("max_macro_iter", C.c_int32), ("scheme", C.c_int32),
                ("micro", C.c_void_p), ("micro_opts", rve.Opts), ("elem", C.c_int32)]


class StepInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("macro_iters", C.c_int32), ("micro_iters", C.c_int64),
                ("res_hist", C.c_double * MAX_HIST), ("u_max", C.c_double), ("failed_rves", C.c_int32),
                ("surrogate_points", C.c_int64), ("fallback_points", C.c_int64)]


_setup_done = False


def lib():
    global _setup_done
    L = rve.lib()
    if not _setup_done:
        vp = C.c_void_p
        L.fehmm_create.argtypes = [C.POINTER(Desc), C.POINTER(vp)]
        L.fehmm_destroy.argtypes = [vp]
        L.fehmm_sizes.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.fehmm_macro_step.argtypes = [vp, C.c_int32, C.POINTER(StepInfo)]
        L.fehmm_get_nodes.argtypes = [vp, vp]
        L.fehmm_get_u.argtypes = [vp, vp]
        L.fehmm_get_qp.argtypes = [vp, vp, vp, vp]
        L.fehmm_get_state.argtypes = [vp, vp, vp]
        L.fehmm_set_state.argtypes = [vp, vp, vp]
        L.fehmm_set_surrogate.argtypes = [vp, vp, C.c_float, C.c_int32, C.c_double]
        L.fehmm_set_graph.argtypes = [vp, C.c_int32]
        _setup_done = True
    return L


def declared_functions():
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"^\s*int\s+(fehmm_\w+)\s*\(", txt, flags=re.M)))


class Driver:
    """FE-HMM macro driver over one RVE mesh (kept alive by the driver)."""

    def __init__(self, mesh, nx, ny, Lx=1.0, Ly=1.0, hole_r=0.0, bc=BC_CLAMPED_PULL, stretch=1.1, nsteps=10,
                 rtol_macro=1e-10, max_macro_iter=30, scheme=NESTED, micro_opts=None, elem=ELEM_Q1):
        self.mesh = mesh
        o = micro_opts if micro_opts is not None else rve.default_opts()
        self.desc = Desc(nx, ny, Lx, Ly, hole_r, bc, stretch, nsteps, rtol_macro, max_macro_iter, scheme,
                         mesh.h.value, o, int(elem))
        h = C.c_void_p()
        rve.check(lib().fehmm_create(C.byref(self.desc), C.byref(h)), "fehmm_create")
        self.h = h
        nd, nq, ns = C.c_int32(), C.c_int32(), C.c_int64()
        rve.check(lib().fehmm_sizes(self.h, C.byref(nd), C.byref(nq), C.byref(ns)), "fehmm_sizes")
        self.ndof, self.nqp, self.state_doubles = nd.value, nq.value, ns.value

    def step(self, k):
        info = StepInfo()
        code = lib().fehmm_macro_step(self.h, k, C.byref(info))
        rve.check(code, "fehmm_macro_step")
        return dict(code=code, status=info.status, macro_iters=info.macro_iters, micro_iters=info.micro_iters,
                    res_hist=np.array(info.res_hist[: info.macro_iters + 1]), u_max=info.u_max,
                    failed_rves=info.failed_rves, surrogate_points=info.surrogate_points,
                    fallback_points=info.fallback_points)

    def set_surrogate(self, surrogate, threshold=1e-3, precision=1, macro_rtol=1e-4):
        """Use a trained surrogate (paper_1908_08292_amd.surrogate.Surrogate) where its
        indicator is <= threshold; None switches it off."""
        self._surrogate = surrogate
        rve.check(lib().fehmm_set_surrogate(self.h, surrogate.h if surrogate is not None else None,
                                            float(threshold), int(precision), float(macro_rtol)),
                  "fehmm_set_surrogate")

    def set_graph(self, enable=True):
        """Run each load step as one captured HIP graph (fehmm_set_graph)."""
        rve.check(lib().fehmm_set_graph(self.h, 1 if enable else 0), "fehmm_set_graph")

    def u(self):
        out = np.zeros(self.ndof)
        rve.check(lib().fehmm_get_u(self.h, out.ctypes.data_as(C.c_void_p)), "fehmm_get_u")
        return out

    def nodes(self):
        out = np.zeros((self.ndof // 2, 2))
        rve.check(lib().fehmm_get_nodes(self.h, out.ctypes.data_as(C.c_void_p)), "fehmm_get_nodes")
        return out

    def qp(self):
        F = np.zeros((self.nqp, 2, 2)); P = np.zeros((self.nqp, 2, 2)); A = np.zeros((self.nqp, 4, 4))
        rve.check(lib().fehmm_get_qp(self.h, F.ctypes.data_as(C.c_void_p), P.ctypes.data_as(C.c_void_p),
                                     A.ctypes.data_as(C.c_void_p)), "fehmm_get_qp")
        return F, P, A

    def get_state(self):
        u = np.zeros(self.ndof); w = np.zeros(self.state_doubles)
        rve.check(lib().fehmm_get_state(self.h, u.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p)),
                  "fehmm_get_state")
        return u, w

    def set_state(self, u, w):
        u = np.ascontiguousarray(u, np.float64); w = np.ascontiguousarray(w, np.float64)
        rve.check(lib().fehmm_set_state(self.h, u.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p)),
                  "fehmm_set_state")

    def destroy(self):
        if self.h is not None:
            rve.check(lib().fehmm_destroy(self.h), "fehmm_destroy")
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
