"""FP64 CPU oracle of the periodic-RVE hot path (TEST INFRASTRUCTURE ONLY).

Plain, slow, obviously-correct C code (``rve.c``, ``sparse.c``, ``macro.c``)
written from the paper (Eidel, Fischer, Gote, arXiv:1908.08292) in its
total-Lagrangian S/E notation, loaded here through ctypes.  Only ``tests/``,
the smoke check and the benchmark's CPU-baseline leg may import this package;
the product library shares no code with it.

Conventions: F, P row-major d x d ([i][J]); A is d^2 x d^2 with
A[(i*d+J), (k*d+L)] = dP_iJ/dF_kL; fluctuations node-major [node][d] with node
(i,j[,k]) -> i + n j [+ n^2 k]; element ids likewise.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")

OK, NOCONV, DETF, SINGULAR, NONFINITE = 0, 1, 2, 3, 4


def build():
    """Compile the oracle with gcc (test infrastructure)."""
    subprocess.check_call(["sh", os.path.join(_HERE, "build.sh")])


def _load():
    if not os.path.exists(_LIB):
        build()
    return C.CDLL(_LIB)


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load()
        _setup(_lib)
    return _lib


class Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("max_iter", C.c_int),
                ("max_backtrack", C.c_int), ("want_A", C.c_int)]


class MacroDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("Lx", C.c_double), ("Ly", C.c_double),
                ("hole_r", C.c_double), ("bc", C.c_int), ("stretch", C.c_double), ("nsteps", C.c_int),
                ("rtol_macro", C.c_double), ("scheme", C.c_int), ("max_macro_iter", C.c_int),
                ("n", C.c_int), ("phase", C.c_void_p), ("lame", C.c_void_p), ("elem", C.c_int)]


_dp = C.POINTER(C.c_double)


def _setup(L):
    L.oracle_nh_sc.restype = C.c_int
    L.oracle_nh_sc.argtypes = [C.c_int, C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.oracle_set_law.restype = None
    L.oracle_set_law.argtypes = [C.c_int]
    L.oracle_get_law.restype = C.c_int
    L.oracle_law_sc.restype = C.c_int
    L.oracle_law_sc.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.c_void_p]
    L.oracle_set_element.restype = None
    L.oracle_set_element.argtypes = [C.c_int]
    L.oracle_get_element.restype = C.c_int
    L.oracle_set_bc.restype = None
    L.oracle_set_bc.argtypes = [C.c_int]
    L.oracle_get_bc.restype = C.c_int
    L.oracle_phase_by_centroid.restype = None
    L.oracle_phase_by_centroid.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_double, C.c_int, C.c_int, C.c_void_p]
    L.oracle_element.restype = C.c_int
    L.oracle_element.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p]
    L.oracle_residual.restype = C.c_int
    L.oracle_residual.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p]
    L.oracle_rve_solve.restype = C.c_int
    L.oracle_rve_solve.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.POINTER(Opts), C.c_void_p, C.c_void_p, C.POINTER(C.c_int), C.c_void_p]
    L.oracle_rve_solve_batch.restype = C.c_int
    L.oracle_rve_solve_batch.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.POINTER(Opts), C.c_void_p, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_int]
    L.oracle_linear_homogenized.restype = C.c_int
    L.oracle_linear_homogenized.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    L.oracle__rve_one_step.restype = C.c_int
    L.oracle__rve_one_step.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.POINTER(Opts), C.c_void_p, C.c_void_p, _dp]
    L.oracle_debug_system.restype = C.c_int
    L.oracle_debug_system.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p]
    L.oracle_macro_create.restype = C.c_void_p
    L.oracle_macro_create.argtypes = [C.POINTER(MacroDesc), C.POINTER(Opts)]
    L.oracle_macro_destroy.restype = None
    L.oracle_macro_destroy.argtypes = [C.c_void_p]
    L.oracle_macro_ndof.restype = C.c_int
    L.oracle_macro_ndof.argtypes = [C.c_void_p]
    L.oracle_macro_nqp.restype = C.c_int
    L.oracle_macro_nqp.argtypes = [C.c_void_p]
    L.oracle_macro_step.restype = C.c_int
    L.oracle_macro_step.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.c_void_p, C.POINTER(C.c_int64)]
    L.oracle_macro_get_u.restype = None
    L.oracle_macro_get_u.argtypes = [C.c_void_p, C.c_void_p]
    L.oracle_macro_get_qp.restype = None
    L.oracle_macro_get_qp.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.oracle_macro_get_nodes.restype = None
    L.oracle_macro_get_nodes.argtypes = [C.c_void_p, C.c_void_p]
    L.oracle_macro_nelem.restype = C.c_int
    L.oracle_macro_nelem.argtypes = [C.c_void_p]
    L.oracle_macro_get_conn.restype = None
    L.oracle_macro_get_conn.argtypes = [C.c_void_p, C.c_void_p]
    L.oracle_macro_get_state.restype = None
    L.oracle_macro_get_state.argtypes = [C.c_void_p, C.c_void_p]
    L.oracle_macro_set_qp.restype = None
    L.oracle_macro_set_qp.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.oracle_macro_element_stiffness.restype = C.c_int
    L.oracle_macro_element_stiffness.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    L.oracle_rve_transfer_states.restype = C.c_int
    L.oracle_rve_transfer_states.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                             C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_atol(lame, n, d):
    """atol = 1e-12 * mu_max * h^(d-1) (Newton floor; needed when Fbar = I gives R0 = 0)."""
    mu_max = float(np.max(np.asarray(lame, dtype=np.float64)[:, 1]))
    return 1e-12 * mu_max * (1.0 / n) ** (d - 1)


def make_opts(lame, n, d, rtol=1e-10, atol=None, max_iter=25, max_backtrack=8, want_A=True):
    return Opts(rtol, default_atol(lame, n, d) if atol is None else atol, max_iter, max_backtrack, int(want_A))


def lame(E, nu):
    """Lame parameters from Young's modulus and Poisson's ratio (3D relations,
    also used for plane strain), as tabulated in the paper's material table."""
    return E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


def two_phase_lame(ratio, E=1.0, nu=0.3):
    """[[lambda, mu] matrix, [lambda, mu] inclusion] with E_incl = ratio * E."""
    return np.array([lame(E, nu), lame(ratio * E, nu)], dtype=np.float64)


def debug_system(d, n, phase, lame_, Fbar, w):
    nf = d * n_free_nodes(d, n)
    Rf = np.zeros(nf); K = np.zeros((nf, nf)); dw = np.zeros(nf)
    st = lib().oracle_debug_system(d, n, _p(np.ascontiguousarray(phase, np.uint8)), _p(_f64(lame_)),
                                   _p(_f64(Fbar)), _p(_f64(w)), _p(Rf), _p(K), _p(dw))
    return st, Rf, K, dw


def nh_sc(d, lam, mu, F):
    """Second Piola-Kirchhoff stress S, material tangent C (d^4) and psi."""
    F = _f64(F).reshape(d, d)
    S = np.zeros((d, d)); Cm = np.zeros((d,) * 4); psi = np.zeros(1)
    st = lib().oracle_nh_sc(d, lam, mu, _p(F), _p(S), _p(Cm), _p(psi))
    return st, S, Cm, float(psi[0])


LAW_NEOHOOKE, LAW_SVK, LAW_LINEAR = 0, 1, 2


def set_law(law):
    """Micro constitutive law of every later oracle call (process-wide)."""
    lib().oracle_set_law(int(law))


def get_law():
    return lib().oracle_get_law()


class law:
    """Context manager: `with oracle.law(oracle.LAW_SVK): ...`."""

    def __init__(self, which):
        self.which = which

    def __enter__(self):
        self.prev = get_law()
        set_law(self.which)
        return self

    def __exit__(self, *exc):
        set_law(self.prev)


BC_PERIODIC, BC_LINEAR = 0, 1


def set_bc(bc):
    """Micro boundary conditions of every later oracle call (process-wide)."""
    lib().oracle_set_bc(int(bc))


def get_bc():
    return lib().oracle_get_bc()


class bc:
    """Context manager: `with oracle.bc(oracle.BC_LINEAR): ...`."""

    def __init__(self, which):
        self.which = which

    def __enter__(self):
        self.prev = get_bc()
        set_bc(self.which)
        return self

    def __exit__(self, *exc):
        set_bc(self.prev)


ELEM_Q1, ELEM_P1 = 0, 1


def set_element(kind):
    """Micro element kind of every later oracle call (process-wide)."""
    lib().oracle_set_element(int(kind))


def get_element():
    return lib().oracle_get_element()


class element_kind:
    """Context manager: `with oracle.element_kind(oracle.ELEM_P1): ...`."""

    def __init__(self, which):
        self.which = which

    def __enter__(self):
        self.prev = get_element()
        set_element(self.which)
        return self

    def __exit__(self, *exc):
        set_element(self.prev)


def n_free_nodes(d, n):
    """Free nodes of the n^d grid under the current micro boundary conditions."""
    return n ** d - 1 if get_bc() == BC_PERIODIC else (n - 1) ** d


def law_sc(which, d, lam, mu, F):
    """S (sigma for the linear law), material tangent (d^4) and psi."""
    F = _f64(F).reshape(d, d)
    S = np.zeros((d, d)); Cm = np.zeros((d,) * 4); psi = np.zeros(1)
    st = lib().oracle_law_sc(int(which), d, lam, mu, _p(F), _p(S), _p(Cm), _p(psi))
    return st, S, Cm, float(psi[0])


def phase_by_centroid(d, n, r, center=None, incl_phase=1, base_phase=0):
    c = _f64(center if center is not None else [0.5] * d)
    ph = np.zeros(n ** d, dtype=np.uint8)
    lib().oracle_phase_by_centroid(d, n, _p(c), float(r), incl_phase, base_phase, _p(ph))
    return ph


def element(d, n, phase, lame, e, Fbar, w):
    nd = (2 ** d) * d
    fe = np.zeros(nd); ke = np.zeros((nd, nd)); en = np.zeros(1)
    st = lib().oracle_element(d, n, _p(np.ascontiguousarray(phase, np.uint8)), _p(_f64(lame)), e,
                              _p(_f64(Fbar)), _p(_f64(w)), _p(fe), _p(ke), _p(en))
    return st, fe, ke, float(en[0])


def residual(d, n, phase, lame, Fbar, w):
    R = np.zeros(d * n ** d); en = np.zeros(1)
    st = lib().oracle_residual(d, n, _p(np.ascontiguousarray(phase, np.uint8)), _p(_f64(lame)), _p(_f64(Fbar)),
                               _p(_f64(w)), _p(R), _p(en))
    return st, R, float(en[0])


def rve_solve(d, n, phase, lame, Fbar, w=None, opts=None, **kw):
    """One RVE: returns dict(status, P, A, iters, w, res_hist)."""
    lame = _f64(lame)
    o = opts if opts is not None else make_opts(lame, n, d, **kw)
    P = np.zeros((d, d)); A = np.zeros((d * d, d * d))
    hist = np.zeros(o.max_iter + 2)
    it = C.c_int(0)
    wv = None if w is None else _f64(w).copy()
    st = lib().oracle_rve_solve(d, n, _p(np.ascontiguousarray(phase, np.uint8)), _p(lame), _p(_f64(Fbar)),
                                _p(wv), C.byref(o), _p(P), _p(A), C.byref(it), _p(hist))
    return dict(status=st, P=P, A=A, iters=it.value, w=wv, res_hist=hist[: it.value + 1])


def rve_one_step(d, n, phase, lame, Fbar, w, opts=None):
    lame = _f64(lame)
    o = opts if opts is not None else make_opts(lame, n, d)
    P = np.zeros((d, d)); A = np.zeros((d * d, d * d)); rn = C.c_double(0)
    wv = _f64(w).copy()
    st = lib().oracle__rve_one_step(d, n, _p(np.ascontiguousarray(phase, np.uint8)), _p(lame), _p(_f64(Fbar)),
                                    _p(wv), C.byref(o), _p(P), _p(A), C.byref(rn))
    return dict(status=st, P=P, A=A, w=wv, rnorm=rn.value)


def rve_solve_batch(d, n, phases, lame, F, w=None, opts=None, nthreads=0, **kw):
    """Batch of B RVEs of one size; phases [B, n^d]; F [B, d, d]."""
    lame = _f64(lame)
    F = _f64(F)
    B = F.shape[0]
    o = opts if opts is not None else make_opts(lame, n, d, **kw)
    ph = np.ascontiguousarray(phases, np.uint8)
    P = np.zeros((B, d, d)); A = np.zeros((B, d * d, d * d))
    status = np.zeros(B, np.int32); iters = np.zeros(B, np.int32)
    wv = None if w is None else _f64(w)
    lib().oracle_rve_solve_batch(d, n, B, _p(ph), _p(lame), _p(F), _p(wv), C.byref(o), _p(P), _p(A),
                                 _p(status), _p(iters), int(nthreads))
    return dict(status=status, P=P, A=A, iters=iters, w=wv)


def transfer_states(d, n, phase, lame_, Fbar, w, G, t=None):
    """T^T K T [nstate, nstate] for prescribed gradient states G [nstate, d, d]
    (translations t [nstate, d] or None) at the micro state (Fbar, w)."""
    G = _f64(G).reshape(-1, d * d)
    ns = G.shape[0]
    kT = np.zeros((ns, ns))
    tt = None if t is None else _f64(t).reshape(ns, d)
    st = lib().oracle_rve_transfer_states(d, n, _p(np.ascontiguousarray(phase, np.uint8)), _p(_f64(lame_)),
                                          _p(_f64(Fbar)), _p(_f64(w)), ns, _p(G), _p(tt), _p(kT))
    return st, kT


def linear_homogenized(d, n, phase, lame):
    Ch = np.zeros((d * d, d * d))
    st = lib().oracle_linear_homogenized(d, n, _p(np.ascontiguousarray(phase, np.uint8)), _p(_f64(lame)), _p(Ch))
    return st, Ch


class Macro:
    """Macro FE-HMM driver of the oracle (2D, Q1 macro, 2x2 Gauss)."""

    def __init__(self, nx, ny, n, phase, lame, Lx=1.0, Ly=1.0, hole_r=0.0, bc=0, stretch=1.1, nsteps=10,
                 rtol_macro=1e-10, scheme=0, max_macro_iter=30, micro_opts=None, elem=0):
        self._phase = np.ascontiguousarray(phase, np.uint8)
        self._lame = _f64(lame)
        self.desc = MacroDesc(nx, ny, Lx, Ly, hole_r, bc, stretch, nsteps, rtol_macro, scheme, max_macro_iter,
                              n, _p(self._phase), _p(self._lame), int(elem))
        self.opts = micro_opts if micro_opts is not None else make_opts(self._lame, n, 2)
        self.h = lib().oracle_macro_create(C.byref(self.desc), C.byref(self.opts))
        self.ndof = lib().oracle_macro_ndof(self.h)
        self.nqp = lib().oracle_macro_nqp(self.h)
        self.max_macro_iter = max_macro_iter

    def step(self, k):
        it = C.c_int(0); mic = C.c_int64(0)
        hist = np.zeros(self.max_macro_iter + 2)
        st = lib().oracle_macro_step(self.h, k, C.byref(it), _p(hist), C.byref(mic))
        return dict(status=st, macro_iters=it.value, res_hist=hist[: it.value + 1], micro_iters=mic.value)

    def u(self):
        u = np.zeros(self.ndof)
        lib().oracle_macro_get_u(self.h, _p(u))
        return u

    def nodes(self):
        xy = np.zeros((self.ndof // 2, 2))
        lib().oracle_macro_get_nodes(self.h, _p(xy))
        return xy

    def qp(self):
        F = np.zeros((self.nqp, 2, 2)); P = np.zeros((self.nqp, 2, 2)); A = np.zeros((self.nqp, 4, 4))
        lib().oracle_macro_get_qp(self.h, _p(F), _p(P), _p(A))
        return F, P, A

    def nelem(self):
        return lib().oracle_macro_nelem(self.h)

    def conn(self):
        c = np.zeros((self.nelem(), 4), np.int32)
        lib().oracle_macro_get_conn(self.h, _p(c))
        return c

    def state(self):
        w = np.zeros((self.nqp, 2 * self.desc.n ** 2))
        lib().oracle_macro_get_state(self.h, _p(w))
        return w

    def set_qp(self, F=None, P=None, A=None, w=None):
        lib().oracle_macro_set_qp(self.h, *[None if x is None else _p(_f64(x)) for x in (F, P, A, w)])

    def element_stiffness(self, e, literal=True):
        """[8, 8] macro element stiffness at the stored micro states: the literal
        T^T K T transfer of the unit nodal states, or B^T Abar B."""
        k = np.zeros((8, 8))
        st = lib().oracle_macro_element_stiffness(self.h, int(e), 1 if literal else 0, _p(k))
        if st:
            raise RuntimeError(f"element stiffness failed: {st}")
        return k

    def close(self):
        if self.h:
            lib().oracle_macro_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
