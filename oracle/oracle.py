"""ctypes wrapper of the CPU oracle (test infrastructure only).

State dictionaries hold float64 numpy arrays in caller order:
  x0, u, uc, v, a : (N, 3)
  vol, phi, J, Sr, mass, s, pc : (N,)
  sig : (N, 6) effective stress, Voigt (xx, yy, zz, yz, xz, xy), tension +
  fixed : (N,) uint8
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build

__all__ = ["OracleParams", "lib", "make_params", "init_column", "families", "bond_fields",
           "step", "step_dual", "step_bond_history", "step_dual_bond_history", "BondHistory", "dt_crit", "return_map", "rm_residual", "swrc", "copy_state",
           "empty_state", "params_dict", "STATE_FIELDS"]

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_i8p = C.POINTER(C.c_int8)
_u8p = C.POINTER(C.c_uint8)


class OracleParams(C.Structure):
    _fields_ = [("delta", C.c_double), ("K", C.c_double), ("mu", C.c_double), ("M", C.c_double),
                ("lam", C.c_double), ("kap", C.c_double), ("eta", C.c_double), ("b1", C.c_double),
                ("b2", C.c_double), ("rho_s", C.c_double), ("rho_w", C.c_double), ("a1", C.c_double),
                ("a2", C.c_double), ("n_vg", C.c_double), ("g", C.c_double * 3), ("dt", C.c_double),
                ("newton_tol", C.c_double), ("newton_maxit", C.c_int32), ("force_mode", C.c_int32),
                ("cs", C.c_double), ("mu_f", C.c_double), ("delta_c", C.c_double),
                ("sub_origin", C.c_double * 3), ("sub_dx", C.c_double), ("sub_n", C.c_int32 * 3),
                ("plane", C.c_int32)]


class OracleState(C.Structure):
    _fields_ = [("n", C.c_int64), ("x0", _dp), ("u", _dp), ("uc", _dp), ("v", _dp), ("a", _dp),
                ("vol", _dp), ("phi", _dp), ("J", _dp), ("Sr", _dp), ("mass", _dp), ("s", _dp),
                ("sig", _dp), ("pc", _dp), ("fixed", _u8p)]


class OracleBondHistory(C.Structure):
    _fields_ = [("n", C.c_int64), ("cap", C.c_int64), ("nb", C.c_int64), ("row", _i64p), ("col", _i32p),
                ("st", _dp)]


class OracleStats(C.Structure):
    _fields_ = [("n_bonds", C.c_int64), ("n_degenerate", C.c_int64), ("n_plastic", C.c_int64),
                ("max_newton", C.c_int64), ("n_noconv", C.c_int64), ("n_tests", C.c_int64),
                ("n_triples", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


STATE_FIELDS = dict(x0=3, u=3, uc=3, v=3, a=3, vol=1, phi=1, J=1, Sr=1, mass=1, s=1, sig=6, pc=1)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.oracle_families.restype = C.c_int64
        L.oracle_families.argtypes = [C.c_int64, _dp, C.c_double, C.c_int32, _i64p, _i32p, C.c_int64]
        L.oracle_bond_fields.restype = C.c_int64
        L.oracle_bond_fields.argtypes = [C.POINTER(OracleParams), C.POINTER(OracleState), C.c_double,
                                         C.c_int64, _i64p, _i32p, _dp, _dp, _dp, _dp, _dp, _dp, _i32p,
                                         _i8p, _dp, _dp, _dp, _dp, _dp, C.POINTER(OracleStats)]
        L.oracle_step.restype = C.c_int
        L.oracle_step.argtypes = [C.POINTER(OracleParams), C.POINTER(OracleState), C.c_int32, _dp,
                                  C.POINTER(OracleStats)]
        L.oracle_step_bond_history.restype = C.c_int
        L.oracle_step_bond_history.argtypes = [C.POINTER(OracleParams), C.POINTER(OracleState),
                                               C.POINTER(OracleBondHistory), C.c_int32, _dp,
                                               C.POINTER(OracleStats)]
        L.oracle_step_dual.restype = C.c_int
        L.oracle_step_dual.argtypes = [C.POINTER(OracleParams), _dp, C.POINTER(OracleState),
                                       C.POINTER(OracleState), C.c_int32, _dp, C.POINTER(OracleStats)]
        L.oracle_step_dual_bond_history.restype = C.c_int
        L.oracle_step_dual_bond_history.argtypes = [C.POINTER(OracleParams), _dp, C.POINTER(OracleState),
                                                    C.POINTER(OracleState), C.POINTER(OracleBondHistory), _dp,
                                                    C.c_int32, _dp, C.POINTER(OracleStats)]
        L.oracle_init_state.restype = C.c_int
        L.oracle_init_state.argtypes = [C.POINTER(OracleParams), C.POINTER(OracleState), C.c_double]
        L.oracle_dt_crit.restype = C.c_double
        L.oracle_dt_crit.argtypes = [C.POINTER(OracleParams), C.POINTER(OracleState)]
        L.oracle_return_map.restype = C.c_int
        L.oracle_return_map.argtypes = [C.POINTER(OracleParams), C.c_double, _dp, C.c_double, _dp, _dp, _dp]
        L.oracle_rm_residual.restype = None
        L.oracle_rm_residual.argtypes = [C.POINTER(OracleParams), C.c_double, C.c_double, C.c_double,
                                         C.c_double, _dp, _dp, _dp]
        L.oracle_swrc.restype = C.c_double
        L.oracle_swrc.argtypes = [C.POINTER(OracleParams), C.c_double, C.c_double, C.c_double]
        _lib = L
    return _lib


def _p(a, t=_dp):
    return a.ctypes.data_as(t) if a is not None else None


def make_params(prm: dict, **over) -> OracleParams:
    d = dict(prm)
    d.update(over)
    p = OracleParams()
    for k in ("delta", "K", "mu", "M", "lam", "kap", "eta", "b1", "b2", "rho_s", "rho_w", "a1", "a2",
              "n_vg", "dt", "newton_tol"):
        setattr(p, k, float(d[k]))
    p.g[:] = [float(c) for c in d["g"]]
    p.newton_maxit = int(d.get("newton_maxit", 50))
    p.force_mode = int(d.get("force_mode", 0))
    p.plane = int(d.get("plane", 0))
    c = d.get("contact")
    if c:
        p.cs, p.mu_f, p.delta_c = float(c["cs"]), float(c["mu_f"]), float(c["delta_c"])
        p.sub_origin[:] = [float(v) for v in c["origin"]]
        p.sub_dx = float(c["spacing"])
        p.sub_n[:] = [int(v) for v in c["n"]]
    return p


def params_dict(p: OracleParams) -> dict:
    d = {k: getattr(p, k) for k, _ in OracleParams._fields_
         if k not in ("g", "cs", "mu_f", "delta_c", "sub_origin", "sub_dx", "sub_n")}
    d["g"] = list(p.g)
    if p.cs > 0.0:
        d["contact"] = dict(cs=p.cs, mu_f=p.mu_f, delta_c=p.delta_c, origin=list(p.sub_origin),
                            spacing=p.sub_dx, n=list(p.sub_n))
    return d


def _cstate(S: dict) -> OracleState:
    cs = OracleState()
    cs.n = int(S["x0"].shape[0])
    for k in STATE_FIELDS:
        arr = S[k]
        assert arr.dtype == np.float64 and arr.flags.c_contiguous, k
        setattr(cs, k, _p(arr))
    assert S["fixed"].dtype == np.uint8
    cs.fixed = _p(S["fixed"], _u8p)
    return cs


def copy_state(S: dict) -> dict:
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in S.items()}


def empty_state(n: int) -> dict:
    S = {k: np.zeros((n, w) if w > 1 else n) for k, w in STATE_FIELDS.items()}
    S["fixed"] = np.zeros(n, np.uint8)
    return S


def init_column(col: dict, prm: OracleParams, ocr: float, v0=None) -> dict:
    """Initial state of a column from the input generator's arrays."""
    n = col["n"]
    S = empty_state(n)
    S["x0"][:] = col["x0"]
    S["vol"][:] = col["vol0"]
    S["phi"][:] = col["phi0"]
    S["s"][:] = col["suction"]
    S["sig"][:] = col["sig_geo"]
    S["fixed"][:] = col["fixed"]
    if v0 is not None:
        S["v"][:] = v0
    cs = _cstate(S)
    rc = lib().oracle_init_state(C.byref(prm), C.byref(cs), float(ocr))
    assert rc == 0
    return S


def families(x: np.ndarray, delta: float, brute: bool = False):
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    row = np.zeros(n + 1, np.int64)
    nb = lib().oracle_families(n, _p(x), float(delta), int(brute), _p(row, _i64p), None, 0)
    col = np.zeros(max(nb, 1), np.int32)
    lib().oracle_families(n, _p(x), float(delta), int(brute), _p(row, _i64p), _p(col, _i32p), nb)
    return row, col[:nb]


def bond_fields(S: dict, prm: OracleParams, dt_inc: float) -> dict:
    """Algorithm 1 at the state's positions; per-bond arrays in CSR order."""
    n = S["x0"].shape[0]
    cs = _cstate(S)
    st = OracleStats()
    nb = -lib().oracle_bond_fields(C.byref(prm), C.byref(cs), float(dt_inc), 0, *([None] * 15), C.byref(st))
    nb = max(nb, 0)
    out = dict(row=np.zeros(n + 1, np.int64), col=np.zeros(max(nb, 1), np.int32),
               K=np.zeros((max(nb, 1), 6)), L=np.zeros((max(nb, 1), 9)), sig=np.zeros((max(nb, 1), 6)),
               pc=np.zeros(max(nb, 1)), T=np.zeros((max(nb, 1), 3)), varpi=np.zeros(max(nb, 1)),
               nsub=np.zeros(max(nb, 1), np.int32), active=np.zeros(max(nb, 1), np.int8),
               f=np.zeros((n, 3)), Jd=np.zeros(n), Sr_new=np.zeros(n), sig_pt=np.zeros((n, 6)),
               pc_pt=np.zeros(n))
    st = OracleStats()
    r = lib().oracle_bond_fields(C.byref(prm), C.byref(cs), float(dt_inc), nb, _p(out["row"], _i64p),
                                 _p(out["col"], _i32p), _p(out["K"]), _p(out["L"]), _p(out["sig"]),
                                 _p(out["pc"]), _p(out["T"]), _p(out["varpi"]), _p(out["nsub"], _i32p),
                                 _p(out["active"], _i8p), _p(out["f"]), _p(out["Jd"]), _p(out["Sr_new"]),
                                 _p(out["sig_pt"]), _p(out["pc_pt"]), C.byref(st))
    assert r == nb, (r, nb)
    for k in ("col", "K", "L", "sig", "pc", "T", "varpi", "nsub", "active"):
        out[k] = out[k][:nb]
    out["stats"] = st.as_dict()
    return out


def step(S: dict, prm: OracleParams, n_steps: int = 1, energy=None):
    """Advance the state in place; returns (rc, energy[3], stats)."""
    e = np.zeros(3) if energy is None else energy
    cs = _cstate(S)
    st = OracleStats()
    rc = lib().oracle_step(C.byref(prm), C.byref(cs), int(n_steps), _p(e), C.byref(st))
    return rc, e, st.as_dict()


class BondHistory:
    """History carried on the bonds between oracle_step_bond_history calls:
    families (row, col) and 8 values per bond (sigma Voigt, p_c, unused)."""

    def __init__(self, n: int, cap: int):
        self.row = np.zeros(n + 1, np.int64)
        self.col = np.zeros(max(cap, 1), np.int32)
        self.st = np.zeros((max(cap, 1), 8))
        self.dst = np.zeros((max(cap, 1), 8))      # tangents of st (dual-number runs)
        self.c = OracleBondHistory(0, cap, 0, _p(self.row, _i64p), _p(self.col, _i32p), _p(self.st))

    @property
    def nb(self) -> int:
        return int(self.c.nb)


def step_bond_history(S: dict, prm: OracleParams, H: BondHistory, n_steps: int = 1, energy=None):
    """Advance with the history on the bonds; H carries it between calls."""
    e = np.zeros(3) if energy is None else energy
    cs = _cstate(S)
    st = OracleStats()
    rc = lib().oracle_step_bond_history(C.byref(prm), C.byref(cs), C.byref(H.c), int(n_steps), _p(e),
                                        C.byref(st))
    return rc, e, st.as_dict()


def step_dual(S: dict, dS: dict, prm: OracleParams, dparam, n_steps: int = 1, energy=None):
    """Forward-mode tangent of n_steps steps; S and dS advanced in place.
    dparam = tangents of (M, lam, kap, eta); suction tangent in dS['s']."""
    e = np.zeros(3) if energy is None else energy
    dp = np.ascontiguousarray(np.asarray(dparam, np.float64))
    cs, cd = _cstate(S), _cstate(dS)
    st = OracleStats()
    rc = lib().oracle_step_dual(C.byref(prm), _p(dp), C.byref(cs), C.byref(cd), int(n_steps), _p(e),
                                C.byref(st))
    return rc, e, st.as_dict()


def step_dual_bond_history(S: dict, dS: dict, prm: OracleParams, dparam, H: BondHistory, n_steps: int = 1,
                           energy=None):
    """step_dual with the history on the bonds: H.st and its tangents H.dst
    are carried between calls like S and dS."""
    e = np.zeros(3) if energy is None else energy
    dp = np.ascontiguousarray(np.asarray(dparam, np.float64))
    cs, cd = _cstate(S), _cstate(dS)
    st = OracleStats()
    rc = lib().oracle_step_dual_bond_history(C.byref(prm), _p(dp), C.byref(cs), C.byref(cd), C.byref(H.c),
                                             _p(H.dst), int(n_steps), _p(e), C.byref(st))
    return rc, e, st.as_dict()


def dt_crit(S: dict, prm: OracleParams) -> float:
    return float(lib().oracle_dt_crit(C.byref(prm), C.byref(_cstate(S))))


def return_map(prm: OracleParams, dt: float, sig_n, pc_n: float, deps):
    sig_n = np.ascontiguousarray(sig_n, np.float64)
    deps = np.ascontiguousarray(deps, np.float64)
    out = np.zeros(6)
    pc = np.zeros(1)
    it = lib().oracle_return_map(C.byref(prm), float(dt), _p(sig_n), float(pc_n), _p(deps), _p(out), _p(pc))
    return out, float(pc[0]), int(it)


def rm_residual(prm: OracleParams, c: float, ptr: float, qtr: float, pcn: float, x):
    x = np.ascontiguousarray(x, np.float64)
    r = np.zeros(3)
    A = np.zeros(9)
    lib().oracle_rm_residual(C.byref(prm), float(c), float(ptr), float(qtr), float(pcn), _p(x), _p(r), _p(A))
    return r, A.reshape(3, 3)


def swrc(prm: OracleParams, J: float, phi: float, s_pa: float) -> float:
    return float(lib().oracle_swrc(C.byref(prm), float(J), float(phi), float(s_pa)))
