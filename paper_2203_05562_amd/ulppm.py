"""Thin Python binding of libulppm.so (argument marshalling only).

Every step of the method runs in the HIP library; this module only lays out
torch device tensors, fills the C structs of include/ulppm.h and checks return
codes.  If the library is missing it raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ULPPM_LIB") or os.path.join(HERE, "libulppm.so")

ULPPM_FP64, ULPPM_MIXED = 0, 1
ULPPM_FORCE_CONJUGATE, ULPPM_FORCE_EQ51, ULPPM_FORCE_STANDARD = 0, 1, 2
ULPPM_HISTORY_POINT, ULPPM_HISTORY_BOND = 0, 1
STATUS = {0: "OK", -1: "E_ARG", -2: "E_CAPACITY", -4: "E_NOCONV", -5: "E_NONFINITE", -6: "E_ENERGY",
          -7: "E_HIP"}

_dp = C.POINTER(C.c_double)


class Params(C.Structure):
    _fields_ = [("delta", C.c_double), ("K", C.c_double), ("mu", C.c_double), ("M", C.c_double),
                ("lam", C.c_double), ("kap", C.c_double), ("eta", C.c_double), ("b1", C.c_double),
                ("b2", C.c_double), ("rho_s", C.c_double), ("rho_w", C.c_double), ("a1", C.c_double),
                ("a2", C.c_double), ("n_vg", C.c_double), ("g", C.c_double * 3), ("dt", C.c_double),
                ("newton_tol", C.c_double), ("newton_maxit", C.c_int32), ("precision", C.c_int32),
                ("energy_check", C.c_int32), ("force_mode", C.c_int32), ("energy_tol", C.c_double),
                ("timing", C.c_int32), ("plane", C.c_int32), ("history", C.c_int32), ("pad", C.c_int32)]


class State(C.Structure):
    _fields_ = [("n", C.c_int64), ("x0", _dp * 3), ("u", _dp * 3), ("uc", _dp * 3), ("v", _dp * 3),
                ("a", _dp * 3), ("vol", _dp), ("phi", _dp), ("J", _dp), ("Sr", _dp), ("mass", _dp),
                ("s", _dp), ("sig", _dp * 6), ("pc", _dp), ("fixed", C.POINTER(C.c_uint8))]


class Report(C.Structure):
    _fields_ = [("W_int", C.c_double), ("W_ext", C.c_double), ("W_kin", C.c_double),
                ("n_bonds", C.c_int64), ("n_degenerate", C.c_int64), ("n_plastic", C.c_int64),
                ("max_newton", C.c_int64), ("n_noconv", C.c_int64), ("n_tests", C.c_int64),
                ("n_triples", C.c_int64), ("max_family", C.c_int64), ("steps", C.c_int64),
                ("n_bond_updates", C.c_int64), ("timed_steps", C.c_int64), ("t_predict_ms", C.c_double),
                ("t_family_ms", C.c_double), ("t_bond_ms", C.c_double), ("t_gather_ms", C.c_double),
                ("t_kin_ms", C.c_double), ("n_rebuilds", C.c_int64)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if t is C.c_double else int(getattr(self, k)))
                for k, t in self._fields_}


class Contact(C.Structure):
    _fields_ = [("cs", C.c_double), ("mu_f", C.c_double), ("delta_c", C.c_double), ("origin", C.c_double * 3),
                ("spacing", C.c_double), ("n", C.c_int32 * 3), ("pad", C.c_int32)]


EXPORTS = ["ulppm_create", "ulppm_destroy", "ulppm_last_error", "ulppm_init_state", "ulppm_dt_crit",
           "ulppm_build_families", "ulppm_forces", "ulppm_step", "ulppm_reset_energy", "ulppm_adjoint_reserve",
           "ulppm_adjoint_step", "ulppm_adjoint_init", "ulppm_selfcheck_tail", "ulppm_set_contact",
           "ulppm_history_reserve", "ulppm_history_export", "ulppm_history_import",
           "ulppm_adjoint_step_bond_history", "ulppm_forces_static"]

_lib = None


class UlppmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load the HIP library (no GPU call is made by loading)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() (no CPU fallback exists)")
    L = C.CDLL(path)
    vp = C.c_void_p
    L.ulppm_create.argtypes = [C.POINTER(vp), C.c_int64, C.c_int32, vp]
    L.ulppm_destroy.argtypes = [vp]
    L.ulppm_last_error.argtypes = [vp]
    L.ulppm_last_error.restype = C.c_char_p
    L.ulppm_init_state.argtypes = [vp, C.POINTER(State), C.POINTER(Params), C.c_double]
    L.ulppm_dt_crit.argtypes = [vp, C.POINTER(State), C.POINTER(Params), C.POINTER(C.c_double)]
    L.ulppm_build_families.argtypes = [vp, C.POINTER(State), C.POINTER(Params), C.c_void_p, C.c_void_p,
                                       C.c_int64, C.POINTER(C.c_int64)]
    L.ulppm_forces.argtypes = [vp, C.POINTER(State), C.POINTER(Params), C.c_double, C.POINTER(_dp),
                               C.POINTER(_dp), C.POINTER(Report)]
    L.ulppm_forces_static.argtypes = [C.POINTER(State), C.POINTER(Params), C.c_double, C.POINTER(_dp),
                                      C.POINTER(_dp), C.POINTER(Report), vp]
    L.ulppm_step.argtypes = [vp, C.POINTER(State), C.POINTER(Params), C.c_int32, C.POINTER(Report)]
    L.ulppm_reset_energy.argtypes = [vp]
    L.ulppm_adjoint_reserve.argtypes = [vp]
    L.ulppm_adjoint_step.argtypes = [vp, C.POINTER(State), C.POINTER(State), C.POINTER(Params), C.POINTER(State),
                                     C.POINTER(State), C.c_void_p, C.POINTER(Report)]
    L.ulppm_adjoint_init.argtypes = [vp, C.POINTER(State), C.POINTER(Params), C.c_double, C.POINTER(State),
                                     C.c_void_p, C.c_void_p]
    L.ulppm_selfcheck_tail.argtypes = [C.POINTER(Params), C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32)]
    L.ulppm_set_contact.argtypes = [vp, C.POINTER(Contact)]
    L.ulppm_history_reserve.argtypes = [vp]
    L.ulppm_history_export.argtypes = [vp, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]
    L.ulppm_history_import.argtypes = [vp, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]
    L.ulppm_adjoint_step_bond_history.argtypes = [vp, C.POINTER(State), C.POINTER(State), C.POINTER(Params),
                                                  C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                                  C.POINTER(State), C.POINTER(State), C.c_void_p, C.c_void_p,
                                                  C.POINTER(Report)]
    for name in EXPORTS:
        if name != "ulppm_last_error":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def make_params(prm: dict, precision: int = ULPPM_FP64, **over) -> Params:
    d = dict(prm)
    d.update(over)
    p = Params()
    for k in ("delta", "K", "mu", "M", "lam", "kap", "eta", "b1", "b2", "rho_s", "rho_w", "a1", "a2",
              "n_vg", "dt", "newton_tol"):
        setattr(p, k, float(d[k]))
    p.g[:] = [float(c) for c in d["g"]]
    p.newton_maxit = int(d.get("newton_maxit", 50))
    p.precision = int(d.get("precision", precision))
    p.energy_check = int(d.get("energy_check", 0))
    p.energy_tol = float(d.get("energy_tol", 1e-2))
    p.force_mode = int(d.get("force_mode", 0))
    p.timing = int(d.get("timing", 0))
    p.plane = int(d.get("plane", 0))
    p.history = int(d.get("history", 0))
    return p


VEC = ("x0", "u", "uc", "v", "a")
SCAL = ("vol", "phi", "J", "Sr", "mass", "s", "pc")
# rows of the block a step writes, then the rows it only reads
_MUT = (("u", 3), ("uc", 3), ("v", 3), ("a", 3), ("vol", 1), ("phi", 1), ("J", 1), ("Sr", 1), ("mass", 1),
        ("sig", 6), ("pc", 1))
_RO = (("x0", 3), ("s", 1))
N_MUT_ROWS = sum(r for _, r in _MUT)


class DeviceState:
    """Point state as SoA torch tensors on one device (caller-owned memory).
    The fields a step writes are views into one (24, n) float64 block, so a
    snapshot of them is a single copy; x0 and s sit in a second block."""

    def __init__(self, n: int, device="cuda"):
        import torch
        self.n = n
        self.device = torch.device(device)
        f = dict(dtype=torch.float64, device=self.device)
        self._bind(torch.zeros((N_MUT_ROWS, n), **f), torch.zeros((4, n), **f),
                   torch.zeros(n, dtype=torch.uint8, device=self.device))

    def _bind(self, mut, ro, fixed):
        self.mut, self.ro = mut, ro
        self._cs = None                     # the C view of the fields, built once (they never move)
        self.t: Dict[str, "torch.Tensor"] = {}
        for block, rows in ((mut, _MUT), (ro, _RO)):
            r0 = 0
            for k, r in rows:
                self.t[k] = block[r0:r0 + r] if r > 1 else block[r0]
                r0 += r
        self.t["fixed"] = fixed

    def __getitem__(self, k):
        return self.t[k]

    def snapshot(self) -> "DeviceState":
        """Copy of the fields a step writes; x0, s and fixed are shared."""
        S = DeviceState.__new__(DeviceState)
        S.n, S.device = self.n, self.device
        S._bind(self.mut.clone(), self.ro, self.t["fixed"])
        return S

    @classmethod
    def from_arrays(cls, arrs: dict, device="cuda") -> "DeviceState":
        """arrs in the AoS layout of the test harness: (N,3) vectors, (N,6) stress."""
        import torch
        n = int(np.asarray(arrs["x0"]).shape[0])
        S = cls(n, device)
        for k, v in arrs.items():
            if k not in S.t:
                continue
            a = np.asarray(v)
            if k in VEC or k == "sig":
                a = a.T
            S.t[k].copy_(torch.from_numpy(np.ascontiguousarray(a)))
        return S

    def to_arrays(self) -> dict:
        out = {}
        for k, v in self.t.items():
            a = v.detach().cpu().numpy()
            if k in VEC or k == "sig":
                a = np.ascontiguousarray(a.T)
            out[k] = a
        return out

    def clone(self) -> "DeviceState":
        S = DeviceState.__new__(DeviceState)
        S.n, S.device = self.n, self.device
        S._bind(self.mut.clone(), self.ro.clone(), self.t["fixed"].clone())
        return S

    def cstruct(self) -> State:
        """The ulppm_state of these fields (a copy of one built at the first
        call: a call per C entry point adds no per-field pointer casts)."""
        if self._cs is None:
            self._cs = self._build_cstruct()
        return State.from_buffer_copy(self._cs)

    def _build_cstruct(self) -> State:
        s = State()
        s.n = self.n
        for k in VEC:
            arr = getattr(s, k)
            for c in range(3):
                arr[c] = C.cast(self.t[k][c].data_ptr(), _dp)
        for k in SCAL:
            setattr(s, k, C.cast(self.t[k].data_ptr(), _dp))
        for c in range(6):
            s.sig[c] = C.cast(self.t["sig"][c].data_ptr(), _dp)
        s.fixed = C.cast(self.t["fixed"].data_ptr(), C.POINTER(C.c_uint8))
        return s


class Context:
    """One ulppm context (scratch for up to n points) on the current stream."""

    def __init__(self, n_points: int, max_family: int = 0, stream=None):
        import torch
        self.L = load_library()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.h = C.c_void_p()
        rc = self.L.ulppm_create(C.byref(self.h), int(n_points), int(max_family), C.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise UlppmError(rc, "ulppm_create failed")
        self.n_points = n_points
        self.max_family = max_family

    def close(self):
        if self.h:
            self.L.ulppm_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != 0:
            msg = self.L.ulppm_last_error(self.h)
            raise UlppmError(rc, msg.decode() if msg else "")

    def set_contact(self, desc=None):
        """Attach the substrate described by `desc` (keys cs, mu_f, delta_c,
        origin, spacing, n), or detach it with None."""
        if not desc:
            self._check(self.L.ulppm_set_contact(self.h, None))
            return
        c = Contact()
        c.cs, c.mu_f, c.delta_c = float(desc["cs"]), float(desc["mu_f"]), float(desc["delta_c"])
        c.origin[:] = [float(v) for v in desc["origin"]]
        c.spacing = float(desc["spacing"])
        c.n[:] = [int(v) for v in desc["n"]]
        self._check(self.L.ulppm_set_contact(self.h, C.byref(c)))

    def history_reserve(self):
        self._check(self.L.ulppm_history_reserve(self.h))

    def history_export(self, device="cuda"):
        """(row, col, states (nb, 8)) of the bond history of the last step."""
        import torch
        nb = C.c_int64()
        self._check(self.L.ulppm_history_export(self.h, None, None, None, 0, C.byref(nb)))
        m = int(nb.value)
        row = torch.empty(self.n_points + 1, dtype=torch.int64, device=device)
        col = torch.empty(max(m, 1), dtype=torch.int32, device=device)
        st = torch.empty((max(m, 1), 8), dtype=torch.float64, device=device)
        self._check(self.L.ulppm_history_export(self.h, C.c_void_p(row.data_ptr()), C.c_void_p(col.data_ptr()),
                                                C.c_void_p(st.data_ptr()), m, C.byref(nb)))
        return row, col[:m], st[:m]

    def history_import(self, hist):
        """Load (row, col, states) as history_export returned them; None clears
        the held history."""
        if hist is None:
            self._check(self.L.ulppm_history_import(self.h, self.n_points, None, None, None, 0))
            return
        row, col, st = hist
        nb = int(col.shape[0])
        st = st.contiguous()
        self._check(self.L.ulppm_history_import(self.h, int(row.shape[0]) - 1, C.c_void_p(row.data_ptr()),
                                                C.c_void_p(col.data_ptr()), C.c_void_p(st.data_ptr()), nb))

    def init_state(self, S: DeviceState, p: Params, ocr: float):
        cs = S.cstruct()
        self._check(self.L.ulppm_init_state(self.h, C.byref(cs), C.byref(p), float(ocr)))

    def dt_crit(self, S: DeviceState, p: Params) -> float:
        out = C.c_double()
        cs = S.cstruct()
        self._check(self.L.ulppm_dt_crit(self.h, C.byref(cs), C.byref(p), C.byref(out)))
        return float(out.value)

    def build_families(self, S: DeviceState, p: Params, export: bool = True):
        import torch
        cs = S.cstruct()
        nb = C.c_int64()
        self._check(self.L.ulppm_build_families(self.h, C.byref(cs), C.byref(p), None, None, 0, C.byref(nb)))
        if not export:
            return int(nb.value)
        row = torch.empty(S.n + 1, dtype=torch.int64, device=S.device)
        col = torch.empty(max(int(nb.value), 1), dtype=torch.int32, device=S.device)
        self._check(self.L.ulppm_build_families(self.h, C.byref(cs), C.byref(p), C.c_void_p(row.data_ptr()),
                                                C.c_void_p(col.data_ptr()), col.numel(), C.byref(nb)))
        return row, col[: int(nb.value)]

    def forces(self, S: DeviceState, p: Params, dt_inc: float, want_T: bool = False):
        import torch
        f = torch.zeros((3, S.n), dtype=torch.float64, device=S.device)
        fp = (_dp * 3)(*[C.cast(f[c].data_ptr(), _dp) for c in range(3)])
        rep = Report()
        cs = S.cstruct()
        T = None
        Tp = None
        if want_T:
            nb = self.build_families(S, p, export=False)
            T = torch.zeros((3, max(nb, 1)), dtype=torch.float64, device=S.device)
            Tp = (_dp * 3)(*[C.cast(T[c].data_ptr(), _dp) for c in range(3)])
        self._check(self.L.ulppm_forces(self.h, C.byref(cs), C.byref(p), float(dt_inc), fp, Tp, C.byref(rep)))
        return f, (T[:, : rep.n_bonds] if want_T else None), rep.as_dict()

    def step(self, S: DeviceState, p: Params, n_steps: int) -> dict:
        rep = Report()
        cs = S.cstruct()
        self._check(self.L.ulppm_step(self.h, C.byref(cs), C.byref(p), int(n_steps), C.byref(rep)))
        return rep.as_dict()

    def reset_energy(self):
        self._check(self.L.ulppm_reset_energy(self.h))

    def adjoint_reserve(self):
        self._check(self.L.ulppm_adjoint_reserve(self.h))

    def adjoint_step(self, S: "DeviceState", p: Params, adj1: "DeviceState", adj0: "DeviceState", theta_bar,
                     S1: Optional["DeviceState"] = None) -> dict:
        """One reverse step: adj0 <- (d state_{n+1} / d state_n)^T adj1; theta_bar
        (device float64 tensor of 4: M, lam, kap, eta) accumulates.  S1, the
        state the forward step produced from S, saves re-running that step."""
        rep = Report()
        cs, c1, c0 = S.cstruct(), adj1.cstruct(), adj0.cstruct()
        n1 = C.byref(S1.cstruct()) if S1 is not None else None
        self._check(self.L.ulppm_adjoint_step(self.h, C.byref(cs), n1, C.byref(p), C.byref(c1), C.byref(c0),
                                              C.c_void_p(theta_bar.data_ptr()), C.byref(rep)))
        return rep.as_dict()

    def adjoint_step_bond_history(self, S: "DeviceState", S1: "DeviceState", p: Params, hist_n, hist_bar1,
                                  adj1: "DeviceState", adj0: "DeviceState", theta_bar) -> tuple:
        """One reverse step with the history on the bonds.  hist_n = (row, col,
        states) after step n as history_export returned them (None at the
        first step); hist_bar1 = adjoint of the states after step n+1 (device
        float64 (nb_{n+1}, 8)).  Returns (adjoint of hist_n's states, report)."""
        import torch
        rep = Report()
        cs, c1s, c1, c0 = S.cstruct(), S1.cstruct(), adj1.cstruct(), adj0.cstruct()
        if hist_n is None:
            nb, rp, cp, hp, hbar0 = 0, None, None, None, None
            out = None
        else:
            row, col, st = hist_n
            nb = int(col.shape[0])
            out = torch.zeros((max(nb, 1), 8), dtype=torch.float64, device=st.device)
            rp, cp, hp = (C.c_void_p(t.data_ptr()) for t in (row, col, st))
            hbar0 = C.c_void_p(out.data_ptr())
        hb1 = hist_bar1.contiguous()
        self._check(self.L.ulppm_adjoint_step_bond_history(
            self.h, C.byref(cs), C.byref(c1s), C.byref(p), nb, rp, cp, hp, C.c_void_p(hb1.data_ptr()),
            C.byref(c1), C.byref(c0), hbar0, C.c_void_p(theta_bar.data_ptr()), C.byref(rep)))
        return (out[:nb] if out is not None else None), rep.as_dict()

    def adjoint_init(self, S0: "DeviceState", p: Params, ocr: float, adj0: "DeviceState", s_bar, theta_bar):
        """Reverse of init_state at its output S0: s_bar (device float64 (n,))
        receives the suction adjoint; theta_bar[0] accumulates the M adjoint."""
        c0, ca = S0.cstruct(), adj0.cstruct()
        self._check(self.L.ulppm_adjoint_init(self.h, C.byref(c0), C.byref(p), float(ocr), C.byref(ca),
                                              C.c_void_p(s_bar.data_ptr()), C.c_void_p(theta_bar.data_ptr())))


STATIC_MAX_POINTS, STATIC_MAX_FAMILY = 2048, 128


def forces_static(S: DeviceState, p: Params, dt_inc: float, f, T=None, stream=None) -> dict:
    """ulppm_forces_static: Algorithm 1 with no context and no device
    allocation.  f (3, n) and, if given, T (3, >= n_bonds) are caller-owned
    float64 device tensors that receive the nodal forces and force states."""
    import torch
    L = load_library()
    if stream is None:
        stream = torch.cuda.current_stream()
    fp = (_dp * 3)(*[C.cast(f[c].data_ptr(), _dp) for c in range(3)])
    Tp = (_dp * 3)(*[C.cast(T[c].data_ptr(), _dp) for c in range(3)]) if T is not None else None
    rep = Report()
    cs = S.cstruct()
    rc = L.ulppm_forces_static(C.byref(cs), C.byref(p), float(dt_inc), fp, Tp, C.byref(rep),
                               C.c_void_p(stream.cuda_stream))
    if rc != 0:
        raise UlppmError(rc, "ulppm_forces_static failed")
    return rep.as_dict()


def selfcheck_tail(p: Params, seed: int = 0, n_cases: int = 40):
    """Host-only check of the library's reverse of the per-bond tail (no GPU)."""
    L = load_library()
    m = C.c_double()
    npl = C.c_int32()
    rc = L.ulppm_selfcheck_tail(C.byref(p), int(seed), int(n_cases), C.byref(m), C.byref(npl))
    if rc != 0:
        raise UlppmError(rc, "selfcheck failed")
    return float(m.value), int(npl.value)


def column_state(col: dict, device="cuda", v0: Optional[np.ndarray] = None) -> DeviceState:
    """Device state of a seeded column before ulppm_init_state: total stress in
    sig, initial porosity and volume, suction, fixed base."""
    n = col["n"]
    arrs = dict(x0=col["x0"], vol=col["vol0"], phi=col["phi0"], s=col["suction"], sig=col["sig_geo"],
                fixed=col["fixed"], v=(v0 if v0 is not None else np.zeros((n, 3))))
    return DeviceState.from_arrays(arrs, device)
