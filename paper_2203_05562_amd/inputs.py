"""Seeded synthetic inputs: soil-column lattices and their set-up parameters.

This module is shared by the GPU path and by the tests' CPU oracle, so it holds
none of the method's arithmetic: no families, shape tensors, gradients, return
mapping, retention curve or force states.  It only lays points on a jittered
cubic lattice, draws the seeded random numbers, and derives problem set-up
constants (geostatic total stress, solid grain density, Perzyna viscosity)
from the workload description.

Workloads (3D stand-ins for the paper's 2D column-collapse examples of
Section 4.2; the paper's own geometry, experimental data and figures are not
available, so every input here is synthetic):

    C0  8 x 8 x 16     =     1,024 points, seed 0, suction 20 kPa, FP64
    C1  40 x 40 x 80   =   128,000 points, seeds 1.., suction U(10, 40) kPa, FP64
    C2  80 x 80 x 160  = 1,024,000 points, seed 2, suction 20 kPa, mixed precision
    C3  24 x 24 x 48   =    27,648 points, seed 3, suction 20 kPa, adjoint
    C4  128 x 128 x 256 = 4,194,304 points, seed 4, suction 20 kPa, mixed + adjoint
    P0  24 x 48 plane strain   =   1,152 points, seed 10, suction 20 kPa, FP64
    P1  512 x 1024 plane strain = 524,288 points, seed 11, suction 20 kPa, FP64
    U2, U3  uniaxial compression bar 40 x 12 x 12 (Section 4.1), horizon 2 and
        3 spacings, unjittered, elastic, one end driven (make_uniaxial_block)

Plane-strain columns (the paper's examples are 2D) lie in the x-z plane at
y = 0 with jitter in x and z only; each point's volume is dx^2 times a unit
thickness.

Lattice: index = ix + nx*(iy + ny*iz), z vertical, spacing dx = 0.01 m,
x = (ix, iy, iz)*dx + U(-0.05, 0.05)*dx per component (drawn first from
numpy.random.default_rng(seed)); horizon delta = 3.015 dx; the bottom layer
iz = 0 is fixed; lateral faces are free from t = 0.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

DX = 0.01
DELTA_OVER_DX = 3.015


@dataclasses.dataclass(frozen=True)
class ColumnConfig:
    name: str
    nx: int
    ny: int
    nz: int
    seed: int
    suction_kpa: Optional[float]   # None -> drawn U(10, 40) kPa after the jitter
    steps: int
    precision: str                  # "fp64" or "mixed"
    checkpoint_every: int = 0
    plane: bool = False             # plane strain in the x-z plane (ny = 1)

    @property
    def n_points(self) -> int:
        return self.nx * self.ny * self.nz


CONFIGS: Dict[str, ColumnConfig] = {
    "C0": ColumnConfig("C0", 8, 8, 16, 0, 20.0, 200, "fp64"),
    "C1": ColumnConfig("C1", 40, 40, 80, 1, None, 2000, "fp64"),
    "C2": ColumnConfig("C2", 80, 80, 160, 2, 20.0, 1000, "mixed"),
    "C3": ColumnConfig("C3", 24, 24, 48, 3, 20.0, 1000, "fp64", checkpoint_every=50),
    "C4": ColumnConfig("C4", 128, 128, 256, 4, 20.0, 500, "mixed", checkpoint_every=25),
    "P0": ColumnConfig("P0", 24, 1, 48, 10, 20.0, 200, "fp64", plane=True),
    "P1": ColumnConfig("P1", 512, 1, 1024, 11, 20.0, 1000, "fp64", plane=True),
}

# Material constants.  Critical-state values (M, lambda, kappa, e0, tau,
# density, gravity) are those of the workload description; elastic moduli,
# over-consolidation ratio and retention-curve constants are the ones printed
# for the paper's column-collapse example (Section 4.2).
MATERIAL = dict(
    K=25.0e6,          # bulk modulus [Pa]
    mu=15.0e6,         # shear modulus [Pa]
    M=1.2,             # slope of the critical state line
    lam=0.1,           # compression index (lambda tilde)
    kap=0.02,          # swell index (kappa tilde)
    e0=0.8,            # initial void ratio
    tau=1.0e-3,        # Perzyna relaxation time [s]
    rho_sat=2000.0,    # bulk density of the column [kg/m^3]
    rho_w=1000.0,      # water density [kg/m^3]
    g=9.81,            # gravity [m/s^2]
    ocr=1.25,          # over-consolidation ratio
    a1=0.038, a2=3.49, n_vg=1.25,   # retention-curve constants
    b1=0.0, b2=1.0,    # apparent pre-consolidation exponents (Eq. 45)
)


def default_params(cfg: ColumnConfig, suction_pa: float, **over) -> dict:
    """Problem set-up constants for one column.

    Set-up readings (not the method):
      * rho_s: the stated density is the saturated bulk density, so the grain
        density follows from the mixture rule at S_r = 1:
        rho_s = (rho_sat - rho_w*phi0) / (1 - phi0).
      * eta: the Perzyna coefficient of Eq. 43 carries units Pa^3 s; the
        stated viscosity is a relaxation time tau, so eta = tau*K*p_ref^2
        with p_ref = rho_sat*g*H + s, a fixed stress scale of the column.
    """
    m = dict(MATERIAL)
    m.update(over)
    phi0 = m["e0"] / (1.0 + m["e0"])
    height = cfg.nz * DX
    p_ref = m["rho_sat"] * m["g"] * height + suction_pa
    return dict(
        delta=DELTA_OVER_DX * DX,
        K=m["K"], mu=m["mu"], M=m["M"], lam=m["lam"], kap=m["kap"],
        eta=m["tau"] * m["K"] * p_ref * p_ref,
        b1=m["b1"], b2=m["b2"],
        rho_s=(m["rho_sat"] - m["rho_w"] * phi0) / (1.0 - phi0),
        rho_w=m["rho_w"], a1=m["a1"], a2=m["a2"], n_vg=m["n_vg"],
        g=(0.0, 0.0, -m["g"]),
        dt=0.0,
        newton_tol=1e-13, newton_maxit=50,
        ocr=m["ocr"],
    )


def morton_order(lat: np.ndarray) -> np.ndarray:
    """Permutation that lists integer lattice coordinates (n, 3) in Morton
    (Z-curve) order: the bits of x, y and z interleaved, x lowest."""
    key = np.zeros(lat.shape[0], np.uint64)
    for b in range(21):
        for c in range(3):
            key |= ((lat[:, c].astype(np.uint64) >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + c)
    return np.argsort(key, kind="stable")


def make_column(cfg: ColumnConfig, seed: Optional[int] = None,
                suction_kpa: Optional[float] = None, jitter: float = 0.05,
                dims=None, fixed_base: bool = True, order: str = "lattice") -> dict:
    """Return the seeded column: arrays in caller (lattice) order plus params.

    Arrays (float64 unless stated):
      x0 (N,3), v0 (N,3) zeros, vol0 (N,), phi0 (N,), suction (N,) [Pa],
      fixed (N,) uint8, sig_geo (N,6) total K0 geostatic stress in Voigt
      order (xx, yy, zz, yz, xz, xy), tension positive.
    fixed_base=False frees the bottom layer (a column resting on a substrate).
    order="morton" numbers the points along the Morton curve of their lattice
    coordinates instead of lattice order (the same points and random draws).
    """
    nx, ny, nz = dims if dims is not None else (cfg.nx, cfg.ny, cfg.nz)
    if cfg.plane and ny != 1:
        raise ValueError("a plane-strain column has ny = 1")
    seed = cfg.seed if seed is None else seed
    rng = np.random.default_rng(seed)
    n = nx * ny * nz
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    lat = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    jit = rng.uniform(-jitter, jitter, (n, 3)) if jitter > 0 else np.zeros((n, 3))
    if cfg.plane:
        jit[:, 1] = 0.0
    x0 = (lat + jit) * DX
    if suction_kpa is None:
        suction_kpa = cfg.suction_kpa
    if suction_kpa is None:
        suction_kpa = float(rng.uniform(10.0, 40.0))
    s = suction_kpa * 1e3
    prm = default_params(cfg, s)
    prm["plane"] = 1 if cfg.plane else 0
    m = MATERIAL
    phi0 = m["e0"] / (1.0 + m["e0"])
    # K0 geostatic total stress: sigma_zz = -rho g depth, sigma_h = K0 sigma_zz,
    # K0 = nu/(1-nu) from the elastic moduli.
    nu = (3 * m["K"] - 2 * m["mu"]) / (2 * (3 * m["K"] + m["mu"]))
    k0 = nu / (1 - nu)
    top = (nz - 0.5) * DX
    szz = -m["rho_sat"] * m["g"] * (top - lat[:, 2] * DX)
    sig = np.zeros((n, 6))
    sig[:, 0] = k0 * szz
    sig[:, 1] = k0 * szz
    sig[:, 2] = szz
    fixed = ((lat[:, 2] == 0) & fixed_base).astype(np.uint8)
    if order == "morton":
        p = morton_order(lat.astype(np.int64))
        lat, x0, sig, fixed = lat[p], x0[p], sig[p], fixed[p]
    elif order != "lattice":
        raise ValueError("order is 'lattice' or 'morton'")
    return dict(
        n=n, dims=(nx, ny, nz), lattice=lat.astype(np.int64),
        x0=np.ascontiguousarray(x0),
        v0=np.zeros((n, 3)),
        vol0=np.full(n, DX ** 2 if cfg.plane else DX ** 3),
        phi0=np.full(n, phi0),
        suction=np.full(n, s),
        fixed=fixed,
        sig_geo=np.ascontiguousarray(sig),
        params=prm,
        suction_kpa=suction_kpa,
        order=order,
    )


def random_velocity(n: int, seed: int, scale: float = 1e-2) -> np.ndarray:
    """Seeded velocity field U(-scale, scale) [m/s] for one-step checks."""
    return np.random.default_rng(seed).uniform(-scale, scale, (n, 3))


# Uniaxial compression (Section 4.1): an elastic specimen at zero suction
# pressed along x.  The paper's specimen is 2D (12,000 points, geometry in a
# figure that is not available); this is a synthetic 3D bar with its stated
# constants.
UNIAXIAL = dict(
    spacing=0.005,     # distance between adjacent points [m]
    K=25.0e6, mu=15.0e6,
    rho_s=2200.0,      # solid skeleton density [kg/m^3]
    phi0=0.2,          # initial porosity
    u_total=0.5e-3,    # applied displacement [m]
    t_load=0.1,        # loading time [s]
    dt_dynamic=3.0e-6, # time step of the dynamic case [s]
)


def make_uniaxial_block(m: int, dims=(40, 12, 12), sigma0: float = -1.0) -> dict:
    """Bar of nx x ny x nz points on the unjittered cubic lattice of spacing
    0.005 m, horizon delta = m * spacing (m = 2 or 3; families of 32 and 122
    in the interior), zero suction, no
    gravity, isotropic elastic range only: the initial effective stress is a
    negligible isotropic sigma0 [Pa] and the over-consolidation ratio is huge
    (1e12), so the critical-state yield surface is never reached.  Boundary
    codes: the face ix = 0 fixed (1); the face ix = nx - 1 driven (2) at the
    constant velocity -u_total / t_load along x; other faces free.  Arrays in
    the layout of make_column."""
    u = UNIAXIAL
    nx, ny, nz = dims
    n = nx * ny * nz
    h = u["spacing"]
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    lat = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)
    x0 = lat.astype(np.float64) * h
    fixed = np.zeros(n, np.uint8)
    fixed[lat[:, 0] == 0] = 1
    fixed[lat[:, 0] == nx - 1] = 2
    v0 = np.zeros((n, 3))
    v0[lat[:, 0] == nx - 1, 0] = -u["u_total"] / u["t_load"]
    sig = np.zeros((n, 6))
    sig[:, :3] = sigma0
    m_ = MATERIAL
    # delta a hair above m * spacing: on the unjittered lattice the points at
    # exactly m spacings would otherwise enter or not by rounding
    prm = dict(delta=m * h * (1.0 + 1e-9), K=u["K"], mu=u["mu"], M=m_["M"], lam=m_["lam"], kap=m_["kap"],
               eta=1.0e30, b1=m_["b1"], b2=m_["b2"], rho_s=u["rho_s"], rho_w=m_["rho_w"], a1=m_["a1"],
               a2=m_["a2"], n_vg=m_["n_vg"], g=(0.0, 0.0, 0.0), dt=0.0, newton_tol=1e-13, newton_maxit=50,
               ocr=1.0e12, plane=0)
    return dict(n=n, dims=tuple(dims), lattice=lat.astype(np.int64), x0=np.ascontiguousarray(x0), v0=v0,
                vol0=np.full(n, h ** 3), phi0=np.full(n, u["phi0"]), suction=np.zeros(n), fixed=fixed,
                sig_geo=sig, params=prm, suction_kpa=0.0, m=m)


def subsample_ids(n: int, every: int = 64) -> np.ndarray:
    """Every `every`-th caller id, the 1/64 subsample of the mixed column."""
    return np.arange(0, n, every, dtype=np.int64)


def runout_objective_weights(lattice: np.ndarray, dims) -> dict:
    """Index sets for the runout + settlement objective: the initial top layer
    and the column axis.  Pure bookkeeping."""
    nx, ny, nz = dims
    top = np.nonzero(lattice[:, 2] == nz - 1)[0]
    axis = np.array([(nx - 1) * 0.5 * DX, (ny - 1) * 0.5 * DX])
    return dict(top=top, axis=axis, height=(nz - 0.5) * DX)


# Substrate set-up for contact (Section 4.2: C_s, mu_f, delta_c = 0.8 dx).
CONTACT = dict(mu_f=0.25, delta_c_over_dx=0.8, cs_ratio=1.0)


def make_substrate(col: dict, extent: float = 1.0, layers: int = 1, mu_f: Optional[float] = None,
                   cs_ratio: Optional[float] = None, delta_c_over_dx: Optional[float] = None) -> dict:
    """Rigid substrate lattice under a column, as a contact description.

    Sites at origin + dx (a, b, -c) for a < n[0], b < n[1], c < n[2] =
    layers, spacing dx: the column footprint plus `extent` times its larger
    width on every side.  The top layer lies 0.9 delta_c below the lowest
    point, so no point starts within the cut-off.

    Set-up readings (not the method):
      * C_s: the paper's value belongs to its 2D model.  Here T_c is a force
        per volume squared, so C_s carries N/m^7 (N/m^6 per unit thickness
        in plane strain).  It is set so that one site's contact stiffness
        2 C_s V_i V_s equals cs_ratio times K dx, the axial stiffness of a
        point's cell: C_s = cs_ratio K / (2 dx^(d+2)), d = 3 or 2.
      * delta_c = 0.8 dx and mu_f = 0.25 as stated for the collapse examples.
    """
    c = dict(CONTACT)
    if mu_f is not None:
        c["mu_f"] = mu_f
    if cs_ratio is not None:
        c["cs_ratio"] = cs_ratio
    if delta_c_over_dx is not None:
        c["delta_c_over_dx"] = delta_c_over_dx
    prm = col["params"]
    x0 = col["x0"]
    lo, hi = x0.min(axis=0), x0.max(axis=0)
    width = float(max(hi[0] - lo[0], hi[1] - lo[1]))
    ox = float(lo[0] - extent * width)
    nx = int(math.ceil((hi[0] + extent * width - ox) / DX)) + 1
    if prm.get("plane"):
        oy, ny = float(lo[1]), 1                  # one row of sites in the plane
    else:
        oy = float(lo[1] - extent * width)
        ny = int(math.ceil((hi[1] + extent * width - oy) / DX)) + 1
    dc = c["delta_c_over_dx"] * DX
    d = 2 if prm.get("plane") else 3
    return dict(cs=c["cs_ratio"] * prm["K"] / (2.0 * DX ** (d + 2)), mu_f=c["mu_f"],
                delta_c=dc, origin=[ox, oy, float(lo[2] - 0.9 * dc)], spacing=DX, n=[nx, ny, int(layers)])
