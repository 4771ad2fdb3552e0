/* ulppm.h -- C ABI of the MI355X (gfx950) library for the per-step bond loop of
 * updated Lagrangian unsaturated periporomechanics (Menon & Song, arXiv
 * 2203.05562): families in the deformed configuration, bond-associated
 * sub-horizon shape tensors and velocity gradients, the critical-state
 * Perzyna update of the effective force state under constant suction, the
 * nodal force gather, and the central-difference Newmark update.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All state arrays are caller-owned DEVICE memory (e.g. torch tensors on
 *   cuda:0), FP64, structure-of-arrays, length n, indexed by the caller's
 *   point ids.  The library never frees or reallocates them.
 * - Symmetric tensors (stress) are six separate arrays in Voigt order
 *   (xx, yy, zz, yz, xz, xy); tension positive (Section 1 of the paper),
 *   pore-water pressure p_w = -s with suction s >= 0 [Pa].
 * - The context owns only its scratch (cell lists, families, reverse-bond
 *   index, bond force states, reduction partials), sized at ulppm_create
 *   for n_points and max_family members per family.
 * - Every call enqueues its kernels on the context's HIP stream, in order;
 *   a call synchronises that stream only where it must read device results
 *   back to the host (error counters, reports, bond counts).
 * - Return values are ulppm_status codes.  Kernels never trap: they raise
 *   device counters that the host turns into codes, with text available from
 *   ulppm_last_error.  After an error the state is finite or flagged but
 *   otherwise unspecified; restore it from a copy.
 * - One context per host thread / stream.  The only global state is the
 *   static scratch of ulppm_forces_static, one array per device.
 */
#ifndef ULPPM_H
#define ULPPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ulppm_ctx ulppm_ctx;

typedef enum {
  ULPPM_OK = 0,
  ULPPM_E_ARG = -1,       /* bad argument (NULL pointer, size mismatch, n out of range) */
  ULPPM_E_CAPACITY = -2,  /* a family exceeded max_family, or col_cap too small */
  ULPPM_E_NOCONV = -4,    /* Newton of the return map did not converge (Section 3.2.1) */
  ULPPM_E_NONFINITE = -5, /* NaN/Inf produced in velocities or accelerations */
  ULPPM_E_ENERGY = -6,    /* energy balance check of Eq. 69 failed */
  ULPPM_E_HIP = -7        /* a HIP runtime call failed */
} ulppm_status;

enum { ULPPM_FP64 = 0, ULPPM_MIXED = 1 };

/* How bond force states are formed from the sub-horizon stresses.
 * ULPPM_FORCE_CONJUGATE (default): the force state of bond (i,k) collects the
 *   sub-horizon force state (V_j/V_H)(sigma_ij + S_r s 1) K_ij^{-1} zeta_ik of
 *   every sub-horizon S_ij that holds k (Eqs. 27, 31 and the double integral
 *   of Eq. 35), so its power equals the volume-weighted mean of sigma_ij : L_ij
 *   that also updates the point history.
 * ULPPM_FORCE_EQ51: Eq. 51 as printed, T_ij = varpi_ij (sigma_ij + S_r s 1)
 *   K_ij^{-1} zeta_ij, the bond's own term only.  With history stored on the
 *   points this form is linearly unstable (flutter); kept for comparison.
 * ULPPM_FORCE_STANDARD: the standard, unstabilised correspondence model of
 *   Eqs. 12-14: one stress per point, updated from the full-horizon gradient
 *   L_i, and T_ij = (sigma_i + S_r s 1) K_i^{-1} zeta_ij.  It has the
 *   zero-energy modes the sub-horizons remove (Eqs. 20-21); kept as the
 *   comparison model.  No sub-horizons are formed (n_tests = n_triples = 0). */
enum { ULPPM_FORCE_CONJUGATE = 0, ULPPM_FORCE_EQ51 = 1, ULPPM_FORCE_STANDARD = 2 };

/* Where the history (effective stress, p_c) lives between steps.
 * ULPPM_HISTORY_POINT (default): on the points; every bond starts each step
 *   from its point's history, and the point's new history is the
 *   volume-weighted mean of its bonds' updated states.
 * ULPPM_HISTORY_BOND: on the bonds; a bond keeps its own state from step to
 *   step while it stays in the family, a bond that enters a family starts
 *   from its point's history, and the points still receive the mean (for
 *   output and for new bonds).  The states live in the context
 *   (ulppm_history_reserve), ulppm_init_state clears them, and only
 *   ulppm_step uses them (ulppm_forces starts every bond from its point);
 *   its reverse is ulppm_adjoint_step_bond_history. */
enum { ULPPM_HISTORY_POINT = 0, ULPPM_HISTORY_BOND = 1 };

/* Material and integration parameters, copied by value on every call. */
typedef struct {
  double delta;                 /* horizon, constant in the current configuration (Eq. 1) [m] */
  double K, mu;                 /* elastic bulk and shear moduli (Eq. 41) [Pa] */
  double M;                     /* slope of the critical state line (Eq. 40) */
  double lam, kap;              /* compression / swell indices (Eq. 46) */
  double eta;                   /* Perzyna viscosity coefficient (Eq. 43) [Pa^3 s] */
  double b1, b2;                /* apparent pre-consolidation exponents (Eq. 45) */
  double rho_s, rho_w;          /* solid grain and water densities (Eqs. 3, 48) [kg/m^3] */
  double a1, a2, n_vg;          /* retention-curve constants (Eq. 15), suction in kPa */
  double g[3];                  /* gravity [m/s^2] */
  double dt;                    /* time step [s] */
  double newton_tol;            /* relative tolerance of the return-map Newton */
  int32_t newton_maxit;         /* Newton iteration cap */
  int32_t precision;            /* ULPPM_FP64 or ULPPM_MIXED */
  int32_t energy_check;         /* nonzero: check Eq. 69 at the end of ulppm_step */
  int32_t force_mode;           /* ULPPM_FORCE_CONJUGATE or ULPPM_FORCE_EQ51 */
  double energy_tol;            /* epsilon of Eq. 69 (the paper uses ~1e-2) */
  int32_t timing;               /* nonzero: time each phase of ulppm_step with HIP events */
  int32_t plane;                /* 1: plane strain in the x-z plane (see below); 0: 3D */
  int32_t history;              /* ULPPM_HISTORY_POINT or ULPPM_HISTORY_BOND */
  int32_t pad;
} ulppm_params;

/* Plane strain (plane = 1).  All points lie in one x-z plane (equal y) with
 * v_y = 0, and every volume is an area times a unit thickness.  Shape tensors
 * are inverted on their x-z block (a bond is inactive with fewer than two
 * sub-horizon members or det <= 1e-12 (tr/2)^2), so gradients, force states
 * and forces have no y component, while the stress keeps all six components
 * (sigma_yy from the zero out-of-plane strain).  ulppm_dt_crit uses the plane
 * bond micromodulus C = 72K/(5 pi delta^3) per unit thickness, and contact
 * sites weigh spacing^2.  The adjoint entry points differentiate the same
 * block inversion (its derivative has no y row or column). */

/* Point state: caller-owned device arrays of length n (SoA). */
typedef struct {
  int64_t n;
  double *x0[3];                /* initial positions (read only) */
  double *u[3], *uc[3];         /* displacement and its Kahan compensation term */
  double *v[3], *a[3];          /* velocity, acceleration */
  double *vol, *phi, *J;        /* current volume, porosity, volume ratio */
  double *Sr, *mass, *s;        /* degree of saturation, lumped mass, suction [Pa] (read only) */
  double *sig[6];               /* effective stress (Voigt), the point history */
  double *pc;                   /* saturated pre-consolidation pressure p_c < 0, point history */
  const uint8_t *fixed;         /* boundary code: 0 free; 1 fixed (v = a = 0); 2 driven: the point keeps
                                   its velocity v (a = 0), a prescribed-velocity boundary.  The work
                                   done by fixed and driven points is not booked in the energies, so
                                   Eq. 69 is meaningful only without driven points. */
} ulppm_state;

/* Host-side report of the last ulppm_step / ulppm_forces call. */
typedef struct {
  double W_int, W_ext, W_kin;   /* energies of Eqs. 66-68, accumulated since create/reset */
  int64_t n_bonds;              /* directed bonds of the last step (sum of family sizes) */
  int64_t n_degenerate;         /* bonds with |S_ij| < 3 or singular K_ij (inactive), summed */
  int64_t n_plastic;            /* bond updates that took the viscoplastic branch, summed */
  int64_t max_newton;           /* largest Newton iteration count */
  int64_t n_noconv;             /* Newton failures, summed */
  int64_t n_tests;              /* sub-horizon membership tests (sum |H_i|^2), summed */
  int64_t n_triples;            /* sub-horizon members visited (sum |S_ij|), summed */
  int64_t max_family;           /* largest family of the last rebuild */
  int64_t steps;                /* steps taken by the call */
  int64_t n_bond_updates;       /* directed bonds summed over the call's steps */
  int64_t timed_steps;          /* steps covered by the phase timings (p->timing) */
  double t_predict_ms;          /* summed HIP-event durations per phase over timed steps */
  double t_family_ms;
  double t_bond_ms;             /* the bond kernel alone */
  double t_gather_ms;
  double t_kin_ms;              /* point kinematics before the bond kernel */
  int64_t n_rebuilds;           /* candidate-list rebuilds (a point moved half the skin), summed */
} ulppm_report;

/* Create a context for up to n_points points and max_family members per family
 * (0 selects 152: a jittered cubic lattice with delta = 3.015 dx starts with
 * at most about 121, and compression adds members).  The bond kernel's LDS is
 * sized by max_family (about 192 bytes per member in FP64): 152 fits four
 * FP64 bond workgroups per CU, 128 six, and a max_family of at most 64 runs
 * the bond kernel with one wave per point.  A family larger than max_family
 * is an error (ULPPM_E_CAPACITY), never a truncation.  hip_stream is a
 * hipStream_t (NULL = the null stream).
 * Allocates all scratch now; afterwards only ulppm_adjoint_reserve and
 * ulppm_history_reserve allocate.
 * Errors: ULPPM_E_ARG (n_points <= 0 or > 2^31-1, max_family > 1024),
 * ULPPM_E_HIP (allocation failed). */
int ulppm_create(ulppm_ctx **out, int64_t n_points, int32_t max_family, void *hip_stream);

/* Release the context's scratch.  Never touches caller memory. */
int ulppm_destroy(ulppm_ctx *ctx);

/* Text of the last error on this context (static storage inside the context). */
const char *ulppm_last_error(const ulppm_ctx *ctx);

/* Contact with a rigid substrate (Eqs. 91-93), held by the context.
 * The substrate is a lattice of fixed sites origin + spacing (a, b, -c),
 * a < n[0], b < n[1], c < n[2] (layers go down from origin), each of volume
 * spacing^3; it carries contact only (no bonds with the points).  For point i
 * and a site s with Y = x_s - x_i and |Y|^2 < delta_c^2 (rounded as
 * ((Y0^2 + Y1^2) + Y2^2)):
 *   T_c = -cs (delta_c - |Y|) Y/|Y|                       (Eq. 91)
 *   T_f = -mu_f sign(d|Y|/dt) T_c, d|Y|/dt = -Y.v_i/|Y|    (Eq. 92 as printed)
 * and the nodal force gains V_i sum_s 2 (T_c + T_f) V_s: the contact integrand
 * of Eq. 93, with the reverse pair's states T_c' = -T_c, T_f' = -T_f.  v_i is
 * the step's velocity predictor in ulppm_step and the state velocity in
 * ulppm_forces / ulppm_init_state; V_i the point volume of step n.  cs is a
 * force per volume squared per length [N/m^7].  The work of contact forces is
 * booked in W_int (the substrate is at rest and does no work), so the energy
 * balance of Eq. 69 is unchanged.  ulppm_dt_crit ignores contact.  The
 * adjoint entry points include the contact forces, with the sign of Eq. 92
 * frozen like the other branches of the step. */
typedef struct {
  double cs;                    /* contact stiffness C_s of Eq. 91 [N/m^7]; <= 0 turns contact off */
  double mu_f;                  /* friction coefficient of Eq. 92 */
  double delta_c;               /* cut-off distance of the repulsion [m] */
  double origin[3];             /* position of site (0, 0, 0) [m] */
  double spacing;               /* lattice spacing [m] */
  int32_t n[3];                 /* sites along x, y and layers downward */
  int32_t pad;
} ulppm_contact;

/* Attach (or, with c == NULL or c->cs <= 0, detach) the substrate; the
 * description is copied into the context and used by every later
 * ulppm_init_state, ulppm_forces, ulppm_step and ulppm_adjoint_step.
 * Errors: ULPPM_E_ARG (spacing or delta_c <= 0, a count < 1, or more than
 * 2^31-1 sites). */
int ulppm_set_contact(ulppm_ctx *ctx, const ulppm_contact *c);

/* Initial conditions of the explicit scheme (Algorithm 2, set-up and initial
 * acceleration).  On entry sig holds the TOTAL stress, phi the initial
 * porosity, vol the initial volume, s the suction, v the initial velocity.
 * On return: u = uc = 0, J = 1, Sr from Eq. 15, sig = effective stress
 * total - Sr s 1 (Eq. 2 with p_w = -s), pc the pre-consolidation pressure of
 * the yield surface (Eq. 40) through that stress scaled by ocr and inverted
 * through Eq. 45, mass from Eq. 48, and a = f/mass + g with the nodal force of
 * Algorithm 1 at bond stress = point stress (fixed points: a = 0).
 * Energies are reset to zero.  Errors: ULPPM_E_ARG, ULPPM_E_CAPACITY, ULPPM_E_HIP. */
int ulppm_init_state(ulppm_ctx *ctx, ulppm_state *state, const ulppm_params *p, double ocr);

/* Critical time step of Eq. 65, read as sqrt(2(1-phi) rho_s / sum_j V_j C/|zeta_ij|)
 * with the bond micro-modulus C = 18K/(pi delta^4); the minimum over points with a
 * non-empty family at the current positions x0+u is written to *dt_out (host).
 * Errors: ULPPM_E_ARG, ULPPM_E_CAPACITY, ULPPM_E_HIP. */
int ulppm_dt_crit(ulppm_ctx *ctx, const ulppm_state *state, const ulppm_params *p, double *dt_out);

/* Neighbour search of Algorithm 1 (Eq. 1 with a constant horizon in the
 * current configuration): family H_i = { j != i : |x_j - x_i| <= delta } at
 * x = x0 + u, with the squared distance rounded as ((dx^2 + dy^2) + dz^2), no
 * fused multiply-add.  Builds the context's internal CSR and reverse-bond
 * index.  If row_ptr (n+1, device int64) is non-NULL the families are exported
 * in the caller's ids, rows ascending; col (device int32, col_cap entries) is
 * filled when non-NULL and large enough.  *n_bonds_out (host) receives the bond
 * count.  Errors: ULPPM_E_ARG, ULPPM_E_CAPACITY (family > max_family or
 * col_cap < bonds), ULPPM_E_HIP. */
int ulppm_build_families(ulppm_ctx *ctx, const ulppm_state *state, const ulppm_params *p,
                         int64_t *row_ptr, int32_t *col, int64_t col_cap, int64_t *n_bonds_out);

/* Algorithm 1 alone at the current state, without mutating it: families at
 * x0 + u; sub-horizon shape tensors (Eq. 23) and velocity gradients (Eq. 57)
 * from the velocities v; strain increment dt_inc * sym(L_ij) (Eqs. 26, 59);
 * bond stress from the Perzyna return map (Section 3.2.1), or equal to the
 * point stress when dt_inc == 0; force states T_ij (Eqs. 27, 31-32, 35, or
 * Eqs. 51, 53 as printed, per p->force_mode); nodal
 * force f_i = sum_j (T_ij - T_ji) V_i V_j (Eqs. 49-50 with the sign of Eq. 33)
 * written to f[3] (device, length n each).  T_out, if non-NULL, receives the
 * bond force states as three device arrays of length n_bonds (x, y, z), in the
 * CSR order of ulppm_build_families.  rep (host) may be NULL.
 * With a substrate attached (ulppm_set_contact) f includes the contact forces.
 * Errors: ULPPM_E_ARG, ULPPM_E_CAPACITY, ULPPM_E_NOCONV, ULPPM_E_HIP. */
int ulppm_forces(ulppm_ctx *ctx, const ulppm_state *state, const ulppm_params *p, double dt_inc,
                 double *f[3], double *T_out[3], ulppm_report *rep);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ulppm_forces
 * without a context.  The scratch it needs lives in a file-scope device
 * array of the library, 16 MiB on each GPU the library runs on, held until
 * the process ends; it serves at most ULPPM_STATIC_MAX_POINTS points and
 * ULPPM_STATIC_MAX_FAMILY members per family.  The first call on a device
 * (with that device current) looks the array up; no call allocates device
 * memory.  Arguments and results are those of ulppm_forces (no substrate is
 * attached); hip_stream is a hipStream_t (NULL = the null stream).  Every call
 * on one device shares that device's array, which keeps the last call's
 * contents (each call clears what must start at zero): calls that overlap on
 * one device, on any streams or host threads, race and must not be issued.
 * Errors: ULPPM_E_ARG (state NULL, n < 1 or n > ULPPM_STATIC_MAX_POINTS,
 * other arguments as ulppm_forces), ULPPM_E_CAPACITY (a family larger than
 * ULPPM_STATIC_MAX_FAMILY), ULPPM_E_NOCONV, ULPPM_E_HIP. */
#define ULPPM_STATIC_MAX_POINTS 2048
#define ULPPM_STATIC_MAX_FAMILY 128
int ulppm_forces_static(const ulppm_state *state, const ulppm_params *p, double dt_inc, double *f[3],
                        double *T_out[3], ulppm_report *rep, void *hip_stream);

/* Algorithm 2, n_steps explicit central-difference Newmark steps (beta1 = 1/2,
 * beta2 = 0, Eqs. 60-64), state updated in place.  Each step: velocity
 * predictor and boundary conditions; displacement with Kahan compensation;
 * family rebuild; Algorithm 1 with dt_inc = dt (volume change from the
 * full-horizon gradient, Eqs. 16-17; saturation Eq. 15; mass Eq. 48; point
 * history = volume-weighted mean of its bond states); acceleration a = f/M + g
 * (Eq. 62 with the sign of Eq. 33); velocity corrector (Eq. 63); energy
 * increments of Eqs. 66-68.  rep (host) may be NULL.  With p->energy_check the
 * balance of Eq. 69 is checked after the last step (ULPPM_E_ENERGY).
 * Errors: ULPPM_E_ARG, ULPPM_E_CAPACITY, ULPPM_E_NOCONV, ULPPM_E_NONFINITE,
 * ULPPM_E_ENERGY, ULPPM_E_HIP. */
int ulppm_step(ulppm_ctx *ctx, ulppm_state *state, const ulppm_params *p, int32_t n_steps,
               ulppm_report *rep);

/* Allocate the bond states of ULPPM_HISTORY_BOND: two buffers of 8 doubles
 * per bond slot (n_points * max_family) and a copy of the families they
 * follow; if ulppm_adjoint_reserve has run, also the 16 doubles per bond
 * slot of ulppm_adjoint_step_bond_history.  Call once before the first
 * ulppm_step with history = ULPPM_HISTORY_BOND.  Errors: ULPPM_E_ARG,
 * ULPPM_E_HIP. */
int ulppm_history_reserve(ulppm_ctx *ctx);

/* Copy the bond history of the last step to caller device memory: row_out
 * (n+1 int64), col_out (int32) and st_out (8 doubles per bond: sigma in Voigt
 * order, p_c, 0), each may be NULL; *nb_out (host) receives the bond count.
 * With all three NULL only the count is returned.  Errors: ULPPM_E_ARG (no
 * history held), ULPPM_E_CAPACITY (cap < bonds), ULPPM_E_HIP. */
int ulppm_history_export(ulppm_ctx *ctx, int64_t *row_out, int32_t *col_out, double *st_out, int64_t cap,
                         int64_t *nb_out);

/* Load a bond history into the context, as ulppm_history_export wrote it
 * after some step (device arrays: row n+1 int64, col n_bonds int32, st 8
 * doubles per bond), so that the next ulppm_step with history =
 * ULPPM_HISTORY_BOND carries these states; restarting from a checkpoint
 * needs it.  n_bonds = 0 clears the history (every bond then starts from its
 * point, as after ulppm_init_state).  The row must have been built for the
 * same n and family capacity.  Errors: ULPPM_E_ARG (not reserved, sizes out of
 * range), ULPPM_E_HIP. */
int ulppm_history_import(ulppm_ctx *ctx, int64_t n, const int64_t *row, const int32_t *col, const double *st,
                         int64_t n_bonds);

/* Allocate the scratch of ulppm_adjoint_step (a copy of one state, the point
 * adjoints and 16 doubles per bond slot) and, if ulppm_history_reserve has
 * run, the 16 doubles per bond slot of ulppm_adjoint_step_bond_history.  Call
 * once, before the first adjoint step; the adjoint steps themselves never
 * allocate.  Errors: ULPPM_E_ARG, ULPPM_E_HIP. */
int ulppm_adjoint_reserve(ulppm_ctx *ctx);

/* Reverse mode of one step n -> n+1 (the workload's hand-written adjoint of
 * Algorithm 2 driving Algorithm 1), with that step's families, sub-horizons,
 * degenerate bonds and elastic/plastic branches frozen.  state_np1, if not
 * NULL, must be the state ulppm_step produced from state_n with the same
 * params (a checkpointed sweep has it); then only the positions, half-step
 * velocities and families are rebuilt.  If NULL, the forward step is re-run
 * from state_n on scratch.  Propagates adj_np1 (the adjoint of state n+1, same
 * layout as a state: u, uc, v, a, vol, phi, J, Sr, mass, sig, pc; device
 * arrays) back through the corrector, the gather (Eqs. 49-50), the
 * conjugate force states, the bond tail (inversion, Eqs. 25-26 and 59, the
 * return map by the implicit-function theorem at its solution), the
 * sub-horizon sums (Eqs. 22-25, 57), the point kinematics (Eqs. 15-17, 48)
 * and the predictor (Eqs. 60-61, 64), writing the adjoint of state n into
 * adj_n.  adj_n->s receives adj_np1->s plus this step's suction adjoint and
 * adj_n->x0 receives adj_np1->x0 plus the adjoint of x0, so both accumulate
 * over a backward sweep; adj_n->Sr and adj_n->mass are zero (the step
 * recomputes them).  theta_bar (device, 4 doubles) accumulates the adjoints of
 * (M, lam, kap, eta).  adj_n may alias adj_np1.  p must have conjugate
 * force states.  With p->precision = ULPPM_FP64 the reverse is FP64
 * throughout; with ULPPM_MIXED its two membership-matrix sweeps (the re-run
 * of the sub-horizon sums and the reverse of those sums) run on FP32 matrix
 * cores with FP32 accumulation, and everything else stays FP64.  state_n and
 * state_np1 may come from a mixed-precision run (the reverse is then taken
 * about that run's states).
 * rep (host) may be NULL; it receives the step's family counts and, when the
 * step is re-run from state_n, the re-run's counters (with state_np1 given
 * only the families are rebuilt, and the return-map counters stay zero).
 * The step's workgroup memory is laid out for the largest family that the
 * forward calls on this context have reported (for this step's own largest
 * family when none has); a family larger than that fails the step with
 * ULPPM_E_CAPACITY, after which adj_n and theta_bar are not usable.
 * Errors: ULPPM_E_ARG, ULPPM_E_CAPACITY, ULPPM_E_NOCONV, ULPPM_E_HIP. */
int ulppm_adjoint_step(ulppm_ctx *ctx, const ulppm_state *state_n, const ulppm_state *state_np1,
                       const ulppm_params *p, const ulppm_state *adj_np1, ulppm_state *adj_n,
                       double *theta_bar, ulppm_report *rep);

/* Reverse mode of one step n -> n+1 with the history on the bonds
 * (p->history = ULPPM_HISTORY_BOND; an alternative reading of the paper's
 * history, see ULPPM_HISTORY_BOND), otherwise as ulppm_adjoint_step.
 * state_np1 is required.  row_n (n+1 int64), col_n (n_bonds_n int32) and
 * hist_n (8 doubles per bond: sigma in Voigt order, p_c, 0) are the families
 * and bond states after step n, as ulppm_history_export returned them after
 * the step that produced state_n (device arrays; n_bonds_n = 0 and NULLs
 * when step n is the first: every bond then starts from its point).
 * hist_bar_np1 is the adjoint of the bond states after step n+1, in the
 * order of the families of state_np1 (the order ulppm_history_export gives
 * after step n+1).  Writes hist_bar_n, the adjoint of hist_n (same layout,
 * zero for bonds not carried into step n+1); a bond that enters a family
 * hands its start-state adjoint to its point's history (adj_n->sig, pc).
 * Needs ulppm_history_reserve and ulppm_adjoint_reserve (the second of them
 * reserves 16 doubles per bond slot for this call); allocates nothing itself.
 * Errors: ULPPM_E_ARG, ULPPM_E_CAPACITY, ULPPM_E_NOCONV, ULPPM_E_HIP. */
int ulppm_adjoint_step_bond_history(ulppm_ctx *ctx, const ulppm_state *state_n, const ulppm_state *state_np1,
                                    const ulppm_params *p, int64_t n_bonds_n, const int64_t *row_n,
                                    const int32_t *col_n, const double *hist_n, const double *hist_bar_np1,
                                    const ulppm_state *adj_np1, ulppm_state *adj_n, double *hist_bar_n,
                                    double *theta_bar, ulppm_report *rep);

/* Reverse of ulppm_init_state (the initial conditions of Algorithm 2) at the
 * state state0 it produced with the same p and ocr.  adj0 is the adjoint of
 * that state (after a backward sweep of ulppm_adjoint_step, the adjoint of
 * state 0).  Writes s_bar (device, n doubles): the adjoint of each point's
 * suction through the initial saturation (Eq. 15), effective stress (Eq. 2),
 * pre-consolidation (Eqs. 40, 45), mass (Eq. 48) and, through the mass, the
 * initial acceleration (Eq. 62), plus adj0->s.  Adds the pre-consolidation's
 * dependence on M to theta_bar[0] (device, 4 doubles as in
 * ulppm_adjoint_step).  The initial nodal force depends on the total stress
 * only (Eq. 32 at zero strain increment), so neither suction nor M reach it.
 * The adjoint of the initial velocity is adj0->v unchanged.  Needs
 * ulppm_adjoint_reserve.  Errors: ULPPM_E_ARG, ULPPM_E_HIP. */
int ulppm_adjoint_init(ulppm_ctx *ctx, const ulppm_state *state0, const ulppm_params *p, double ocr,
                       const ulppm_state *adj0, double *s_bar, double *theta_bar);

/* Host-only self-check (no GPU call) of the library's hand-written reverse of the
 * per-bond tail (inversion, velocity gradient, strain increment, Perzyna return
 * map with its implicit-function adjoint, force-state factor) against central
 * finite differences on n_cases random bonds, alternating elastic and plastic
 * branches.  *max_rel receives the largest relative gradient error over all
 * inputs and the parameters (M, lam, kap, eta); *n_plastic the plastic cases.
 * Errors: ULPPM_E_ARG, ULPPM_E_NOCONV. */
int ulppm_selfcheck_tail(const ulppm_params *p, int32_t seed, int32_t n_cases, double *max_rel,
                         int32_t *n_plastic);

/* Zero the accumulated energies W_int, W_ext (W_kin is recomputed each step). */
int ulppm_reset_energy(ulppm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* ULPPM_H */
