// ulppm_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, obviously-correct FP64 CPU implementation of one explicit
// Newmark step of updated Lagrangian unsaturated periporomechanics with
// bond-associated sub-horizons (Menon & Song, "Updated Lagrangian unsaturated
// periporomechanics for extreme large deformation in unsaturated porous
// media", arXiv 2203.05562).  It follows the paper's Algorithm 2 driving
// Algorithm 1, loop by loop, in original point order.  Only the tests, the
// smoke check and the CPU-baseline leg of the benchmark may load it; the GPU
// library never does, and the two share no code.
//
// Every arithmetic step is templated on the scalar type R.  R = double is the
// oracle proper; R = Dual (value + one tangent) gives forward-mode directional
// derivatives of the same arithmetic, the CPU reference for the GPU adjoint.
// Set decisions (families, sub-horizons, degeneracy, elastic/plastic branch)
// are always taken on the value part.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fopenmp -shared -fPIC.
// No FMA contraction, so the canonical distance predicate below rounds each
// product.
//
// Readings of points where the paper is silent or garbled (listed in full in
// the design notes of the repository):
//   families exclude the point itself; the sub-horizon of bond (i,j) is
//   {k in H_i : |x_k - x_j| <= delta}; influence function = 1; geometry at
//   x^{n+1}, relative velocities from the Newmark velocity predictor, volumes
//   of step n as quadrature weights; D_ij = sym(L_ij); history on points as the
//   volume-weighted mean of the bond states; backward-Euler Perzyna return in
//   (p, q, p_c) with the hardening exponent signed as Eq. 46 requires;
//   retention exponent -(n-1)/n with suction in kPa; J increment
//   1/det(I - dt L_i); EOM sign of Eq. 33; the force state of bond (i,k)
//   collects the sub-horizon force states of all sub-horizons holding k
//   (Eqs. 27, 31, 35), since keeping only the bond's own term (Eq. 51) with
//   point-stored history is linearly unstable (flutter); contact (Eqs. 91-93)
//   with a rigid substrate of lattice sites, the pair integrand of Eq. 93
//   equal to 2 (T_c + T_f), and the friction term of Eq. 92 as printed, along
//   the pair direction; plane strain as the x-z plane with unit thickness, the
//   shape tensors inverted on their x-z block and the bond micromodulus
//   72 K / (5 pi delta^3) in the time-step bound.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

namespace {

// ---------------------------------------------------------------- scalars --

struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}  // NOLINT: implicit on purpose
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline Dual exp(Dual a) { double e = std::exp(a.v); return {e, e * a.d}; }
inline Dual log(Dual a) { return {std::log(a.v), a.d / a.v}; }
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return {s, s > 0 ? a.d / (2 * s) : 0.0};
}
// a^b for a > 0
inline Dual pow(Dual a, Dual b) {
  double p = std::pow(a.v, b.v);
  return {p, p * (b.d * std::log(a.v) + b.v * a.d / a.v)};
}
inline double val(double a) { return a; }
inline double val(Dual a) { return a.v; }
using std::exp;
using std::log;
using std::pow;
using std::sqrt;

// --------------------------------------------------------------- params --

struct Params {             // mirrors OracleParams below, in scalar type R
  double delta;
  double K, mu, M, lam, kap, eta, b1, b2;
  double rho_s, rho_w, a1, a2, n_vg;
  double g[3];
  double dt;
  double newton_tol;
  int newton_maxit;
  int force_mode;           // 0: conjugate force states (default), 1: Eq. 51 as printed,
                            // 2: standard full-horizon correspondence (Eq. 14)
  // contact with a rigid substrate (Eqs. 91-93); cs == 0 turns it off
  double cs, mu_f, delta_c;
  double sub_origin[3], sub_dx;
  int sub_n[3];
  int plane;                // 1: plane strain in x-z (y out of plane, unit thickness)
};

template <class R>
struct Mat {                // material constants that may carry a tangent
  R K, mu, M, lam, kap, eta, b1, b2, rho_s, rho_w, a1, a2, n_vg;
};

// ------------------------------------------------------- 3x3 tensor helpers --
// Symmetric tensors use Voigt order (xx, yy, zz, yz, xz, xy); full tensors are
// row-major A[3*r + c].

template <class R>
void sym_to_full(const R* s, R* A) {
  A[0] = s[0]; A[1] = s[5]; A[2] = s[4];
  A[3] = s[5]; A[4] = s[1]; A[5] = s[3];
  A[6] = s[4]; A[7] = s[3]; A[8] = s[2];
}

template <class R>
R det3(const R* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}

// Inverse of a general 3x3 matrix by the adjugate divided by the determinant.
template <class R>
void inv3(const R* A, R det, R* B) {
  B[0] = (A[4] * A[8] - A[5] * A[7]) / det;
  B[1] = (A[2] * A[7] - A[1] * A[8]) / det;
  B[2] = (A[1] * A[5] - A[2] * A[4]) / det;
  B[3] = (A[5] * A[6] - A[3] * A[8]) / det;
  B[4] = (A[0] * A[8] - A[2] * A[6]) / det;
  B[5] = (A[2] * A[3] - A[0] * A[5]) / det;
  B[6] = (A[3] * A[7] - A[4] * A[6]) / det;
  B[7] = (A[1] * A[6] - A[0] * A[7]) / det;
  B[8] = (A[0] * A[4] - A[1] * A[3]) / det;
}

template <class R>
void matmul3(const R* A, const R* B, R* C) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      R s = 0.0;
      for (int m = 0; m < 3; ++m) s += A[3 * r + m] * B[3 * m + c];
      C[3 * r + c] = s;
    }
}

// Inverse of a shape tensor K (Voigt xx, yy, zz, yz, xz, xy) built from
// `count` members, or false when it is degenerate: fewer members than
// dimensions, or det K <= 1e-12 (tr K / d)^d.  In plane strain (x-z plane, y
// out of plane) only the x-z block is inverted; the y row and column of the
// inverse are zero, so no gradient or force state gains a y component.
template <class R>
bool shape_inverse(const Params& P, const R* K6, int64_t count, R* Kinv) {
  if (!P.plane) {
    R KF[9];
    sym_to_full(K6, KF);
    const R dK = det3(KF);
    const double trk = val(K6[0] + K6[1] + K6[2]) / 3.0;
    if (count < 3 || !(val(dK) > 1e-12 * trk * trk * trk)) return false;
    inv3(KF, dK, Kinv);
    return true;
  }
  const R a = K6[0], c = K6[2], e = K6[4];
  const R d2 = a * c - e * e;
  const double tr = val(a + c) / 2.0;
  if (count < 2 || !(val(d2) > 1e-12 * tr * tr)) return false;
  for (int k = 0; k < 9; ++k) Kinv[k] = R(0.0);
  Kinv[0] = c / d2;
  Kinv[2] = -e / d2;
  Kinv[6] = -e / d2;
  Kinv[8] = a / d2;
  return true;
}


// Canonical squared distance |b - a|^2: each difference and product rounded,
// summed as ((dx^2 + dy^2) + dz^2).  Families (Eq. 1) and sub-horizons
// (Eq. 22) are decided with this predicate against delta*delta.
inline double r2(const double* a, const double* b) {
  double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
  double xx = dx * dx, yy = dy * dy, zz = dz * dz;
  return (xx + yy) + zz;
}

// ----------------------------------------------------------- families --

struct Families {
  std::vector<int64_t> row;   // n+1
  std::vector<int32_t> col;   // bonds, each row ascending
  std::vector<int64_t> rev;   // slot of (j,i) for slot of (i,j)
};

// Family of every point in the current configuration (Eq. 1 with a constant
// horizon; Algorithm 1, neighbour search).  The point itself is excluded.
// Cell-list search: cells of edge >= delta, so all members of H_i lie in the
// 27 cells around i.
void build_families_cells(int64_t n, const double* x, double delta, Families& F) {
  const double d2 = delta * delta;
  F.row.assign(n + 1, 0);
  F.col.clear();
  if (n == 0) return;
  double lo[3] = {x[0], x[1], x[2]}, hi[3] = {x[0], x[1], x[2]};
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      lo[c] = std::min(lo[c], x[3 * i + c]);
      hi[c] = std::max(hi[c], x[3 * i + c]);
    }
  double cs = delta * (1.0 + 1e-9);
  int64_t dim[3];
  for (int c = 0; c < 3; ++c) dim[c] = (int64_t)std::floor((hi[c] - lo[c]) / cs) + 1;
  while ((double)dim[0] * dim[1] * dim[2] > 4.0 * n + 64) {   // keep the grid small
    cs *= 2.0;
    for (int c = 0; c < 3; ++c) dim[c] = (int64_t)std::floor((hi[c] - lo[c]) / cs) + 1;
  }
  auto cell_of = [&](int64_t i, int64_t* cc) {
    for (int c = 0; c < 3; ++c) {
      int64_t v = (int64_t)std::floor((x[3 * i + c] - lo[c]) / cs);
      cc[c] = std::min<int64_t>(std::max<int64_t>(v, 0), dim[c] - 1);
    }
  };
  const int64_t ncell = dim[0] * dim[1] * dim[2];
  std::vector<std::vector<int64_t>> cells(ncell);
  for (int64_t i = 0; i < n; ++i) {
    int64_t cc[3];
    cell_of(i, cc);
    cells[cc[0] + dim[0] * (cc[1] + dim[1] * cc[2])].push_back(i);
  }
  std::vector<std::vector<int32_t>> rows(n);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    int64_t cc[3];
    cell_of(i, cc);
    for (int64_t dz = -1; dz <= 1; ++dz)
      for (int64_t dy = -1; dy <= 1; ++dy)
        for (int64_t dx = -1; dx <= 1; ++dx) {
          int64_t a = cc[0] + dx, b = cc[1] + dy, c = cc[2] + dz;
          if (a < 0 || b < 0 || c < 0 || a >= dim[0] || b >= dim[1] || c >= dim[2]) continue;
          for (int64_t j : cells[a + dim[0] * (b + dim[1] * c)])
            if (j != i && r2(&x[3 * i], &x[3 * j]) <= d2) rows[i].push_back((int32_t)j);
        }
    std::sort(rows[i].begin(), rows[i].end());
  }
  for (int64_t i = 0; i < n; ++i) F.row[i + 1] = F.row[i] + (int64_t)rows[i].size();
  F.col.resize(F.row[n]);
  for (int64_t i = 0; i < n; ++i)
    std::copy(rows[i].begin(), rows[i].end(), F.col.begin() + F.row[i]);
}

// O(N^2) brute force of the same definition, for pinning the cell search.
void build_families_brute(int64_t n, const double* x, double delta, Families& F) {
  const double d2 = delta * delta;
  F.row.assign(n + 1, 0);
  F.col.clear();
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < n; ++j)
      if (j != i && r2(&x[3 * i], &x[3 * j]) <= d2) F.col.push_back((int32_t)j);
    F.row[i + 1] = (int64_t)F.col.size();
  }
}

// Reverse-bond index: rev[slot(i,j)] = slot(j,i), found by scanning row j.
void build_reverse(int64_t n, Families& F) {
  F.rev.assign(F.col.size(), -1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t s = F.row[i]; s < F.row[i + 1]; ++s) {
      const int64_t j = F.col[s];
      auto first = F.col.begin() + F.row[j], last = F.col.begin() + F.row[j + 1];
      auto it = std::lower_bound(first, last, (int32_t)i);
      if (it != last && *it == i) F.rev[s] = it - F.col.begin();
    }
}

// ---------------------------------------------------- constitutive model --

// Apparent pre-consolidation pressure, Eq. 45.
template <class R>
R apparent_pc(const Mat<R>& m, R pc) {
  return -exp(m.b1) * pow(-pc, m.b2);
}

// Yield function of modified Cam-clay, Eq. 40.
template <class R>
R yield_f(const Mat<R>& m, R p, R q, R pcbar) {
  return q * q / (m.M * m.M) + p * (p - pcbar);
}

// Residuals of the backward-Euler Perzyna update in the invariants, Eqs. 70-75,
// with unknowns x = (p, q, p_c).  c = dt/eta.  The hardening exponent carries
// the sign of Eq. 46 integrated over the step (compaction, d f/d p < 0 with
// compression negative, makes p_c more negative).
template <class R>
void rm_residual(const Mat<R>& m, R c, R ptr, R qtr, R pcn, const R* x, R* r) {
  R p = x[0], q = x[1], pc = x[2];
  R P = apparent_pc(m, pc);
  R f = yield_f(m, p, q, P);
  R dfdp = 2.0 * p - P;                 // d f / d p
  R dfdq = 2.0 * q / (m.M * m.M);       // d f / d q
  r[0] = p - ptr + m.K * c * f * dfdp;
  r[1] = q - qtr + 3.0 * m.mu * c * f * dfdq;
  r[2] = pc - pcn * exp(-c * f * dfdp / (m.lam - m.kap));
}

// Exact Jacobian dr/dx of rm_residual, differentiated by hand from it (the
// printed tangent entries, Eqs. 77-90, are partly garbled).
template <class R>
void rm_jacobian(const Mat<R>& m, R c, R pcn, const R* x, R* A) {
  R p = x[0], q = x[1], pc = x[2];
  R P = apparent_pc(m, pc);
  R dP = m.b2 * exp(m.b1) * pow(-pc, m.b2 - 1.0);   // d pcbar / d pc, Eq. 89
  R f = yield_f(m, p, q, P);
  R g = 2.0 * p - P;
  R h = 2.0 * q / (m.M * m.M);
  R fp = g, fq = h, fpc = -p * dP;                    // gradient of f
  R lk = m.lam - m.kap;
  // d(f*g)/dx and d(f*h)/dx
  R fg_p = fp * g + f * 2.0, fg_q = fq * g, fg_c = fpc * g + f * (-dP);
  R fh_p = fp * h, fh_q = fq * h + f * (2.0 / (m.M * m.M)), fh_c = fpc * h;
  A[0] = 1.0 + m.K * c * fg_p;
  A[1] = m.K * c * fg_q;
  A[2] = m.K * c * fg_c;
  A[3] = 3.0 * m.mu * c * fh_p;
  A[4] = 1.0 + 3.0 * m.mu * c * fh_q;
  A[5] = 3.0 * m.mu * c * fh_c;
  R E = exp(-c * f * g / lk);
  R k3 = pcn * E * c / lk;
  A[6] = k3 * fg_p;
  A[7] = k3 * fg_q;
  A[8] = 1.0 + k3 * fg_c;
}

// Solve A y = b (3x3) by Gaussian elimination with partial pivoting on values.
template <class R>
void solve3(const R* A0, const R* b0, R* y) {
  R A[9], b[3];
  for (int k = 0; k < 9; ++k) A[k] = A0[k];
  for (int k = 0; k < 3; ++k) b[k] = b0[k];
  int perm[3] = {0, 1, 2};
  for (int col = 0; col < 3; ++col) {
    int piv = col;
    for (int r = col + 1; r < 3; ++r)
      if (std::fabs(val(A[3 * perm[r] + col])) > std::fabs(val(A[3 * perm[piv] + col]))) piv = r;
    std::swap(perm[col], perm[piv]);
    for (int r = col + 1; r < 3; ++r) {
      R fct = A[3 * perm[r] + col] / A[3 * perm[col] + col];
      for (int c = col; c < 3; ++c) A[3 * perm[r] + c] -= fct * A[3 * perm[col] + c];
      b[perm[r]] -= fct * b[perm[col]];
    }
  }
  for (int r = 2; r >= 0; --r) {
    R s = b[perm[r]];
    for (int c = r + 1; c < 3; ++c) s -= A[3 * perm[r] + c] * y[c];
    y[r] = s / A[3 * perm[r] + r];
  }
}

// The same backward-Euler equations (Eqs. 70-75) written with the
// consistency parameter dg = c f >= 0 (c = dt/eta):
//   q   = q_tr / (1 + 6 mu dg / M^2),
//   p   = (p_tr + K dg P) / (1 + 2 K dg),       so 2p - P = (2 p_tr - P)/(1 + 2 K dg),
//   p_c = p_c,n exp(-dg (2 p_tr - P) / ((lam - kap)(1 + 2 K dg))),  P = P(p_c) (Eq. 45),
//   dg  = c f(p, q, P).
// For fixed dg the p_c equation is strictly increasing in p_c (slope >= 1);
// dg - c f changes sign on [0, inf).  Both are bracketed, so this solve
// cannot stall; it is used where Newton on (p, q, p_c) does.
struct Bracketed {
  double K, mu, M, lk, b1, b2, c, ptr, qtr, pcn;
  double P(double pc) const { return -std::exp(b1) * std::pow(-pc, b2); }
  double dP(double pc) const { return b2 * std::exp(b1) * std::pow(-pc, b2 - 1.0); }
  // p_c for a given dg: safeguarded Newton inside a bracket [lo, hi) with hi = 0.
  double pc_of(double dg) const {
    const double A = dg / (lk * (1.0 + 2.0 * K * dg));
    auto h = [&](double x) { return x - pcn * std::exp(-A * (2.0 * ptr - P(x))); };
    double lo = pcn, hi = 0.0;
    for (int k = 0; k < 4000 && h(lo) > 0.0; ++k) { hi = lo; lo *= 2.0; }
    double x = pcn;
    if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
      const double hx = h(x);
      if (hx == 0.0) return x;
      if (hx > 0.0) hi = x; else lo = x;
      const double E = std::exp(-A * (2.0 * ptr - P(x)));
      const double d = 1.0 - pcn * E * A * dP(x);
      double xn = x - hx / d;
      if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
      if (std::fabs(xn - x) <= 1e-16 * std::fabs(x) || hi - lo <= 1e-16 * std::fabs(lo)) return xn;
      x = xn;
    }
    return x;
  }
  void state(double dg, double* x) const {
    const double pc = pc_of(dg);
    const double Pb = P(pc);
    x[0] = (ptr + K * dg * Pb) / (1.0 + 2.0 * K * dg);
    x[1] = qtr / (1.0 + 6.0 * mu * dg / (M * M));
    x[2] = pc;
  }
  double phi(double dg) const {
    double x[3];
    state(dg, x);
    const double f = x[1] * x[1] / (M * M) + x[0] * (x[0] - P(x[2]));
    return dg - c * f;
  }
  // Illinois false position on phi over a doubling bracket.
  void solve(double ftr, double* x) const {
    double lo = 0.0, flo = -c * ftr;
    double hi = c * ftr, fhi = phi(hi);
    for (int k = 0; k < 2000 && fhi < 0.0; ++k) { lo = hi; flo = fhi; hi *= 2.0; fhi = phi(hi); }
    int side = 0;
    double dg = hi;
    for (int it = 0; it < 300; ++it) {
      dg = (lo * fhi - hi * flo) / (fhi - flo);
      if (!(dg > lo && dg < hi)) dg = 0.5 * (lo + hi);
      const double fm = phi(dg);
      if (fm == 0.0 || hi - lo <= 2e-16 * hi) break;
      if (fm > 0.0) {
        hi = dg; fhi = fm;
        if (side == 1) flo *= 0.5;
        side = 1;
      } else {
        lo = dg; flo = fm;
        if (side == -1) fhi *= 0.5;
        side = -1;
      }
    }
    state(dg, x);
  }
};

// Local constitutive update (Section 3.2.1): elastic trial stress from the
// strain increment (linear elasticity in invariants, Eq. 41, applied to the
// increment), then, if the trial state violates the yield condition (Eq. 40),
// the backward-Euler Perzyna return (Eqs. 43, 70-76) solved by Newton's method,
// and a radial reconstruction of the deviator.  Returns the number of Newton
// iterations (0 = elastic), or -1 if Newton did not converge.
template <class R>
int return_map(const Mat<R>& m, const Params& P, R dt, const R* sig_n, R pc_n, const R* deps,
               R* sig_out, R* pc_out) {
  R tr = deps[0] + deps[1] + deps[2];
  R st[6];
  for (int k = 0; k < 6; ++k) {
    R dev = deps[k] - (k < 3 ? tr / 3.0 : R(0.0));
    st[k] = sig_n[k] + (k < 3 ? m.K * tr : R(0.0)) + 2.0 * m.mu * dev;
  }
  R ptr = (st[0] + st[1] + st[2]) / 3.0;
  R s[6];
  for (int k = 0; k < 6; ++k) s[k] = st[k] - (k < 3 ? ptr : R(0.0));
  R ss = s[0] * s[0] + s[1] * s[1] + s[2] * s[2] + 2.0 * (s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
  R qtr = sqrt(1.5 * ss);
  R ftr = yield_f(m, ptr, qtr, apparent_pc(m, pc_n));
  if (!(val(ftr) > 0.0)) {
    for (int k = 0; k < 6; ++k) sig_out[k] = st[k];
    *pc_out = pc_n;
    return 0;
  }
  R c = dt / m.eta;
  R x[3] = {ptr, qtr, pc_n};
  double sref = std::max(std::fabs(val(ptr)), std::max(val(qtr), std::fabs(val(apparent_pc(m, pc_n)))));
  double pref = std::fabs(val(pc_n));
  int it = 0;
  bool stalled = false;
  for (;;) {
    R r[3];
    rm_residual(m, c, ptr, qtr, pc_n, x, r);
    bool ok = std::fabs(val(r[0])) <= P.newton_tol * sref && std::fabs(val(r[1])) <= P.newton_tol * sref &&
              std::fabs(val(r[2])) <= P.newton_tol * pref;
    if (ok) break;
    if (it >= P.newton_maxit || stalled) {
      // Newton stalled: solve the same equations by bracketing (see Bracketed).
      Bracketed B{val(m.K), val(m.mu), val(m.M), val(m.lam) - val(m.kap), val(m.b1), val(m.b2),
                  val(c), val(ptr), val(qtr), val(pc_n)};
      double xb[3];
      B.solve(val(ftr), xb);
      for (int k = 0; k < 3; ++k) x[k] = xb[k];
      rm_residual(m, c, ptr, qtr, pc_n, x, r);
      if (!(std::fabs(val(r[0])) <= 1e3 * P.newton_tol * sref && std::fabs(val(r[1])) <= 1e3 * P.newton_tol * sref &&
            std::fabs(val(r[2])) <= 1e3 * P.newton_tol * pref))
        return -1;
      it = P.newton_maxit + 1;
      break;
    }
    R A[9], dx[3], nr[3] = {-r[0], -r[1], -r[2]};
    rm_jacobian(m, c, pc_n, x, A);
    solve3(A, nr, dx);
    // The residuals drop the Macaulay bracket of Eq. 43, so they also have
    // roots with f <= 0 that the model excludes.  Keep every iterate in the
    // admissible set {f > 0, q >= 0, p_c < 0}, which holds the solution and
    // the trial state, by halving a step that would leave it.
    R step = 1.0;
    for (int h = 0; h < 60; ++h) {
      R xt[3] = {x[0] + step * dx[0], x[1] + step * dx[1], x[2] + step * dx[2]};
      if (val(xt[2]) < 0.0 && val(xt[1]) >= 0.0 &&
          val(yield_f(m, xt[0], xt[1], apparent_pc(m, xt[2]))) > 0.0)
        break;
      step = 0.5 * step;
    }
    for (int k = 0; k < 3; ++k) x[k] += step * dx[k];
    ++it;
    stalled = val(step) < 1e-6;
  }
  if constexpr (std::is_same<R, Dual>::value) {
    // One more Newton step at the converged point: the value moves by
    // rounding only, and the tangent becomes the implicit-function derivative
    // -A^{-1} dr/dtheta exactly.
    R r[3], A[9], dx[3];
    rm_residual(m, c, ptr, qtr, pc_n, x, r);
    R nr[3] = {-r[0], -r[1], -r[2]};
    rm_jacobian(m, c, pc_n, x, A);
    solve3(A, nr, dx);
    for (int k = 0; k < 3; ++k) x[k] += dx[k];
  }
  // Radial reconstruction: sigma = p 1 + (q / q_tr) s_tr.
  R ratio = val(qtr) > 0.0 ? x[1] / qtr : R(0.0);
  for (int k = 0; k < 6; ++k) sig_out[k] = (k < 3 ? x[0] : R(0.0)) + ratio * s[k];
  *pc_out = x[2];
  return it > 0 ? it : 1;
}

// Soil-water retention curve, Eq. 15, with the exponent read as -(n-1)/n
// (the printed sign gives S_r > 1), suction s = -p_w in kPa, and
// e = phi/(1-phi) the current void ratio.
template <class R>
R swrc(const Mat<R>& m, R J, R phi, R s_pa) {
  if (!(val(s_pa) > 0.0)) return R(1.0);
  R e = phi / (1.0 - phi);
  R arg = m.a1 * pow(e, m.a2) * J * (s_pa * 1e-3);
  return pow(1.0 + pow(arg, m.n_vg), -(m.n_vg - 1.0) / m.n_vg);
}

// -------------------------------------------------- one pass of Alg. 1 --

template <class R>
struct PointState {          // one array per field, caller order, AoS vectors
  int64_t n = 0;
  std::vector<double> x0;     // n*3, never differentiated
  std::vector<R> u, uc, v, a; // n*3
  std::vector<R> vol, phi, J, Sr, mass, s, pc;  // n
  std::vector<R> sig;         // n*6
  std::vector<uint8_t> fixed;
};

struct Stats {
  int64_t n_bonds = 0, n_degenerate = 0, n_plastic = 0, max_newton = 0, n_noconv = 0;
  int64_t n_tests = 0, n_triples = 0;
};

// Per-bond and per-point outputs of Algorithm 1 (transient; CSR order).
template <class R>
struct BondOut {
  std::vector<R> K;      // 6 per bond, sub-horizon shape tensor (Eq. 23)
  std::vector<R> L;      // 9 per bond, sub-horizon velocity gradient (Eq. 57)
  std::vector<R> sig;    // 6 per bond, bond effective stress after the update
  std::vector<R> pc;     // 1 per bond
  std::vector<R> T;      // 3 per bond, total force state (Eq. 32 / 51 + 53)
  std::vector<R> varpi;  // 1 per bond, weighting factor (Eq. 55)
  std::vector<int32_t> nsub;   // |S_ij|
  std::vector<int8_t> active;
  std::vector<R> Jd, Sr_new, vol_new, phi_new, J_new, mass_new;  // per point
  std::vector<R> sig_new, pc_new;  // per point history after averaging
  std::vector<R> f;      // n*3 internal nodal force (Eqs. 49-50)
};

// Contact with a rigid substrate (Eqs. 91-93).  The substrate is a lattice of
// fixed sites origin + dx (a, b, -c), each of volume dx^3.  For point i and a
// site s with Y = x_s - x_i closer than delta_c:
//   T_c = -C_s (delta_c - |Y|) Y/|Y|                      (Eq. 91)
//   T_f = -mu_f sign(d|Y|/dt) T_c, d|Y|/dt = -Y.v_i/|Y|   (Eq. 92 as printed;
//                                                           the site is at rest)
// The reverse pair has Y' = -Y, so T_c' = -T_c and T_f' = -T_f, and the
// contact integrand of Eq. 93 is 2 (T_c + T_f); with the volumes as
// quadrature weights the nodal force gains V_i sum_s 2 (T_c + T_f) V_s.
// Every site is visited (no search), so the neighbourhood is exactly the set
// of sites with |Y|^2 < delta_c^2, the squared length rounded as
// ((Y0^2 + Y1^2) + Y2^2).
template <class R>
void contact_forces(const Params& P, int64_t n, const R* x, const R* v, const std::vector<R>& vol,
                    std::vector<R>& f) {
  if (!(P.cs > 0.0)) return;
  const double dc2 = P.delta_c * P.delta_c;
  const double Vs = P.plane ? P.sub_dx * P.sub_dx : P.sub_dx * P.sub_dx * P.sub_dx;   // unit thickness in plane strain
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    R acc[3] = {R(0.0), R(0.0), R(0.0)};
    for (int c = 0; c < P.sub_n[2]; ++c)
      for (int b = 0; b < P.sub_n[1]; ++b)
        for (int a = 0; a < P.sub_n[0]; ++a) {
          const double xs[3] = {P.sub_origin[0] + (double)a * P.sub_dx, P.sub_origin[1] + (double)b * P.sub_dx,
                                P.sub_origin[2] - (double)c * P.sub_dx};
          R Y[3];
          for (int q = 0; q < 3; ++q) Y[q] = xs[q] - x[3 * i + q];
          const double yv[3] = {val(Y[0]), val(Y[1]), val(Y[2])};
          const double r2 = (yv[0] * yv[0] + yv[1] * yv[1]) + yv[2] * yv[2];
          if (!(r2 < dc2) || r2 == 0.0) continue;
          const R r = sqrt(Y[0] * Y[0] + Y[1] * Y[1] + Y[2] * Y[2]);
          const R tc = -P.cs * (P.delta_c - r) / r;                 // T_c = tc Y
          const double rate = -(yv[0] * val(v[3 * i]) + yv[1] * val(v[3 * i + 1]) + yv[2] * val(v[3 * i + 2]));
          const double sg = rate > 0.0 ? 1.0 : (rate < 0.0 ? -1.0 : 0.0);
          const R w = 2.0 * Vs * tc * (1.0 - P.mu_f * sg);          // 2 (T_c + T_f) V_s = w Y
          for (int q = 0; q < 3; ++q) acc[q] += w * Y[q];
        }
    for (int q = 0; q < 3; ++q) f[3 * i + q] += vol[i] * acc[q];
  }
}

// Algorithm 1 at positions x (current configuration) with relative velocities
// taken from vh, strain increment dt_inc * D_ij.  dt_inc = 0 gives the bond
// stress equal to the point stress (used for the initial acceleration).
template <class R>
void algorithm1(const Params& P, const Mat<R>& m, int64_t n, const double* xval, const R* x,
                const R* vh, const PointState<R>& S, const Families& F, R dt_inc, BondOut<R>& O,
                Stats& st, const std::vector<R>* bond_in = nullptr) {
  const double d2 = P.delta * P.delta;
  const int64_t nb = F.row[n];
  O.K.assign(6 * nb, R(0.0));
  O.L.assign(9 * nb, R(0.0));
  O.sig.assign(6 * nb, R(0.0));
  O.pc.assign(nb, R(0.0));
  O.T.assign(3 * nb, R(0.0));
  O.varpi.assign(nb, R(0.0));
  O.nsub.assign(nb, 0);
  O.active.assign(nb, 0);
  O.Jd.assign(n, R(1.0));
  O.Sr_new.assign(n, R(1.0));
  O.vol_new.assign(n, R(0.0));
  O.phi_new.assign(n, R(0.0));
  O.J_new.assign(n, R(0.0));
  O.mass_new.assign(n, R(0.0));
  O.sig_new.assign(6 * n, R(0.0));
  O.pc_new.assign(n, R(0.0));
  O.f.assign(3 * n, R(0.0));
  int64_t n_deg = 0, n_pl = 0, maxit = 0, n_nc = 0, n_tests = 0, n_trip = 0;

  // Loop 1 of Algorithm 1, full-horizon part: shape tensor (Eq. 5), velocity
  // gradient (Eq. 8) and the volume change of the step (Eq. 17 in updated
  // Lagrangian form: the increment F_D satisfies F_D^{-1} = I - dt L_i), then
  // porosity (Eq. 16), degree of saturation (Eq. 15) and mass (Eq. 48).
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : n_deg, n_pl, n_nc) reduction(max : maxit)
  for (int64_t i = 0; i < n; ++i) {
    R Ki[6] = {0, 0, 0, 0, 0, 0}, Ni[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t nfam = F.row[i + 1] - F.row[i];
    for (int64_t s = F.row[i]; s < F.row[i + 1]; ++s) {
      int64_t j = F.col[s];
      R z[3], y[3];
      for (int c = 0; c < 3; ++c) {
        z[c] = x[3 * j + c] - x[3 * i + c];
        y[c] = vh[3 * j + c] - vh[3 * i + c];
      }
      R V = S.vol[j];
      Ki[0] += V * z[0] * z[0]; Ki[1] += V * z[1] * z[1]; Ki[2] += V * z[2] * z[2];
      Ki[3] += V * z[1] * z[2]; Ki[4] += V * z[0] * z[2]; Ki[5] += V * z[0] * z[1];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Ni[3 * a + b] += V * y[a] * z[b];
    }
    R Jd = 1.0;
    R Kinv[9], Li[9];
    const bool full_ok = shape_inverse(P, Ki, nfam, Kinv);
    if (full_ok) {
      R B[9];
      matmul3(Ni, Kinv, Li);
      for (int k = 0; k < 9; ++k) B[k] = (k % 4 == 0 ? R(1.0) : R(0.0)) - dt_inc * Li[k];
      Jd = 1.0 / det3(B);
    }
    O.Jd[i] = Jd;
    O.J_new[i] = S.J[i] * Jd;
    O.vol_new[i] = S.vol[i] * Jd;
    O.phi_new[i] = 1.0 - (1.0 - S.phi[i]) / Jd;
    O.Sr_new[i] = swrc(m, O.J_new[i], O.phi_new[i], S.s[i]);
    O.mass_new[i] = (m.rho_s * (1.0 - O.phi_new[i]) + m.rho_w * O.Sr_new[i] * O.phi_new[i]) * O.vol_new[i];
    if (P.force_mode == 2) {
      // Standard correspondence (Eqs. 12-14): one stress per point, updated
      // from the full-horizon gradient L_i, and force states
      // T_ik = (sigma_i + S_r s 1) K_i^{-1} zeta_ik on every bond of i.
      const R* sig_i = &S.sig[6 * i];
      R sb[6], pcb;
      if (full_ok && val(dt_inc) != 0.0) {
        R deps[6] = {dt_inc * Li[0], dt_inc * Li[4], dt_inc * Li[8], dt_inc * 0.5 * (Li[5] + Li[7]),
                     dt_inc * 0.5 * (Li[2] + Li[6]), dt_inc * 0.5 * (Li[1] + Li[3])};
        int it = return_map(m, P, dt_inc, sig_i, S.pc[i], deps, sb, &pcb);
        if (it < 0) { ++n_nc; it = P.newton_maxit; }
        if (it > 0) ++n_pl;
        if (it > maxit) maxit = it;
      } else {
        for (int k = 0; k < 6; ++k) sb[k] = sig_i[k];
        pcb = S.pc[i];
      }
      for (int k = 0; k < 6; ++k) O.sig_new[6 * i + k] = sb[k];
      O.pc_new[i] = pcb;
      if (full_ok) {
        R sF[9], SK[9];
        sym_to_full(sb, sF);
        R ps = O.Sr_new[i] * S.s[i];
        for (int k = 0; k < 3; ++k) sF[4 * k] += ps;
        matmul3(sF, Kinv, SK);
        for (int64_t t = F.row[i]; t < F.row[i + 1]; ++t) {
          const int64_t k = F.col[t];
          R z[3];
          for (int c = 0; c < 3; ++c) z[c] = x[3 * k + c] - x[3 * i + c];
          for (int r = 0; r < 3; ++r)
            O.T[3 * t + r] = SK[3 * r] * z[0] + SK[3 * r + 1] * z[1] + SK[3 * r + 2] * z[2];
        }
      } else {
        n_deg += nfam;
      }
    }
  }

  // Loops 1-3 of Algorithm 1, bond part.  For each bond (i,j): the
  // sub-horizon S_ij = {k in H_i : |x_k - x_j| <= delta} (Eq. 22), its shape
  // tensor (Eq. 23), velocity gradient (Eqs. 25, 57), weighting factor
  // (Eq. 55), rate of deformation (Eq. 26) and strain increment (Eq. 59); the
  // bond stress from the local model; and the total force state
  // T = varpi (sigma - S_r p_w 1) K^{-1} zeta with p_w = -s (Eqs. 32, 51, 53).
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : n_deg, n_pl, n_nc, n_tests, n_trip) \
    reduction(max : maxit)
  for (int64_t i = 0; i < (P.force_mode == 2 ? 0 : n); ++i) {
    const int64_t b0 = F.row[i], b1 = F.row[i + 1];
    R Vh = 0.0;
    for (int64_t s = b0; s < b1; ++s) Vh += S.vol[F.col[s]];
    R hs[6] = {0, 0, 0, 0, 0, 0}, hpc = 0.0, hw = 0.0;
    const R* sig_i = &S.sig[6 * i];
    std::vector<R> SKb(9 * (b1 - b0), R(0.0));   // (V_j/V_H) (sigma_ij + S_r s 1) K_ij^{-1}
    for (int64_t s = b0; s < b1; ++s) {
      const int64_t j = F.col[s];
      R Kij[6] = {0, 0, 0, 0, 0, 0}, Nij[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, Vs = 0.0;
      int nsub = 0;
      for (int64_t t = b0; t < b1; ++t) {
        const int64_t k = F.col[t];
        ++n_tests;
        if (!(r2(&xval[3 * j], &xval[3 * k]) <= d2)) continue;
        ++nsub;
        R z[3], y[3];
        for (int c = 0; c < 3; ++c) {
          z[c] = x[3 * k + c] - x[3 * i + c];
          y[c] = vh[3 * k + c] - vh[3 * i + c];
        }
        R V = S.vol[k];
        Kij[0] += V * z[0] * z[0]; Kij[1] += V * z[1] * z[1]; Kij[2] += V * z[2] * z[2];
        Kij[3] += V * z[1] * z[2]; Kij[4] += V * z[0] * z[2]; Kij[5] += V * z[0] * z[1];
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) Nij[3 * a + b] += V * y[a] * z[b];
        Vs += V;
      }
      n_trip += nsub;
      O.nsub[s] = nsub;
      for (int k = 0; k < 6; ++k) O.K[6 * s + k] = Kij[k];
      R Kinv[9], L[9];
      if (!shape_inverse(P, Kij, nsub, Kinv)) {                 // degenerate bond: inactive
        ++n_deg;
        continue;
      }
      O.active[s] = 1;
      matmul3(Nij, Kinv, L);
      for (int k = 0; k < 9; ++k) O.L[9 * s + k] = L[k];
      R varpi = Vs / Vh;
      O.varpi[s] = varpi;
      // D = sym(L) (Eq. 26), strain increment dt D (Eq. 59), Voigt order.
      R deps[6] = {dt_inc * L[0], dt_inc * L[4], dt_inc * L[8], dt_inc * 0.5 * (L[5] + L[7]),
                   dt_inc * 0.5 * (L[2] + L[6]), dt_inc * 0.5 * (L[1] + L[3])};
      R sb[6], pcb;
      // state the bond starts from: the point history, or the bond's own
      // history when it is carried on the bonds
      R sig_b[6], pc_b;
      for (int k = 0; k < 6; ++k) sig_b[k] = bond_in ? (*bond_in)[8 * s + k] : sig_i[k];
      pc_b = bond_in ? (*bond_in)[8 * s + 6] : S.pc[i];
      if (val(dt_inc) == 0.0) {
        for (int k = 0; k < 6; ++k) sb[k] = sig_b[k];
        pcb = pc_b;
      } else {
        int it = return_map(m, P, dt_inc, sig_b, pc_b, deps, sb, &pcb);
        if (it < 0) { ++n_nc; it = P.newton_maxit; }
        if (it > 0) ++n_pl;
        if (it > maxit) maxit = it;
      }
      for (int k = 0; k < 6; ++k) O.sig[6 * s + k] = sb[k];
      O.pc[s] = pcb;
      // Total stress of the bond, sigma_ij + S_r s 1 (Eq. 32 with p_w = -s),
      // times K_ij^{-1}.
      R sF[9], SK[9];
      sym_to_full(sb, sF);
      R ps = O.Sr_new[i] * S.s[i];
      for (int k = 0; k < 3; ++k) sF[4 * k] += ps;
      matmul3(sF, Kinv, SK);
      if (P.force_mode == 1) {
        // Eq. 51 as printed: T_ij = varpi (sigma + S_r s 1) K^{-1} zeta_ij.
        R z[3];
        for (int c = 0; c < 3; ++c) z[c] = x[3 * j + c] - x[3 * i + c];
        for (int r = 0; r < 3; ++r)
          O.T[3 * s + r] = varpi * (SK[3 * r + 0] * z[0] + SK[3 * r + 1] * z[1] + SK[3 * r + 2] * z[2]);
      } else {
        for (int k = 0; k < 9; ++k) SKb[9 * (s - b0) + k] = SK[k] * (S.vol[j] / Vh);
      }
      // Point history: volume-weighted mean of the bond states.
      R Vj = S.vol[j];
      for (int k = 0; k < 6; ++k) hs[k] += Vj * sb[k];
      hpc += Vj * pcb;
      hw += Vj;
    }
    if (P.force_mode == 0) {
      // Force state of bond (i,k): the sub-horizon force state of every
      // sub-horizon S_ij that holds k, evaluated on bond ik (Eqs. 27, 31),
      // summed over those sub-horizons as in the double integral of Eq. 35.
      // Its power, sum_k V_k T_ik . Ydot_ik, is the volume-weighted mean of
      // sigma_ij : L_ij over the bonds of i, the same mean that updates the
      // point history.
      for (int64_t t = b0; t < b1; ++t) {
        const int64_t k = F.col[t];
        R acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t s = b0; s < b1; ++s) {
          const int64_t j = F.col[s];
          if (!(r2(&xval[3 * j], &xval[3 * k]) <= d2)) continue;
          for (int q = 0; q < 9; ++q) acc[q] += SKb[9 * (s - b0) + q];
        }
        R z[3];
        for (int c = 0; c < 3; ++c) z[c] = x[3 * k + c] - x[3 * i + c];
        for (int r = 0; r < 3; ++r) O.T[3 * t + r] = acc[3 * r] * z[0] + acc[3 * r + 1] * z[1] + acc[3 * r + 2] * z[2];
      }
    }
    if (val(hw) > 0.0) {
      for (int k = 0; k < 6; ++k) O.sig_new[6 * i + k] = hs[k] / hw;
      O.pc_new[i] = hpc / hw;
    } else {
      for (int k = 0; k < 6; ++k) O.sig_new[6 * i + k] = sig_i[k];
      O.pc_new[i] = S.pc[i];
    }
  }

  // Loop 4 of Algorithm 1: nodal internal force, Eqs. 49-50 combined, with the
  // sign of Eq. 33: f_i = sum_j (T_ij - T_ji) V_i V_j.
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    R fi[3] = {0, 0, 0};
    for (int64_t s = F.row[i]; s < F.row[i + 1]; ++s) {
      int64_t j = F.col[s], t = F.rev[s];
      R w = S.vol[i] * S.vol[j];
      for (int c = 0; c < 3; ++c) fi[c] += (O.T[3 * s + c] - O.T[3 * t + c]) * w;
    }
    for (int c = 0; c < 3; ++c) O.f[3 * i + c] = fi[c];
  }
  contact_forces(P, n, x, vh, S.vol, O.f);
  st.n_bonds += nb;
  st.n_degenerate += n_deg;
  st.n_plastic += n_pl;
  st.n_noconv += n_nc;
  st.n_tests += n_tests;
  st.n_triples += n_trip;
  st.max_newton = std::max<int64_t>(st.max_newton, maxit);
}

template <class R>
std::vector<R> positions(const PointState<R>& S) {
  std::vector<R> x(3 * S.n);
  for (int64_t k = 0; k < 3 * S.n; ++k) x[k] = S.x0[k] + S.u[k];
  return x;
}

template <class R>
std::vector<double> values(const std::vector<R>& a) {
  std::vector<double> v(a.size());
  for (size_t k = 0; k < a.size(); ++k) v[k] = val(a[k]);
  return v;
}

// History carried on the bonds instead of the points (the alternative to the
// point history; the paper stores internal variables on material points but
// does not say how bond stresses relate to them across steps).  Every bond
// keeps its own (sigma_ij, p_c,ij) from one step to the next while it stays in
// the family; a bond that enters a family starts from its point's history
// (the volume-weighted mean of the point's bond states, as before).
template <class R>
struct BondHistory {
  std::vector<int64_t> row;   // families the states belong to (empty: none yet)
  std::vector<int32_t> col;
  std::vector<R> st;          // 8 per bond: sigma (6), p_c, unused
};

// Bond states in the order of the new families F: a bond found in the
// previous families of its point keeps its state; a new bond takes the point's.
template <class R>
void carry_bond_history(const BondHistory<R>& H, const Families& F, const std::vector<R>& sig,
                        const std::vector<R>& pc, std::vector<R>& in) {
  const int64_t n = (int64_t)F.row.size() - 1;
  in.assign(8 * F.row[n], R(0.0));
  const bool have = (int64_t)H.row.size() == n + 1;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t s = F.row[i]; s < F.row[i + 1]; ++s) {
      int64_t found = -1;
      if (have)
        for (int64_t t = H.row[i]; t < H.row[i + 1]; ++t)
          if (H.col[t] == F.col[s]) { found = t; break; }
      for (int k = 0; k < 6; ++k) in[8 * s + k] = found >= 0 ? H.st[8 * found + k] : sig[6 * i + k];
      in[8 * s + 6] = found >= 0 ? H.st[8 * found + 6] : pc[i];
    }
}

// Updated bond states after Algorithm 1; a degenerate (inactive) bond keeps
// the state it started from.
template <class R>
void store_bond_history(BondHistory<R>& H, const Families& F, const BondOut<R>& O, const std::vector<R>& in) {
  const int64_t nb = F.row.back();
  H.row = F.row;
  H.col = F.col;
  H.st.assign(8 * nb, R(0.0));
  for (int64_t s = 0; s < nb; ++s) {
    for (int k = 0; k < 6; ++k) H.st[8 * s + k] = O.active[s] ? O.sig[6 * s + k] : in[8 * s + k];
    H.st[8 * s + 6] = O.active[s] ? O.pc[s] : in[8 * s + 6];
  }
}

// Algorithm 2, one step n -> n+1, central differences (beta1 = 1/2,
// beta2 = 0; Eqs. 60-64), with energies of Eqs. 66-68 accumulated in E.
template <class R>
int newmark_step(const Params& P, const Mat<R>& m, PointState<R>& S, R* E, Stats& st,
                 Families* Fout = nullptr, BondHistory<R>* H = nullptr) {
  const int64_t n = S.n;
  const R dt = P.dt;
  const R hdt = 0.5 * P.dt;
  std::vector<R> vh(3 * n);
  R eint = 0.0, eext = 0.0;
  // Velocity predictor (Eq. 60 with the step size restored), boundary
  // conditions, displacement (Eqs. 61/64 with beta2 = 0: u += dt v_half),
  // summed with Kahan compensation.
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      // fixed points (code 1) stand still, driven points (code 2) keep their velocity
      R vhalf = S.fixed[i] == 2 ? S.v[3 * i + c] : S.fixed[i] ? R(0.0) : R(S.v[3 * i + c] + hdt * S.a[3 * i + c]);
      vh[3 * i + c] = vhalf;
      R y = dt * vhalf - S.uc[3 * i + c];
      R t = S.u[3 * i + c] + y;
      S.uc[3 * i + c] = (t - S.u[3 * i + c]) - y;
      S.u[3 * i + c] = t;
      // energy terms with the old force f^n = M^n (a^n - g) and old mass
      if (!S.fixed[i]) {
        R fn = S.mass[i] * (S.a[3 * i + c] - P.g[c]);
        eint -= hdt * vhalf * fn;
        eext += hdt * vhalf * S.mass[i] * P.g[c];
      }
    }
  std::vector<R> x = positions(S);
  std::vector<double> xv = values(x);
  Families F;
  build_families_cells(n, xv.data(), P.delta, F);
  build_reverse(n, F);
  BondOut<R> O;
  std::vector<R> bond_in;
  if (H) carry_bond_history(*H, F, S.sig, S.pc, bond_in);
  algorithm1(P, m, n, xv.data(), x.data(), vh.data(), S, F, dt, O, st, H ? &bond_in : nullptr);
  if (H) store_bond_history(*H, F, O, bond_in);
  // Acceleration (Eq. 62 with the sign of Eq. 33) and velocity corrector (Eq. 63).
  R ekin = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < 3; ++c) {
      R a = S.fixed[i] ? R(0.0) : R(O.f[3 * i + c] / O.mass_new[i] + P.g[c]);
      S.a[3 * i + c] = a;
      S.v[3 * i + c] = vh[3 * i + c] + hdt * a;
      if (!S.fixed[i]) {
        eint -= hdt * vh[3 * i + c] * O.f[3 * i + c];
        eext += hdt * vh[3 * i + c] * O.mass_new[i] * P.g[c];
      }
      ekin += 0.5 * O.mass_new[i] * S.v[3 * i + c] * S.v[3 * i + c];
    }
    S.J[i] = O.J_new[i];
    S.vol[i] = O.vol_new[i];
    S.phi[i] = O.phi_new[i];
    S.Sr[i] = O.Sr_new[i];
    S.mass[i] = O.mass_new[i];
    for (int k = 0; k < 6; ++k) S.sig[6 * i + k] = O.sig_new[6 * i + k];
    S.pc[i] = O.pc_new[i];
  }
  E[0] += eint;
  E[1] += eext;
  E[2] = ekin;
  if (Fout) *Fout = F;
  for (int64_t k = 0; k < 3 * n; ++k)
    if (!std::isfinite(val(S.v[k]))) return -5;
  return st.n_noconv ? -4 : 0;
}

}  // namespace

// ============================================================ C interface ==

typedef struct {
  double delta;
  double K, mu, M, lam, kap, eta, b1, b2;
  double rho_s, rho_w, a1, a2, n_vg;
  double g[3];
  double dt;
  double newton_tol;
  int32_t newton_maxit;
  int32_t force_mode;
  double cs, mu_f, delta_c;        // contact: stiffness C_s, friction mu_f, cut-off delta_c
  double sub_origin[3], sub_dx;    // substrate sites origin + sub_dx (a, b, -c)
  int32_t sub_n[3];                // a < sub_n[0], b < sub_n[1], c < sub_n[2]
  int32_t plane;                   // 1: plane strain in the x-z plane
} OracleParams;

typedef struct {             // host arrays, caller order
  int64_t n;
  double *x0, *u, *uc, *v, *a;            // n*3
  double *vol, *phi, *J, *Sr, *mass, *s;  // n
  double *sig;                            // n*6 Voigt (xx,yy,zz,yz,xz,xy)
  double *pc;                             // n
  uint8_t *fixed;                         // n
} OracleState;

typedef struct {
  int64_t n_bonds, n_degenerate, n_plastic, max_newton, n_noconv, n_tests, n_triples;
} OracleStats;

static Params to_params(const OracleParams* p) {
  Params P;
  P.delta = p->delta;
  P.K = p->K; P.mu = p->mu; P.M = p->M; P.lam = p->lam; P.kap = p->kap; P.eta = p->eta;
  P.b1 = p->b1; P.b2 = p->b2; P.rho_s = p->rho_s; P.rho_w = p->rho_w;
  P.a1 = p->a1; P.a2 = p->a2; P.n_vg = p->n_vg;
  for (int c = 0; c < 3; ++c) P.g[c] = p->g[c];
  P.dt = p->dt;
  P.newton_tol = p->newton_tol;
  P.newton_maxit = p->newton_maxit;
  P.force_mode = p->force_mode;
  P.cs = p->cs;
  P.mu_f = p->mu_f;
  P.delta_c = p->delta_c;
  for (int c = 0; c < 3; ++c) {
    P.sub_origin[c] = p->sub_origin[c];
    P.sub_n[c] = p->sub_n[c];
  }
  P.sub_dx = p->sub_dx;
  P.plane = p->plane;
  return P;
}

template <class R>
static Mat<R> to_mat(const Params& P) {
  Mat<R> m;
  m.K = P.K; m.mu = P.mu; m.M = P.M; m.lam = P.lam; m.kap = P.kap; m.eta = P.eta;
  m.b1 = P.b1; m.b2 = P.b2; m.rho_s = P.rho_s; m.rho_w = P.rho_w;
  m.a1 = P.a1; m.a2 = P.a2; m.n_vg = P.n_vg;
  return m;
}

static void load_state(const OracleState* s, PointState<double>& S) {
  const int64_t n = s->n;
  S.n = n;
  S.x0.assign(s->x0, s->x0 + 3 * n);
  S.u.assign(s->u, s->u + 3 * n);
  S.uc.assign(s->uc, s->uc + 3 * n);
  S.v.assign(s->v, s->v + 3 * n);
  S.a.assign(s->a, s->a + 3 * n);
  S.vol.assign(s->vol, s->vol + n);
  S.phi.assign(s->phi, s->phi + n);
  S.J.assign(s->J, s->J + n);
  S.Sr.assign(s->Sr, s->Sr + n);
  S.mass.assign(s->mass, s->mass + n);
  S.s.assign(s->s, s->s + n);
  S.sig.assign(s->sig, s->sig + 6 * n);
  S.pc.assign(s->pc, s->pc + n);
  S.fixed.assign(s->fixed, s->fixed + n);
}

static void store_state(const PointState<double>& S, OracleState* s) {
  const int64_t n = S.n;
  std::copy(S.u.begin(), S.u.end(), s->u);
  std::copy(S.uc.begin(), S.uc.end(), s->uc);
  std::copy(S.v.begin(), S.v.end(), s->v);
  std::copy(S.a.begin(), S.a.end(), s->a);
  std::copy(S.vol.begin(), S.vol.end(), s->vol);
  std::copy(S.phi.begin(), S.phi.end(), s->phi);
  std::copy(S.J.begin(), S.J.end(), s->J);
  std::copy(S.Sr.begin(), S.Sr.end(), s->Sr);
  std::copy(S.mass.begin(), S.mass.end(), s->mass);
  std::copy(S.sig.begin(), S.sig.end(), s->sig);
  std::copy(S.pc.begin(), S.pc.end(), s->pc);
  (void)n;
}

static void store_stats(const Stats& st, OracleStats* o) {
  if (!o) return;
  o->n_bonds = st.n_bonds; o->n_degenerate = st.n_degenerate; o->n_plastic = st.n_plastic;
  o->max_newton = st.max_newton; o->n_noconv = st.n_noconv; o->n_tests = st.n_tests;
  o->n_triples = st.n_triples;
}

extern "C" {

// Families of positions x (n*3).  brute != 0 selects the O(N^2) search.
// Fills row_ptr (n+1) and, if col_cap >= bonds, col; returns the bond count.
int64_t oracle_families(int64_t n, const double* x, double delta, int32_t brute, int64_t* row_ptr,
                        int32_t* col, int64_t col_cap) {
  Families F;
  if (brute) build_families_brute(n, x, delta, F);
  else build_families_cells(n, x, delta, F);
  const int64_t nb = F.row[n];
  std::copy(F.row.begin(), F.row.end(), row_ptr);
  if (col && col_cap >= nb) std::copy(F.col.begin(), F.col.end(), col);
  return nb;
}

// Alg. 1 at the state's positions x0 + u, with relative velocities from v and
// strain increment dt_inc * D.  Outputs in CSR order of the families at x.
// Any output pointer may be NULL.  Returns the bond count (or < 0 on error
// when cap is too small).
int64_t oracle_bond_fields(const OracleParams* op, const OracleState* os, double dt_inc, int64_t cap,
                           int64_t* row_ptr, int32_t* col, double* K, double* L, double* sig, double* pc,
                           double* T, double* varpi, int32_t* nsub, int8_t* active, double* f,
                           double* Jd, double* Sr_new, double* sig_pt, double* pc_pt, OracleStats* ost) {
  Params P = to_params(op);
  Mat<double> m = to_mat<double>(P);
  PointState<double> S;
  load_state(os, S);
  std::vector<double> x = positions(S);
  Families F;
  build_families_cells(S.n, x.data(), P.delta, F);
  build_reverse(S.n, F);
  const int64_t nb = F.row[S.n];
  if (nb > cap) return -nb;
  BondOut<double> O;
  Stats st;
  algorithm1(P, m, S.n, x.data(), x.data(), S.v.data(), S, F, dt_inc, O, st);
  const int64_t n = S.n;
  if (row_ptr) std::copy(F.row.begin(), F.row.end(), row_ptr);
  if (col) std::copy(F.col.begin(), F.col.end(), col);
  if (K) std::copy(O.K.begin(), O.K.end(), K);
  if (L) std::copy(O.L.begin(), O.L.end(), L);
  if (sig) std::copy(O.sig.begin(), O.sig.end(), sig);
  if (pc) std::copy(O.pc.begin(), O.pc.end(), pc);
  if (T) std::copy(O.T.begin(), O.T.end(), T);
  if (varpi) std::copy(O.varpi.begin(), O.varpi.end(), varpi);
  if (nsub) std::copy(O.nsub.begin(), O.nsub.end(), nsub);
  if (active) std::copy(O.active.begin(), O.active.end(), active);
  if (f) std::copy(O.f.begin(), O.f.end(), f);
  if (Jd) std::copy(O.Jd.begin(), O.Jd.end(), Jd);
  if (Sr_new) std::copy(O.Sr_new.begin(), O.Sr_new.end(), Sr_new);
  if (sig_pt) std::copy(O.sig_new.begin(), O.sig_new.end(), sig_pt);
  if (pc_pt) std::copy(O.pc_new.begin(), O.pc_new.end(), pc_pt);
  store_stats(st, ost);
  (void)n;
  return nb;
}

// Algorithm 2: n_steps explicit Newmark steps, state updated in place.
// energy[3] = (W_int, W_ext, W_kin) accumulated across calls by the caller.
int oracle_step(const OracleParams* op, OracleState* os, int32_t n_steps, double* energy,
                OracleStats* ost) {
  Params P = to_params(op);
  Mat<double> m = to_mat<double>(P);
  PointState<double> S;
  load_state(os, S);
  Stats st;
  int rc = 0;
  for (int k = 0; k < n_steps && rc == 0; ++k) rc = newmark_step(P, m, S, energy, st);
  store_state(S, os);
  store_stats(st, ost);
  return rc;
}

// Algorithm 2 with the history carried on the bonds (see BondHistory):
// bh holds the families and bond states of the last step (bh->nb = 0 or
// bh->n != n: none yet, every bond starts from its point) and receives those
// of the last step taken.  Returns -2 when bh->cap is too small.
typedef struct {
  int64_t n, cap, nb;
  int64_t* row;   // n+1
  int32_t* col;   // cap
  double* st;     // 8 per bond: sigma (6, Voigt), p_c, unused
} OracleBondHistory;

int oracle_step_bond_history(const OracleParams* op, OracleState* os, OracleBondHistory* bh, int32_t n_steps,
                             double* energy, OracleStats* ost) {
  Params P = to_params(op);
  Mat<double> m = to_mat<double>(P);
  PointState<double> S;
  load_state(os, S);
  BondHistory<double> H;
  if (bh->nb > 0 && bh->n == S.n) {
    H.row.assign(bh->row, bh->row + S.n + 1);
    H.col.assign(bh->col, bh->col + bh->nb);
    H.st.assign(bh->st, bh->st + 8 * bh->nb);
  }
  Stats st;
  int rc = 0;
  for (int k = 0; k < n_steps && rc == 0; ++k) rc = newmark_step(P, m, S, energy, st, nullptr, &H);
  store_state(S, os);
  store_stats(st, ost);
  const int64_t nb = H.row.empty() ? 0 : H.row.back();
  if (nb > bh->cap) return -2;
  bh->n = S.n;
  bh->nb = nb;
  if (nb > 0) {
    std::copy(H.row.begin(), H.row.end(), bh->row);
    std::copy(H.col.begin(), H.col.end(), bh->col);
    std::copy(H.st.begin(), H.st.end(), bh->st);
  }
  return rc;
}

// Initial conditions (Algorithm 2, set-up and initial acceleration) for a
// column whose caller has put the TOTAL geostatic stress in sig:
//   J = 1, u = 0, S_r0 from Eq. 15, effective stress sigma - S_r0 s 1 (Eq. 2
//   with p_w = -s), pre-consolidation from the over-consolidation ratio on
//   the yield surface through the current stress (Eq. 40), inverted through
//   Eq. 45; mass from Eq. 48; a0 = f0 / M0 + g with bond stress = point stress.
int oracle_init_state(const OracleParams* op, OracleState* os, double ocr) {
  Params P = to_params(op);
  Mat<double> m = to_mat<double>(P);
  const int64_t n = os->n;
  for (int64_t i = 0; i < n; ++i) {
    os->J[i] = 1.0;
    for (int c = 0; c < 3; ++c) os->u[3 * i + c] = os->uc[3 * i + c] = 0.0;
    double Sr = swrc(m, 1.0, os->phi[i], os->s[i]);
    os->Sr[i] = Sr;
    double* sg = &os->sig[6 * i];
    for (int k = 0; k < 3; ++k) sg[k] -= Sr * os->s[i];
    double p = (sg[0] + sg[1] + sg[2]) / 3.0;
    double dv[6];
    for (int k = 0; k < 6; ++k) dv[k] = sg[k] - (k < 3 ? p : 0.0);
    double q = std::sqrt(1.5 * (dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2] +
                                2.0 * (dv[3] * dv[3] + dv[4] * dv[4] + dv[5] * dv[5])));
    double pcb = ocr * (p + q * q / (P.M * P.M * p));
    os->pc[i] = -std::pow(-pcb * std::exp(-P.b1), 1.0 / P.b2);
    os->mass[i] = (P.rho_s * (1.0 - os->phi[i]) + P.rho_w * Sr * os->phi[i]) * os->vol[i];
  }
  PointState<double> S;
  load_state(os, S);
  std::vector<double> x = positions(S);
  Families F;
  build_families_cells(n, x.data(), P.delta, F);
  build_reverse(n, F);
  BondOut<double> O;
  Stats st;
  algorithm1(P, m, n, x.data(), x.data(), S.v.data(), S, F, 0.0, O, st);
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c)
      os->a[3 * i + c] = os->fixed[i] ? 0.0 : O.f[3 * i + c] / os->mass[i] + P.g[c];
  return 0;
}

// Critical time step, Eq. 65, read as sqrt(2 (1-phi) rho_s / sum_j V_j C/|zeta|)
// with the bond micro-modulus C = 18 K / (pi delta^4); minimum over points
// with a non-empty family.
double oracle_dt_crit(const OracleParams* op, const OracleState* os) {
  Params P = to_params(op);
  const int64_t n = os->n;
  std::vector<double> x(3 * n);
  for (int64_t k = 0; k < 3 * n; ++k) x[k] = os->x0[k] + os->u[k];
  Families F;
  build_families_cells(n, x.data(), P.delta, F);
  // bond micromodulus: 3D, or plane strain per unit thickness (Poisson 1/4)
  const double C = P.plane ? 72.0 * P.K / (5.0 * M_PI * std::pow(P.delta, 3))
                           : 18.0 * P.K / (M_PI * std::pow(P.delta, 4));
  double best = INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    double sum = 0.0;
    for (int64_t s = F.row[i]; s < F.row[i + 1]; ++s) {
      int64_t j = F.col[s];
      double z = std::sqrt(r2(&x[3 * i], &x[3 * j]));
      sum += os->vol[j] * C / z;
    }
    if (sum > 0.0) best = std::min(best, std::sqrt(2.0 * (1.0 - os->phi[i]) * P.rho_s / sum));
  }
  return best;
}

// Point-level constitutive update, for pins: returns Newton iterations
// (0 elastic, -1 no convergence).
int oracle_return_map(const OracleParams* op, double dt, const double* sig_n, double pc_n,
                      const double* deps, double* sig_out, double* pc_out) {
  Params P = to_params(op);
  Mat<double> m = to_mat<double>(P);
  return return_map(m, P, dt, sig_n, pc_n, deps, sig_out, pc_out);
}

void oracle_rm_residual(const OracleParams* op, double c, double ptr, double qtr, double pcn,
                        const double* x, double* r, double* A) {
  Params P = to_params(op);
  Mat<double> m = to_mat<double>(P);
  if (r) rm_residual(m, c, ptr, qtr, pcn, x, r);
  if (A) rm_jacobian(m, c, pcn, x, A);
}

double oracle_swrc(const OracleParams* op, double J, double phi, double s) {
  Params P = to_params(op);
  Mat<double> m = to_mat<double>(P);
  return swrc(m, J, phi, s);
}

// Forward-mode directional derivative of n_steps steps.  dstate holds the
// tangents of the state fields (x0 and fixed ignored); dparam[4] the tangents
// of (M, lam, kap, eta); the suction tangent is taken from dstate->s.  On return the state and its tangent are advanced.
static int step_dual_run(const OracleParams* op, const double* dparam, OracleState* os, OracleState* ds,
                         int32_t n_steps, double* energy, OracleStats* ost, BondHistory<Dual>* H) {
  Params P = to_params(op);
  Mat<Dual> m = to_mat<Dual>(P);
  m.M.d = dparam[0];
  m.lam.d = dparam[1];
  m.kap.d = dparam[2];
  m.eta.d = dparam[3];
  const int64_t n = os->n;
  PointState<Dual> S;
  S.n = n;
  S.x0.assign(os->x0, os->x0 + 3 * n);
  auto ld = [&](std::vector<Dual>& d, const double* v, const double* t, int64_t len) {
    d.resize(len);
    for (int64_t k = 0; k < len; ++k) d[k] = Dual(v[k], t[k]);
  };
  ld(S.u, os->u, ds->u, 3 * n);
  ld(S.uc, os->uc, ds->uc, 3 * n);
  ld(S.v, os->v, ds->v, 3 * n);
  ld(S.a, os->a, ds->a, 3 * n);
  ld(S.vol, os->vol, ds->vol, n);
  ld(S.phi, os->phi, ds->phi, n);
  ld(S.J, os->J, ds->J, n);
  ld(S.Sr, os->Sr, ds->Sr, n);
  ld(S.mass, os->mass, ds->mass, n);
  ld(S.s, os->s, ds->s, n);
  ld(S.sig, os->sig, ds->sig, 6 * n);
  ld(S.pc, os->pc, ds->pc, n);
  S.fixed.assign(os->fixed, os->fixed + n);
  Stats st;
  Dual E[3] = {Dual(energy[0]), Dual(energy[1]), Dual(energy[2])};
  int rc = 0;
  for (int k = 0; k < n_steps && rc == 0; ++k) rc = newmark_step(P, m, S, E, st, nullptr, H);
  auto st_back = [&](const std::vector<Dual>& d, double* v, double* t) {
    for (size_t k = 0; k < d.size(); ++k) { v[k] = d[k].v; t[k] = d[k].d; }
  };
  st_back(S.u, os->u, ds->u);
  st_back(S.uc, os->uc, ds->uc);
  st_back(S.v, os->v, ds->v);
  st_back(S.a, os->a, ds->a);
  st_back(S.vol, os->vol, ds->vol);
  st_back(S.phi, os->phi, ds->phi);
  st_back(S.J, os->J, ds->J);
  st_back(S.Sr, os->Sr, ds->Sr);
  st_back(S.mass, os->mass, ds->mass);
  st_back(S.sig, os->sig, ds->sig);
  st_back(S.pc, os->pc, ds->pc);
  for (int c = 0; c < 3; ++c) energy[c] = E[c].v;
  store_stats(st, ost);
  return rc;
}


int oracle_step_dual(const OracleParams* op, const double* dparam, OracleState* os, OracleState* ds,
                     int32_t n_steps, double* energy, OracleStats* ost) {
  return step_dual_run(op, dparam, os, ds, n_steps, energy, ost, nullptr);
}

// Forward-mode derivatives with the history on the bonds: dst holds the
// tangents of bh->st (8 per bond), read and written like bh.
int oracle_step_dual_bond_history(const OracleParams* op, const double* dparam, OracleState* os, OracleState* ds,
                                  OracleBondHistory* bh, double* dst, int32_t n_steps, double* energy,
                                  OracleStats* ost) {
  BondHistory<Dual> H;
  if (bh->nb > 0 && bh->n == os->n) {
    H.row.assign(bh->row, bh->row + os->n + 1);
    H.col.assign(bh->col, bh->col + bh->nb);
    H.st.resize(8 * bh->nb);
    for (int64_t k = 0; k < 8 * bh->nb; ++k) H.st[k] = Dual(bh->st[k], dst[k]);
  }
  const int rc = step_dual_run(op, dparam, os, ds, n_steps, energy, ost, &H);
  const int64_t nb = H.row.empty() ? 0 : H.row.back();
  if (nb > bh->cap) return -2;
  bh->n = os->n;
  bh->nb = nb;
  if (nb > 0) {
    std::copy(H.row.begin(), H.row.end(), bh->row);
    std::copy(H.col.begin(), H.col.end(), bh->col);
    for (int64_t k = 0; k < 8 * nb; ++k) { bh->st[k] = H.st[k].v; dst[k] = H.st[k].d; }
  }
  return rc;
}

}  // extern "C"
