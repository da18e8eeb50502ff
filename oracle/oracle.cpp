/*
 * FP64 CPU oracle of one time step of the synthetic-turbulence-generator (STG)
 * wall-modelled MRT lattice Boltzmann channel (Xue, Yao, Davidson,
 * "Synthetic turbulence generator for the wall-modeled LES lattice Boltzmann
 * method", arXiv 2304.04214).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the HIP library: every table below is typed
 * here from the paper.
 *
 * Structure: plain per-node loops in the order of the paper's Algorithm 1
 * (Sec. III.B): streaming with boundary rules, the inlet branch (STG velocity,
 * Zou-He density, regularised populations), the wall branch (base vector,
 * projected speed, Newton solve for u_tau, wall force), then MRT collision with
 * the Smagorinsky relaxation time.  The moment transform is the dense 19x19
 * matrix of Appendix A.1 and its numerical inverse.
 *
 * Readings of the paper used here (where it is garbled, silent or ambiguous):
 *  R1  m2_eq = 3 rho - (11/2) rho |u|^2  (the printed 11/2 rho (3 - |u|^2) is
 *      not the projection of the equilibrium), Sec. II.A, Eq. (8).
 *  R2  m4,6,8_eq = -(2/3) rho u_{x,y,z} (printed fraction inverted), Eq. (8).
 *  R3  rates: omega_0,3,5,7 = 1, omega_1 = 1.19 (omega_1 is listed twice),
 *      Appendix A.1.
 *  R4  Guo forcing applied in moment space: m* += (I - S/2) M Fbar, with Fbar
 *      the population form of Eq. (9) (the printed (1 - omega_i/2) mixes a
 *      moment index with a population index).
 *  R5  tau_eff = tau0/2 + sqrt(tau0^2 + 18 sqrt(2) C_smag Q^(1/2) / rho)/2,
 *      C_smag = C_s^2, Delta = dx = dt = 1 (Eq. (15) misplaces rho; this form
 *      is the root of Eq. (14) with Eq. (5) and Eq. (13)).
 *  R6  Reichardt law u+ = ln(1 + k y+)/k + B [1 - e^(-y+/11) - (y+/11) e^(-y+/3)],
 *      k = 0.41, B = 7.8 (the printed form has u+(1) = 0.80), Eq. (16).
 *  R7  regularised inlet: fneq_i = w_i/(2 cs^4) Q_i : Pi_neq (the printed
 *      w_i/cs^4 rebuilds 2 Pi_neq), Eq. (28).
 *  R8  inlet density rho_in = (rho_0 + 2 rho_-)/(1 - u_in,x), rho_0 over
 *      c_x = 0, rho_- over c_x < 0 (Zou-He mass balance), Eq. (30)-(31).
 *  R9  force density F = rho g + F_w; rho u = sum f c + F/2, Eq. (11).
 *  R10 wall-model velocities u_2 and u_w are the pre-force velocities j/rho of
 *      the post-streaming (post-boundary) state; y_perp = 1/2 (halfway walls);
 *      nu in y+ is the molecular nu0; F_w = -sign(u_hat) rho u_tau^2 e_x, A = 1.
 *  R11 Newton start u_tau = sqrt(nu0 |u_hat| / y_perp); iterate until
 *      |du| <= tol u_tau (max iterations given), then one more step.
 *  R12 STG phase at the inlet: k (d_y y + d_z z) + omega t + phi, y = iy + 1/2,
 *      z = iz; u' = s_b(y) a(y) v'; step n -> n+1 uses t = n+1.
 *  R13 outlet: convective rule f_i = (f_i^prev + U_c f_i(x-1)) / (1 + U_c) for
 *      c_x < 0 at x = nx-1, f(x-1) the post-streaming value of the same step.
 *  R14 inlet and wall rules both apply at inlet/wall corner cells
 *      (Algorithm 1 has two independent branches).
 *  R24 the Smagorinsky tau_eff (Algorithm 1 step 8, listed inside the inlet
 *      branch) applies at every cell: Sec. II.B gives it as the closure of
 *      the whole LES-LBM system.
 *  R20 "pressure-free" outlet, alternative reading: zero gradient,
 *      f_i = f_i(x-1) for c_x < 0 at x = nx-1 (the limit U_c -> infinity of R13).
 *  R21 Musker's law of the wall (Sec. II.C names it as the alternative to the
 *      Reichardt law, by citation): the explicit profile
 *      u+ = 5.424 atan((2y+ - 8.15)/16.7) + log10((y+ + 10.6)^9.6 / (y+^2 - 8.15y+ + 86)^2) + C
 *      with C the constant that gives u+(0) = 0 (C = -3.5113; the rounded -3.52
 *      usually printed leaves u+(0) = -0.0087, and then u_tau u+ = |u_hat| has no
 *      positive root once y+ < 0.009).  Written as differences from y+ = 0,
 *      5.424 [atan(t) - atan(t0)] + (9.6 ln(1 + y+/10.6) - 2 ln(1 + y+(y+ - 8.15)/86)) / ln 10,
 *      t = (2y+ - 8.15)/16.7, t0 = t(0), with atan(t) - atan(t0) = atan2(t - t0, 1 + t t0)
 *      and t - t0 = 2y+/16.7: every term is O(y+) at small y+, free of cancellation.
 *  R22 the "modified von Karman spectrum" of Eq. (25) (details deferred to the
 *      cited STG of Shur et al.): with RANS k(y), omega(y) and the wall
 *      distance d_w = min(y + 1/2, ny - y - 1/2) of each inlet row,
 *      l_t = sqrt(k)/(C_mu omega), l_e = min(2 d_w, C_l l_t), eta = (nu^3/eps)^(1/4),
 *      eps = C_mu k omega, l_cut = 2 min(max(h_y, h_z, 0.3 h_max) + 0.1 d_w, h_max)
 *      (= 2 on the unit lattice), k_e, k_eta, k_cut = 2 pi / (l_e, eta, l_cut);
 *      E(k) = (k/k_e)^4 / (1 + 2.4 (k/k_e)^2)^(17/6) exp(-(12 k/k_eta)^2)
 *             exp(-(4 max(k - 0.9 k_cut, 0)/k_cut)^3),
 *      q^n(y) = E(k_n) dk_n / sum_m E(k_m) dk_m, C_mu = 0.09, C_l = 3, nu = nu0,
 *      dk_n the centred differences of the ascending k_n (one-sided at the ends).
 *      Without k, omega a single table q^n serves every row.
 *  R23 plane-averaged friction velocity (Sec. II.C contrasts its local u_tau
 *      with the plane-averaged one of the works it cites): with wall_avg = 1
 *      the wall-parallel average runs over the homogeneous direction z of
 *      each wall line (x, wall) of the inflow channel; u_hat = u_w . e_x
 *      (Eq. (19), 0 where u_2 has no tangential part) is averaged over z,
 *      u_tau(x, wall) solves Eq. (20) for |mean u_hat| in the same step, and
 *      every cell of the line takes F_w = -sign(mean u_hat) rho u_tau^2 e_x with
 *      its own rho and e_x (Eq. (21)).
 *  R19 outlet sponge (Sec. IV.A names a sponge of thickness delta before the
 *      outlet but not its law): over the last L = sponge_cells planes the
 *      molecular viscosity rises as nu(x) = nu0 + (nu_s - nu0) r^2,
 *      r = (x - (nx - L) + 1) / L, so tau0(x) = 1/2 + 3 nu(x) in Eq. (5) and
 *      Eq. (15); nu in the wall law's y+ stays nu0.
 */
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

extern "C" {

typedef struct {
  int32_t nx, ny, nz;
  int32_t ywall;       /* 0 periodic, 1 halfway bounce-back, 2 specular slip */
  int32_t xbc;         /* 0 periodic, 1 STG inlet at x = 0 and convective outlet at x = nx-1 */
  int32_t wall_model;  /* 1: Reichardt wall force in the first off-wall cells */
  int32_t newton_max;  /* maximum Newton iterations (oracle converges to newton_tol) */
  int32_t sponge_cells;/* outlet sponge: the last sponge_cells x planes (0: none), reading R19 */
  double newton_tol;
  double tau0;         /* molecular relaxation time, nu0 = (tau0 - 1/2)/3 */
  double cs_smag;      /* Smagorinsky C_s, C_smag = C_s^2 */
  double s[19];        /* relaxation rates; 9, 11, 13, 14, 15 are replaced by 1/tau_eff */
  double kappa, b_reich, y_wall;
  double u_conv;       /* outlet convection speed U_c */
  double g[3];         /* body acceleration */
  double sponge_nu;    /* molecular viscosity at the outlet plane inside the sponge */
  int32_t outlet;      /* 0 convective (R13), 1 zero gradient (R20) */
  int32_t wall_law;    /* 0 Reichardt (R6), 1 Musker (R21) */
  int32_t wall_avg;    /* 0 local u_tau (Sec. II.C), 1 z-line average (R23) */
  int32_t pad_;
} oracle_cfg;

typedef struct {
  int32_t n_modes, n_bins;
  const double* q;        /* [N] spectral weights, sum 1 */
  const double* sigma;    /* [3][N] unit amplitude directions, sigma . d = 0 */
  const double* kmag;     /* [N] wavenumber magnitudes */
  const double* d;        /* [3][N] unit wave directions */
  const double* phi;      /* [N] phases */
  const double* omega;    /* [N] temporal frequencies (rad per step) */
  const double* u_rans;   /* [3][ny] mean inflow */
  const double* R;        /* [6][ny] R11 R21 R22 R31 R32 R33 */
  const double* amp_bin;  /* [n_bins] amplitude scalings s_b */
  const int32_t* bin_of_y;/* [ny] */
  const double* k_rans;   /* [ny] RANS turbulent kinetic energy, or NULL (then q is used) */
  const double* omega_rans;/* [ny] RANS specific dissipation rate */
} oracle_stg;

}  // extern "C"

enum { OR_OK = 0, OR_ERR_ARG = 1, OR_ERR_MACH = 4, OR_ERR_NONFINITE = 5, OR_ERR_NEWTON = 7 };

namespace {

/* ---- Sec. II.A, Eq. (1): the D3Q19 velocity set, in the paper's order ---- */
const int C[19][3] = {
    {0, -1, -1}, {-1, 0, -1}, {0, 0, -1}, {1, 0, -1}, {0, 1, -1},
    {-1, -1, 0}, {0, -1, 0},  {1, -1, 0}, {-1, 0, 0}, {0, 0, 0},
    {1, 0, 0},   {-1, 1, 0},  {0, 1, 0},  {1, 1, 0},  {0, -1, 1},
    {-1, 0, 1},  {0, 0, 1},   {1, 0, 1},  {0, 1, 1}};

/* ---- Appendix A.1: the MRT matrix as printed ---- */
const int MI[19][19] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {8, 8, -11, 8, 8, 8, -11, 8, -11, -30, -11, 8, -11, 8, 8, 8, -11, 8, 8},
    {1, 1, -4, 1, 1, 1, -4, 1, -4, 12, -4, 1, -4, 1, 1, 1, -4, 1, 1},
    {0, -1, 0, 1, 0, -1, 0, 1, -1, 0, 1, -1, 0, 1, 0, -1, 0, 1, 0},
    {0, -1, 0, 1, 0, -1, 0, 1, 4, 0, -4, -1, 0, 1, 0, -1, 0, 1, 0},
    {-1, 0, 0, 0, 1, -1, -1, -1, 0, 0, 0, 1, 1, 1, -1, 0, 0, 0, 1},
    {-1, 0, 0, 0, 1, -1, 4, -1, 0, 0, 0, 1, -4, 1, -1, 0, 0, 0, 1},
    {-1, -1, -1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1},
    {-1, -1, 4, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -4, 1, 1},
    {-2, 1, -1, 1, -2, 1, -1, 1, 2, 0, 2, 1, -1, 1, -2, 1, -1, 1, -2},
    {-2, 1, 2, 1, -2, 1, 2, 1, -4, 0, -4, 1, 2, 1, -2, 1, 2, 1, -2},
    {0, -1, -1, -1, 0, 1, 1, 1, 0, 0, 0, 1, 1, 1, 0, -1, -1, -1, 0},
    {0, -1, 2, -1, 0, 1, -2, 1, 0, 0, 0, 1, -2, 1, 0, -1, 2, -1, 0},
    {0, 0, 0, 0, 0, 1, 0, -1, 0, 0, 0, -1, 0, 1, 0, 0, 0, 0, 0},
    {1, 0, 0, 0, -1, 0, 0, 0, 0, 0, 0, 0, 0, 0, -1, 0, 0, 0, 1},
    {0, 1, 0, -1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, -1, 0, 1, 0},
    {0, 1, 0, -1, 0, -1, 0, 1, 0, 0, 0, -1, 0, 1, 0, 1, 0, -1, 0},
    {-1, 0, 0, 0, 1, 1, 0, 1, 0, 0, 0, -1, 0, -1, -1, 0, 0, 0, 1},
    {1, -1, 0, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, -1, 1, 0, 1, -1}};

const double CS2 = 1.0 / 3.0; /* Sec. II.A: c_s^2 = 1/3 */

struct Tables {
  double W[19];
  double M[19][19];
  double Minv[19][19];
  int opp[19];
  int refl_y[19];
  Tables() {
    /* Sec. II.A, Eq. (2): weights listed by index */
    for (int i = 0; i < 19; ++i) W[i] = 1.0 / 36.0;
    const int axis[6] = {2, 6, 8, 10, 12, 16};
    for (int k = 0; k < 6; ++k) W[axis[k]] = 1.0 / 18.0;
    W[9] = 1.0 / 3.0;
    for (int a = 0; a < 19; ++a)
      for (int b = 0; b < 19; ++b) M[a][b] = MI[a][b];
    /* opposite and y-mirror directions found by search over the set */
    for (int i = 0; i < 19; ++i) {
      opp[i] = refl_y[i] = -1;
      for (int j = 0; j < 19; ++j) {
        if (C[j][0] == -C[i][0] && C[j][1] == -C[i][1] && C[j][2] == -C[i][2]) opp[i] = j;
        if (C[j][0] == C[i][0] && C[j][1] == -C[i][1] && C[j][2] == C[i][2]) refl_y[i] = j;
      }
    }
    invert();
  }
  /* Gauss-Jordan elimination with partial pivoting: M^-1 numerically */
  void invert() {
    double a[19][38];
    for (int r = 0; r < 19; ++r)
      for (int c = 0; c < 38; ++c) a[r][c] = c < 19 ? M[r][c] : (c - 19 == r ? 1.0 : 0.0);
    for (int col = 0; col < 19; ++col) {
      int piv = col;
      for (int r = col + 1; r < 19; ++r)
        if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
      if (piv != col)
        for (int c = 0; c < 38; ++c) std::swap(a[piv][c], a[col][c]);
      double p = a[col][col];
      for (int c = 0; c < 38; ++c) a[col][c] /= p;
      for (int r = 0; r < 19; ++r) {
        if (r == col) continue;
        double fac = a[r][col];
        if (fac == 0.0) continue;
        for (int c = 0; c < 38; ++c) a[r][c] -= fac * a[col][c];
      }
    }
    for (int r = 0; r < 19; ++r)
      for (int c = 0; c < 19; ++c) Minv[r][c] = a[r][19 + c];
  }
};

const Tables& T() {
  static Tables t;
  return t;
}

/* Deliberate mistakes switched on only by tests that check a pin catches them. */
int g_mutation = 0;

inline double val(double x) { return x; }

/*
 * Forward-mode dual numbers with K derivative slots: v + sum_k d_k e_k,
 * e_k e_l = 0.  Every template below is written for a generic real type, so
 * evaluating it on Duals gives the exact local Jacobian of that step
 * (used by the adjoint).
 */
template <int K>
struct Dual {
  double v;
  double d[K];
  Dual() : v(0.0) { std::memset(d, 0, sizeof(d)); }
  Dual(double x) : v(x) { std::memset(d, 0, sizeof(d)); }  // NOLINT: constants promote
  static Dual seed(double x, int k) {
    Dual r(x);
    r.d[k] = 1.0;
    return r;
  }
};
template <int K>
double val(const Dual<K>& x) { return x.v; }
template <int K>
Dual<K> chain(const Dual<K>& a, double fa, double dfa) { /* g(a) with g = fa, g' = dfa */
  Dual<K> r;
  r.v = fa;
  for (int k = 0; k < K; ++k) r.d[k] = dfa * a.d[k];
  return r;
}
template <int K>
Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r;
  r.v = a.v + b.v;
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int K>
Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r;
  r.v = a.v - b.v;
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int K>
Dual<K> operator-(const Dual<K>& a) { return chain(a, -a.v, -1.0); }
template <int K>
Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r;
  r.v = a.v * b.v;
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int K>
Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r;
  r.v = a.v / b.v;
  for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
  return r;
}
template <int K> Dual<K> operator+(const Dual<K>& a, double b) { return a + Dual<K>(b); }
template <int K> Dual<K> operator+(double a, const Dual<K>& b) { return Dual<K>(a) + b; }
template <int K> Dual<K> operator-(const Dual<K>& a, double b) { return a - Dual<K>(b); }
template <int K> Dual<K> operator-(double a, const Dual<K>& b) { return Dual<K>(a) - b; }
template <int K> Dual<K> operator*(const Dual<K>& a, double b) { return chain(a, a.v * b, b); }
template <int K> Dual<K> operator*(double a, const Dual<K>& b) { return chain(b, a * b.v, a); }
template <int K> Dual<K> operator/(const Dual<K>& a, double b) { return chain(a, a.v / b, 1.0 / b); }
template <int K> Dual<K> operator/(double a, const Dual<K>& b) { return Dual<K>(a) / b; }
template <int K> bool operator==(const Dual<K>& a, double b) { return a.v == b; }
template <int K> Dual<K> sqrt(const Dual<K>& a) { const double r = std::sqrt(a.v); return chain(a, r, 0.5 / r); }
template <int K> Dual<K> exp(const Dual<K>& a) { const double e = std::exp(a.v); return chain(a, e, e); }
template <int K> Dual<K> log(const Dual<K>& a) { return chain(a, std::log(a.v), 1.0 / a.v); }
template <int K> Dual<K> log1p(const Dual<K>& a) { return chain(a, std::log1p(a.v), 1.0 / (1.0 + a.v)); }
template <int K> Dual<K> expm1(const Dual<K>& a) { return chain(a, std::expm1(a.v), std::exp(a.v)); }
template <int K> Dual<K> atan(const Dual<K>& a) { return chain(a, std::atan(a.v), 1.0 / (1.0 + a.v * a.v)); }
template <int K>
Dual<K> atan2(const Dual<K>& y, const Dual<K>& x) {
  Dual<K> r;
  r.v = std::atan2(y.v, x.v);
  const double n = x.v * x.v + y.v * y.v;
  for (int k = 0; k < K; ++k) r.d[k] = (x.v * y.d[k] - y.v * x.d[k]) / n;
  return r;
}

/* ---- Sec. III.A, Eq. (27): second-order equilibrium ---- */
template <class R>
void feq_poly(const R& rho, const R u[3], R out[19]) {
  const Tables& t = T();
  R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < 19; ++i) {
    R cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
    out[i] = t.W[i] * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

/* ---- Sec. II.A, Eq. (8): equilibrium moments (readings R1, R2) ---- */
template <class R>
void meq_moments(const R& rho, const R u[3], R m[19]) {
  const R ux = u[0], uy = u[1], uz = u[2];
  const R uu = ux * ux + uy * uy + uz * uz;
  m[0] = rho;
  m[1] = -11.0 * rho + 19.0 * rho * uu;
  m[2] = (g_mutation == 1) ? 5.5 * rho * (3.0 - uu) : 3.0 * rho - 5.5 * rho * uu;
  const double c4 = (g_mutation == 2) ? -1.5 : -2.0 / 3.0;
  m[3] = rho * ux;
  m[4] = c4 * rho * ux;
  m[5] = rho * uy;
  m[6] = c4 * rho * uy;
  m[7] = rho * uz;
  m[8] = c4 * rho * uz;
  m[9] = 2.0 * rho * ux * ux - rho * uy * uy - rho * uz * uz;
  m[10] = -rho * ux * ux + 0.5 * rho * uy * uy + 0.5 * rho * uz * uz;
  m[11] = rho * uy * uy - rho * uz * uz;
  m[12] = -0.5 * rho * uy * uy + 0.5 * rho * uz * uz;
  m[13] = rho * ux * uy;
  m[14] = rho * uy * uz;
  m[15] = rho * ux * uz;
  m[16] = m[17] = m[18] = 0.0 * rho;
}

/* ---- Sec. II.A, Eq. (9): Guo forcing populations for force density F ---- */
template <class R>
void guo_populations(const R u[3], const R F[3], R out[19]) {
  const Tables& t = T();
  for (int i = 0; i < 19; ++i) {
    R cu = C[i][0] * u[0] + C[i][1] * u[1] + C[i][2] * u[2];
    R acc = 0.0 * u[0];
    for (int a = 0; a < 3; ++a) {
      R ua = (g_mutation == 3) ? 0.0 * u[a] : u[a];
      acc = acc + ((C[i][a] - ua) / CS2 + cu * C[i][a] / (CS2 * CS2)) * F[a];
    }
    out[i] = t.W[i] * acc;
  }
}

/* ---- Sec. IV.A with reading R19: molecular relaxation time of plane x ---- */
double tau0_at(const oracle_cfg& cfg, int x) {
  const int L = cfg.sponge_cells;
  if (L <= 0 || x < cfg.nx - L) return cfg.tau0;
  const double nu0 = (cfg.tau0 - 0.5) * (1.0 / 3.0);
  const double r = (double)(x - (cfg.nx - L) + 1) / L;
  const double ramp = (g_mutation == 11) ? r : r * r;
  return 0.5 + 3.0 * (nu0 + (cfg.sponge_nu - nu0) * ramp);
}

/* ---- Sec. II.B, Eq. (13)-(15): Smagorinsky relaxation time (reading R5) ---- */
template <class R, class C>
R tau_eff_of(const R& Qhalf, const R& rho, double tau0, const C& cs_smag) {
  using std::sqrt;
  const C csmag = cs_smag * cs_smag;
  return 0.5 * tau0 + 0.5 * sqrt(tau0 * tau0 + 18.0 * std::sqrt(2.0) * csmag * Qhalf / rho);
}

/* sqrt that is 0 with zero derivative at 0 (Pi_neq = 0 exactly) */
template <class R>
R safe_norm(const R& s2) {
  using std::sqrt;
  if (s2 == 0.0) return 0.0 * s2;
  return sqrt(s2);
}

/*
 * ---- Sec. II.A-II.B: MRT collision with forcing and Smagorinsky closure ----
 * f: post-streaming populations of one node; F: force density.
 * out: post-collision populations.  u_out (optional): rho u = sum f c + F/2.
 */
template <class R>
void collide(const oracle_cfg& cfg, double tau0, const R f[19], const R F[3], const R& cs_smag, R out[19],
             R* tau_out, R u_out[3]) {
  using std::sqrt;
  const Tables& t = T();
  R rho = 0.0 * f[0], j[3] = {0.0 * f[0], 0.0 * f[0], 0.0 * f[0]};
  for (int i = 0; i < 19; ++i) {
    rho = rho + f[i];
    for (int a = 0; a < 3; ++a) j[a] = j[a] + f[i] * C[i][a];
  }
  R u[3];
  for (int a = 0; a < 3; ++a) u[a] = (g_mutation == 4) ? j[a] / rho : (j[a] + 0.5 * F[a]) / rho; /* Eq. (11) */
  /* Eq. (7): m = M f */
  R m[19];
  for (int k = 0; k < 19; ++k) {
    R acc = 0.0 * f[0];
    for (int i = 0; i < 19; ++i) acc = acc + t.M[k][i] * f[i];
    m[k] = acc;
  }
  R meq[19];
  meq_moments(rho, u, meq);
  /* Eq. (12) and Pi = Pi_eq + Pi_neq with Pi_eq = rho cs^2 I + rho u u */
  R Pn[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      R acc = 0.0 * f[0];
      for (int i = 0; i < 19; ++i) acc = acc + f[i] * (double)(C[i][a] * C[i][b]);
      Pn[a][b] = acc - rho * u[a] * u[b] - (a == b ? rho * CS2 : 0.0 * rho);
    }
  R q2 = 0.0 * f[0];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) q2 = q2 + Pn[a][b] * Pn[a][b];
  R Qhalf = safe_norm(q2);
  R tau = tau_eff_of(Qhalf, rho, tau0, cs_smag);
  if (tau_out) *tau_out = tau;
  R S[19];
  for (int k = 0; k < 19; ++k) S[k] = cfg.s[k] + 0.0 * f[0];
  const int visc[5] = {9, 11, 13, 14, 15}; /* Sec. II.A: tau_k set */
  for (int k = 0; k < 5; ++k) S[visc[k]] = 1.0 / tau;
  /* Eq. (9) projected to moments (reading R4) */
  R Fb[19], Fm[19];
  guo_populations(u, F, Fb);
  for (int k = 0; k < 19; ++k) {
    R acc = 0.0 * f[0];
    for (int i = 0; i < 19; ++i) acc = acc + t.M[k][i] * Fb[i];
    Fm[k] = acc;
  }
  /* Eq. (6): relax in moment space, then back to populations */
  R ms[19];
  for (int k = 0; k < 19; ++k) ms[k] = m[k] - S[k] * (m[k] - meq[k]) + (1.0 - 0.5 * S[k]) * Fm[k];
  for (int i = 0; i < 19; ++i) {
    R acc = 0.0 * f[0];
    for (int k = 0; k < 19; ++k) acc = acc + t.Minv[i][k] * ms[k];
    out[i] = acc;
  }
  if (u_out)
    for (int a = 0; a < 3; ++a) u_out[a] = u[a];
}

/* ---- Sec. II.C, Eq. (16) with reading R6 ---- */
template <class R>
R uplus(const R& yp, double kappa, double B) {
  using std::exp;
  using std::expm1;
  using std::log;
  using std::log1p;
  if (g_mutation == 5) return 2.5 * log(1.0 + 0.4 * yp) + 7.8 * (1.0 - exp(-yp / 11.0)) - yp * exp(-yp / 3.0);
  /* planted misreadings of the buffer-layer term (tests only): 17 the e^(-y+/3)
     decay read as e^(-y+/2), 18 its y+/11 prefactor read as y+/10 */
  const double c3 = (g_mutation == 17) ? 2.0 : 3.0, c11 = (g_mutation == 18) ? 10.0 : 11.0;
  /* ln(1 + k y+) and 1 - e^(-y+/11) evaluated as log1p / -expm1: the same
     function, without the cancellation at small y+ */
  return log1p(kappa * yp) / kappa + B * (-expm1(-yp / 11.0) - (yp / c11) * exp(-yp / c3));
}
template <class R>
R duplus(const R& yp, double kappa, double B) {
  using std::exp;
  /* the same planted misreadings as uplus, differentiated consistently */
  const double c3 = (g_mutation == 17) ? 2.0 : 3.0, c11 = (g_mutation == 18) ? 10.0 : 11.0;
  return 1.0 / (1.0 + kappa * yp) +
         B * (exp(-yp / 11.0) / 11.0 - exp(-yp / c3) / c11 + (yp / (c11 * c3)) * exp(-yp / c3));
}

/* ---- Sec. II.C with reading R21: Musker's explicit law of the wall ---- */
template <class R>
R uplus_musker(const R& yp) {
  using std::atan2;
  using std::log1p;
  const double c = (g_mutation == 12) ? -8.15 : 8.15;
  const R t = (2.0 * yp - c) / 16.7;
  const double t0 = -8.15 / 16.7;
  const R dt = 2.0 * yp / 16.7 + (8.15 - c) / 16.7; /* t - t0 */
  return 5.424 * atan2(dt, 1.0 + t0 * t) + (9.6 * log1p(yp / 10.6) - 2.0 * log1p(yp * (yp - 8.15) / 86.0)) /
                                               std::log(10.0);
}
template <class R>
R duplus_musker(const R& yp) {
  const R t = (2.0 * yp - 8.15) / 16.7;
  const R q = yp * yp - 8.15 * yp + 86.0;
  return 5.424 * (2.0 / 16.7) / (1.0 + t * t) + (9.6 / (yp + 10.6) - 2.0 * (2.0 * yp - 8.15) / q) / std::log(10.0);
}
template <class R>
R law_uplus(const oracle_cfg& cfg, const R& yp) {
  return cfg.wall_law == 1 ? uplus_musker(yp) : uplus(yp, cfg.kappa, cfg.b_reich);
}
template <class R>
R law_duplus(const oracle_cfg& cfg, const R& yp) {
  return cfg.wall_law == 1 ? duplus_musker(yp) : duplus(yp, cfg.kappa, cfg.b_reich);
}

/* ---- Sec. II.C, Eq. (20): u_tau u+(y u_tau / nu) = |u_hat| by Newton (R11) ---- */
template <class R>
int solve_utau(const R& ua, double y, double nu, const oracle_cfg& cfg, R* out) {
  using std::sqrt;
  R ut = sqrt(nu * ua / y);
  for (int it = 0; it < cfg.newton_max; ++it) {
    R yp = y * ut / nu;
    R up = law_uplus(cfg, yp);
    R g = ut * up - ua;
    R dg = up + yp * law_duplus(cfg, yp);
    R du = g / dg;
    ut = ut - du;
    if (std::fabs(val(du)) <= cfg.newton_tol * std::fabs(val(ut))) {
      yp = y * ut / nu;
      up = law_uplus(cfg, yp);
      g = ut * up - ua;
      dg = up + yp * law_duplus(cfg, yp);
      ut = ut - g / dg; /* one more step: exact implicit-function derivative */
      *out = ut;
      /* a root u_tau <= 0 is not a friction velocity (the Musker fit is negative for y+ < 0.009) */
      return val(ut) > 0.0 ? OR_OK : OR_ERR_NEWTON;
    }
  }
  *out = ut;
  return OR_ERR_NEWTON;
}

/* ---- Sec. II.C, Eq. (18)-(21): wall force in a first off-wall cell (R10) ---- */
/* Eq. (18): the wall-parallel unit vector from the tangential part of u_2;
   false when that part vanishes. */
template <class R>
bool wall_basis(const R u2[3], int top, R e[3]) {
  using std::sqrt;
  const double n[3] = {0.0, top ? -1.0 : 1.0, 0.0};
  R un = u2[0] * n[0] + u2[1] * n[1] + u2[2] * n[2];
  R tv[3];
  for (int a = 0; a < 3; ++a) tv[a] = u2[a] - un * n[a];
  R tn2 = tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2];
  if (val(tn2) == 0.0) return false;
  R tn = sqrt(tn2);
  for (int a = 0; a < 3; ++a) e[a] = tv[a] / tn;
  return true;
}

/* Eq. (19): u_hat = u_w . e_x, 0 where e_x is undefined. */
template <class R>
R wall_uhat(const R uw[3], const R u2[3], int top) {
  R e[3];
  if (!wall_basis(u2, top, e)) return 0.0 * uw[0];
  return uw[0] * e[0] + uw[1] * e[1] + uw[2] * e[2];
}

/* Reading R23: the signed friction velocity sign(ubar) u_tau of a wall line from the
   z-mean ubar of u_hat (Eq. (20) for |ubar|); 0 when ubar = 0. */
template <class R>
int line_utau(const oracle_cfg& cfg, const R& ubar, R* out) {
  const double s = val(ubar) > 0.0 ? 1.0 : (val(ubar) < 0.0 ? -1.0 : 0.0);
  *out = 0.0 * ubar;
  if (s == 0.0) return OR_OK;
  R ut;
  const int st = solve_utau(s * ubar, cfg.y_wall, (cfg.tau0 - 0.5) * CS2, cfg, &ut);
  *out = s * ut;
  return st;
}

template <class R>
int wall_force(const oracle_cfg& cfg, const R& rho_w, const R uw[3], const R u2[3], int top, R F[3],
               R* utau_out, const R* line = nullptr) {
  for (int a = 0; a < 3; ++a) F[a] = 0.0 * rho_w;
  if (utau_out) *utau_out = 0.0 * rho_w;
  R e[3];
  if (line) { /* R23: the line's u_tau, the cell's own rho and e_x */
    const double s = val(*line) > 0.0 ? 1.0 : (val(*line) < 0.0 ? -1.0 : 0.0);
    if (utau_out) *utau_out = s * (*line);
    if (s == 0.0 || !wall_basis(u2, top, e)) return OR_OK;
    R tauw = rho_w * (*line) * (*line);
    for (int a = 0; a < 3; ++a) F[a] = -s * tauw * e[a]; /* Eq. (21), A = 1 */
    return OR_OK;
  }
  if (!wall_basis(u2, top, e)) return OR_OK; /* Eq. (18) */
  R uhat = uw[0] * e[0] + uw[1] * e[1] + uw[2] * e[2]; /* Eq. (19) */
  if (val(uhat) == 0.0) return OR_OK;
  const double sgn = val(uhat) > 0.0 ? 1.0 : -1.0;
  R ua = sgn * uhat;
  const double nu0 = (cfg.tau0 - 0.5) * CS2; /* Eq. (5) */
  R ut;
  int st = solve_utau(ua, cfg.y_wall, nu0, cfg, &ut);
  R tauw = rho_w * ut * ut; /* tau_w = rho u_tau^2 */
  for (int a = 0; a < 3; ++a) F[a] = -sgn * tauw * e[a]; /* Eq. (21), A = 1 */
  if (utau_out) *utau_out = ut;
  return st;
}

/* ---- Sec. III.A, Eq. (26)-(31): regularised inlet populations (R7, R8) ---- */
template <class R>
void inlet_regularize(const R f[19], const R uin[3], R out[19], R* rho_in_out) {
  const Tables& t = T();
  R rho0 = 0.0 * f[9], rhom = 0.0 * f[9];
  for (int i = 0; i < 19; ++i) {
    if (C[i][0] == 0) rho0 = rho0 + f[i];
    if (C[i][0] < 0) rhom = rhom + f[i];
  }
  R rho_in = (g_mutation == 6) ? (2.0 * rho0 + rhom) / (1.0 + uin[0]) : (rho0 + 2.0 * rhom) / (1.0 - uin[0]);
  R feq[19];
  feq_poly(rho_in, uin, feq);
  R fneq[19];
  for (int i = 0; i < 19; ++i)
    if (C[i][0] <= 0) fneq[i] = f[i] - feq[i];
  for (int i = 0; i < 19; ++i)
    if (C[i][0] > 0) fneq[i] = fneq[t.opp[i]];
  R Pi[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      R acc = 0.0 * f[9];
      for (int i = 0; i < 19; ++i) acc = acc + ((double)(C[i][a] * C[i][b]) - (a == b ? CS2 : 0.0)) * fneq[i];
      Pi[a][b] = acc; /* Eq. (29) */
    }
  const double fac = (g_mutation == 7) ? 1.0 / (CS2 * CS2) : 1.0 / (2.0 * CS2 * CS2);
  for (int i = 0; i < 19; ++i) {
    R qp = 0.0 * f[9];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) qp = qp + ((double)(C[i][a] * C[i][b]) - (a == b ? CS2 : 0.0)) * Pi[a][b];
    out[i] = feq[i] + t.W[i] * fac * qp; /* Eq. (26), (28) */
  }
  if (rho_in_out) *rho_in_out = rho_in;
}

/* ---- Sec. III.A, Eq. (24): Cholesky factor of R, [a11 a21 a22 a31 a32 a33] ---- */
void cholesky(const double R6[6], double a[6]) {
  /* R6 = R11 R21 R22 R31 R32 R33 */
  a[0] = std::sqrt(R6[0]);
  a[1] = R6[1] / a[0];
  a[2] = std::sqrt(R6[2] - a[1] * a[1]);
  a[3] = R6[3] / a[0];
  a[4] = (R6[4] - a[1] * a[3]) / a[2];
  a[5] = std::sqrt(R6[5] - a[3] * a[3] - a[4] * a[4]);
}

/* ---- Sec. III.A, Eq. (22)-(25): STG inlet velocity plane at time t (R12) ---- */
/* ---- Sec. III.A, Eq. (25) with reading R22: spectral weights of one inlet row ---- */
int stg_weights(const oracle_cfg& cfg, const oracle_stg& s, int y, double* q) {
  const int N = s.n_modes, ny = cfg.ny;
  if (!s.k_rans) {
    if (!s.q) return OR_ERR_ARG;
    for (int n = 0; n < N; ++n) q[n] = s.q[n];
    return OR_OK;
  }
  if (!s.omega_rans || cfg.ywall == 0) return OR_ERR_ARG; /* the spectrum needs a wall distance */
  const double PI = 3.14159265358979323846;
  const double Cmu = 0.09, Cl = 3.0;
  const double nu = (cfg.tau0 - 0.5) * CS2;
  const double k = s.k_rans[y], om = s.omega_rans[y];
  if (!(k > 0.0) || !(om > 0.0) || !std::isfinite(k) || !std::isfinite(om)) return OR_ERR_ARG;
  const double dw = std::fmin(y + 0.5, ny - y - 0.5);
  const double lt = (g_mutation == 14) ? std::sqrt(k) / om : std::sqrt(k) / (Cmu * om);
  const double le = std::fmin(2.0 * dw, Cl * lt);
  const double eta = std::pow(nu * nu * nu / (Cmu * k * om), 0.25);
  const double h = 1.0; /* lattice spacing in every direction */
  const double lcut = 2.0 * std::fmin(std::fmax(std::fmax(h, h), 0.3 * h) + 0.1 * dw, h);
  const double ke = 2.0 * PI / le, keta = 2.0 * PI / eta, kcut = 2.0 * PI / lcut;
  const double p = (g_mutation == 13) ? 11.0 / 6.0 : 17.0 / 6.0;
  double sum = 0.0;
  for (int n = 0; n < N; ++n) {
    if (n > 0 && !(s.kmag[n] > s.kmag[n - 1])) return OR_ERR_ARG;
    double dk = 1.0;
    if (N > 1) {
      const int lo = n > 0 ? n - 1 : 0, hi = n < N - 1 ? n + 1 : N - 1;
      dk = (s.kmag[hi] - s.kmag[lo]) / (hi - lo);
    }
    const double kn = s.kmag[n], r = kn / ke;
    const double E = std::pow(r, 4.0) / std::pow(1.0 + 2.4 * r * r, p) * std::exp(-std::pow(12.0 * kn / keta, 2.0)) *
                     std::exp(-std::pow(4.0 * std::fmax(kn - 0.9 * kcut, 0.0) / kcut, 3.0));
    q[n] = E * dk;
    sum += q[n];
  }
  if (!(sum > 0.0)) return OR_ERR_ARG;
  for (int n = 0; n < N; ++n) q[n] /= sum;
  return OR_OK;
}

int stg_plane(const oracle_cfg& cfg, const oracle_stg& s, double t, double* uin, double* fluct) {
  const int ny = cfg.ny, nz = cfg.nz, N = s.n_modes;
  int st = OR_OK;
  std::vector<double> q(N);
  for (int y = 0; y < ny; ++y) {
    const int sw = stg_weights(cfg, s, y, q.data());
    if (sw != OR_OK) return sw;
    double R6[6], a[6];
    for (int k = 0; k < 6; ++k) R6[k] = s.R[k * ny + y];
    cholesky(R6, a);
    const double sb = s.amp_bin[s.bin_of_y[y]];
    const double yc = y + 0.5;
    for (int z = 0; z < nz; ++z) {
      double v[3] = {0, 0, 0};
      for (int n = 0; n < N; ++n) {
        const double ph = s.kmag[n] * (s.d[1 * N + n] * yc + s.d[2 * N + n] * z) + s.omega[n] * t + s.phi[n];
        const double c = std::cos(ph);
        const double amp = std::sqrt(6.0 * q[n]); /* Eq. (25): sqrt(6) sqrt(q^n) */
        for (int a3 = 0; a3 < 3; ++a3) v[a3] += amp * s.sigma[a3 * N + n] * c;
      }
      /* Eq. (23): u' = a v' (lower triangular a), scaled by s_b */
      double up[3];
      up[0] = a[0] * v[0];
      up[1] = a[1] * v[0] + a[2] * v[1];
      up[2] = a[3] * v[0] + a[4] * v[1] + a[5] * v[2];
      for (int a3 = 0; a3 < 3; ++a3) {
        const size_t o = ((size_t)a3 * ny + y) * nz + z;
        uin[o] = s.u_rans[a3 * ny + y] + sb * up[a3]; /* Eq. (22) */
        if (fluct) fluct[o] = up[a3];
      }
      /* Sec. III.A: |u_in . n| < 0.3 c_s */
      if (!(std::fabs(uin[((size_t)0 * ny + y) * nz + z]) < 0.3 * std::sqrt(CS2))) st = OR_ERR_MACH;
    }
  }
  return st;
}

/* ---- state access ---- */
struct Ctx {
  const oracle_cfg* cfg;
  const double* f;     /* [19][nx][ny][nz] post-collision state s_n */
  const double* hist;  /* [5][ny][nz] outlet history (post-boundary f at x = nx-1, c_x < 0) */
  const double* uin;   /* [3][ny][nz] inlet velocity at t_{n+1} */
  size_t N;
  int nx, ny, nz;
  const double* line = nullptr; /* [2][nx] signed line u_tau of the wall lines (R23), or NULL */
  size_t at(int i, int x, int y, int z) const { return (size_t)i * N + ((size_t)x * ny + y) * nz + z; }
};

const int OUT5[5] = {1, 5, 8, 11, 15}; /* directions with c_x < 0, outlet history order */

/*
 * Sec. II.A, Eq. (3): pull streaming with the wall rules (Sec. II.C, IV.A).
 * Flat index of the post-collision value that population i of node (x, y, z)
 * takes, or -1 when there is none (outside the x range of an open channel).
 */
long long pull_src(const Ctx& c, int i, int x, int y, int z) {
  const oracle_cfg& cf = *c.cfg;
  const Tables& t = T();
  int xs = x - C[i][0], ys = y - C[i][1];
  int zs = ((z - C[i][2]) % c.nz + c.nz) % c.nz; /* periodic span */
  if (cf.xbc == 0) xs = (xs % c.nx + c.nx) % c.nx;
  if (ys < 0 || ys >= c.ny) {
    if (cf.ywall == 0) {
      ys = (ys % c.ny + c.ny) % c.ny;
    } else if (cf.ywall == 1) { /* halfway bounce-back: the population that left towards the wall */
      return (long long)c.at(t.opp[i], x, y, z);
    } else { /* specular reflection at the halfway wall */
      if (xs < 0 || xs >= c.nx) return -1;
      return (long long)c.at(t.refl_y[i], xs, y, zs);
    }
  }
  if (xs < 0 || xs >= c.nx) return -1;
  return (long long)c.at(i, xs, ys, zs);
}

bool pulled(const Ctx& c, int i, int x, int y, int z, double* v) {
  const long long k = pull_src(c, i, x, y, z);
  if (k < 0) return false;
  *v = c.f[k];
  return true;
}

/*
 * Inputs of one node's boundary rules, gathered from the state: the pulled
 * populations, and at the outlet the history plane and the pulled values of
 * the node upstream; at the inlet the prescribed velocity.
 */
struct NodeIn {
  double pv[19];
  double hist[5], up[5], uin[3];
  bool outlet, inlet;
};

void gather_inputs(const Ctx& c, int x, int y, int z, NodeIn* in) {
  const oracle_cfg& cf = *c.cfg;
  for (int i = 0; i < 19; ++i) {
    double v = 0.0;
    in->pv[i] = pulled(c, i, x, y, z, &v) ? v : 0.0;
  }
  in->outlet = (cf.xbc == 1 && x == c.nx - 1);
  in->inlet = (cf.xbc == 1 && x == 0);
  for (int k = 0; k < 5; ++k) in->hist[k] = in->up[k] = 0.0;
  for (int a = 0; a < 3; ++a) in->uin[a] = 0.0;
  if (in->outlet)
    for (int k = 0; k < 5; ++k) {
      double up = 0.0;
      pulled(c, OUT5[k], x - 1, y, z, &up);
      in->up[k] = up;
      in->hist[k] = c.hist[((size_t)k * c.ny + y) * c.nz + z];
    }
  if (in->inlet)
    for (int a = 0; a < 3; ++a) in->uin[a] = c.uin[((size_t)a * c.ny + y) * c.nz + z];
}

/* Post-streaming, post-boundary populations of one node (Algorithm 1 inlet branch). */
template <class R>
void boundary_rules(const oracle_cfg& cf, bool outlet, bool inlet, const R pv[19], const R hist[5], const R up[5],
                    const R uin[3], R fo[19], R hist_new[5]) {
  for (int i = 0; i < 19; ++i) fo[i] = pv[i];
  if (outlet) { /* convective outlet (R13) */
    for (int k = 0; k < 5; ++k) {
      const int i = OUT5[k];
      fo[i] = (cf.outlet == 1) ? up[k] + 0.0 * hist[k] : (hist[k] + cf.u_conv * up[k]) / (1.0 + cf.u_conv);
      hist_new[k] = fo[i];
    }
  }
  if (inlet) { /* STG inlet, Algorithm 1 steps 6-7 */
    R out[19];
    inlet_regularize(fo, uin, out, (R*)nullptr);
    for (int i = 0; i < 19; ++i) fo[i] = out[i];
  }
}

void post_boundary(const Ctx& c, int x, int y, int z, double fo[19], double hist_new[5], bool* is_outlet) {
  NodeIn in;
  gather_inputs(c, x, y, z, &in);
  boundary_rules(*c.cfg, in.outlet, in.inlet, in.pv, in.hist, in.up, in.uin, fo, hist_new);
  *is_outlet = in.outlet;
}

template <class R>
void pre_force_velocity(const R f[19], R* rho, R u[3]) {
  R r = 0.0 * f[0], j[3] = {0.0 * f[0], 0.0 * f[0], 0.0 * f[0]};
  for (int i = 0; i < 19; ++i) {
    r = r + f[i];
    for (int a = 0; a < 3; ++a) j[a] = j[a] + f[i] * C[i][a];
  }
  *rho = r;
  for (int a = 0; a < 3; ++a) u[a] = j[a] / r;
}

bool is_wall_cell(const oracle_cfg& cf, int y) {
  return cf.wall_model == 1 && cf.ywall != 0 && (y == 0 || y == cf.ny - 1);
}

/*
 * Algorithm 1 steps 8-14 for one node from its post-boundary populations f
 * (and, in a first off-wall cell, those of the next row, f2): wall force,
 * F = rho g + F_w, collision.  out: post-collision populations; u_stat: the
 * force-corrected velocity.  Returns the wall solve's status.
 */
template <class R>
int node_core(const oracle_cfg& cf, int x, int y, const R f[19], const R f2[19], const R& cs_smag, R out[19],
              R u_stat[3], R* utau = nullptr, const R* line = nullptr) {
  R rho, uw[3];
  pre_force_velocity(f, &rho, uw);
  R F[3] = {rho * cf.g[0], rho * cf.g[1], rho * cf.g[2]}; /* R9 */
  int st = OR_OK;
  if (is_wall_cell(cf, y)) { /* Algorithm 1 steps 9-14 */
    const int top = (y == cf.ny - 1);
    R rho2, u2[3];
    pre_force_velocity(f2, &rho2, u2);
    R Fw[3];
    st = wall_force(cf, rho, uw, u2, top, Fw, utau, line);
    for (int a = 0; a < 3; ++a) F[a] = F[a] + Fw[a];
  }
  R tau;
  collide(cf, tau0_at(cf, x), f, F, cs_smag, out, &tau, u_stat);
  return st;
}

int wall_neighbour_row(const oracle_cfg& cf, int y) { return (y == cf.ny - 1) ? y - 1 : y + 1; }

/* One node of Algorithm 1: boundaries, wall branch, stream-collide.  Returns
   status; *utau (optional) receives the wall law's u_tau (0 off the wall rows). */
int node_update(const Ctx& c, int x, int y, int z, double out[19], double hist_new[5], bool* is_outlet,
                double u_stat[3], double* utau = nullptr) {
  const oracle_cfg& cf = *c.cfg;
  double f[19], f2[19];
  post_boundary(c, x, y, z, f, hist_new, is_outlet);
  if (is_wall_cell(cf, y)) {
    double h2[5];
    bool o2;
    post_boundary(c, x, wall_neighbour_row(cf, y), z, f2, h2, &o2);
  } else {
    for (int i = 0; i < 19; ++i) f2[i] = 0.0;
  }
  if (utau) *utau = 0.0;
  const double* line = (c.line && is_wall_cell(cf, y)) ? &c.line[(y == cf.ny - 1 ? cf.nx : 0) + x] : nullptr;
  int st = node_core(cf, x, y, f, f2, cf.cs_smag, out, u_stat, utau, line);
  double rho = 0.0;
  for (int i = 0; i < 19; ++i) rho += f[i];
  if (!(rho > 0.0) || !std::isfinite(rho)) st = OR_ERR_NONFINITE;
  for (int i = 0; i < 19; ++i)
    if (!std::isfinite(out[i])) st = OR_ERR_NONFINITE;
  return st;
}

bool line_mode(const oracle_cfg& cf) { return cf.wall_avg == 1 && cf.wall_model == 1 && cf.ywall != 0; }

/* u_hat of the first off-wall cell (x, wall w, z) of a step (Eq. (18)-(19)). */
double cell_uhat(const Ctx& c, int x, int w, int z) {
  const oracle_cfg& cf = *c.cfg;
  const int y = w ? cf.ny - 1 : 0;
  double f[19], f2[19], h[5], rho, rho2, uw[3], u2[3];
  bool o;
  post_boundary(c, x, y, z, f, h, &o);
  post_boundary(c, x, wall_neighbour_row(cf, y), z, f2, h, &o);
  pre_force_velocity(f, &rho, uw);
  pre_force_velocity(f2, &rho2, u2);
  return wall_uhat(uw, u2, w);
}

/* Reading R23: the z-mean of u_hat of every wall line of a step, and its
   signed u_tau, line[w * nx + x]. */
int wall_lines(const Ctx& c, std::vector<double>& line) {
  const oracle_cfg& cf = *c.cfg;
  line.assign(2 * (size_t)cf.nx, 0.0);
  int st = OR_OK;
  for (int w = 0; w < 2; ++w)
    for (int x = 0; x < cf.nx; ++x) {
      double sum = 0.0;
      for (int z = 0; z < cf.nz; ++z) sum += cell_uhat(c, x, w, z);
      const double ubar = sum / (g_mutation == 15 ? cf.nz + 1 : cf.nz);
      const int s = line_utau(cf, ubar, &line[(size_t)w * cf.nx + x]);
      if (s != OR_OK) st = s;
    }
  return st;
}

bool cfg_ok(const oracle_cfg* cf) {
  if (!cf || cf->nx < 1 || cf->ny < 1 || cf->nz < 1) return false;
  if (cf->xbc == 1 && cf->nx < 3) return false;
  if (cf->wall_model == 1 && cf->ny < 3) return false;
  if (!(cf->tau0 > 0.5)) return false;
  if (cf->sponge_cells < 0 || cf->sponge_cells > cf->nx - 1) return false;
  if (cf->outlet != 0 && cf->outlet != 1) return false;
  if (cf->wall_law != 0 && cf->wall_law != 1) return false;
  if (cf->wall_avg != 0 && cf->wall_avg != 1) return false;
  if (cf->sponge_cells > 0 && (cf->xbc != 1 || !(cf->sponge_nu > 0.0))) return false;
  return true;
}

}  // namespace

extern "C" {

/* ---------------- small building blocks, exported for the pins ---------------- */

void oracle_set_mutation(int k) { g_mutation = k; }

void oracle_tables(int32_t* c /*[19][3]*/, double* w /*[19]*/, double* M /*[19][19]*/, double* Minv,
                   int32_t* opp, int32_t* refl) {
  const Tables& t = T();
  for (int i = 0; i < 19; ++i) {
    for (int a = 0; a < 3; ++a) c[i * 3 + a] = C[i][a];
    w[i] = t.W[i];
    opp[i] = t.opp[i];
    refl[i] = t.refl_y[i];
    for (int k = 0; k < 19; ++k) {
      M[i * 19 + k] = t.M[i][k];
      Minv[i * 19 + k] = t.Minv[i][k];
    }
  }
}

void oracle_feq(double rho, const double* u, double* out) { feq_poly(rho, u, out); }
void oracle_meq(double rho, const double* u, double* out) { meq_moments(rho, u, out); }
void oracle_guo(const double* u, const double* F, double* out) { guo_populations(u, F, out); }

void oracle_collide_node(const oracle_cfg* cfg, const double* f, const double* F, double* out, double* tau_eff,
                         double* u) {
  collide(*cfg, cfg->tau0, f, F, cfg->cs_smag, out, tau_eff, u);
}

double oracle_tau_eff(double Qhalf, double rho, double tau0, double cs_smag) {
  return tau_eff_of(Qhalf, rho, tau0, cs_smag);
}

double oracle_uplus(double yp, double kappa, double B) { return uplus(yp, kappa, B); }
double oracle_duplus(double yp, double kappa, double B) { return duplus(yp, kappa, B); }
double oracle_uplus_musker(double yp) { return uplus_musker(yp); }
double oracle_duplus_musker(double yp) { return duplus_musker(yp); }

int oracle_utau(const oracle_cfg* cfg, double uhat_abs, double* ut) {
  const double nu0 = (cfg->tau0 - 0.5) * CS2;
  return solve_utau(uhat_abs, cfg->y_wall, nu0, *cfg, ut);
}

int oracle_wall_force(const oracle_cfg* cfg, double rho_w, const double* uw, const double* u2, int top,
                      double* F, double* utau) {
  return wall_force(*cfg, rho_w, uw, u2, top, F, utau);
}

void oracle_inlet_node(const double* f, const double* uin, double* out, double* rho_in) {
  inlet_regularize(f, uin, out, rho_in);
}

void oracle_cholesky(const double* R6, double* a) { cholesky(R6, a); }

int oracle_stg_plane(const oracle_cfg* cfg, const oracle_stg* s, double t, double* uin, double* fluct) {
  if (!cfg_ok(cfg) || !s) return OR_ERR_ARG;
  return stg_plane(*cfg, *s, t, uin, fluct);
}

int oracle_stg_weights(const oracle_cfg* cfg, const oracle_stg* s, int32_t y, double* q) {
  if (!cfg_ok(cfg) || !s || y < 0 || y >= cfg->ny) return OR_ERR_ARG;
  return stg_weights(*cfg, *s, y, q);
}

/* Reichardt inflow U(y) = u_tau u+(d u_tau / nu0), d the distance to the nearer wall. */
void oracle_reichardt_inflow(const oracle_cfg* cfg, double u_tau, double* u_rans /*[3][ny]*/) {
  const int ny = cfg->ny;
  const double nu0 = (cfg->tau0 - 0.5) * CS2;
  for (int y = 0; y < ny; ++y) {
    const double d = std::fmin(y + 0.5, ny - y - 0.5);
    u_rans[y] = u_tau * uplus(d * u_tau / nu0, cfg->kappa, cfg->b_reich);
    u_rans[ny + y] = 0.0;
    u_rans[2 * ny + y] = 0.0;
  }
}

/* ---------------- whole-lattice operations ---------------- */

/* f_i = f_eq_i(rho, u) + eps w_i pert_i; outlet history from the same state. */
int oracle_init(const oracle_cfg* cfg, const double* rho /*[N] or NULL*/, const double* u /*[3][N]*/,
                const double* pert /*[19][N] or NULL*/, double eps, double* f, double* hist) {
  if (!cfg_ok(cfg)) return OR_ERR_ARG;
  const Tables& t = T();
  const int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
  const size_t N = (size_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
  for (long long n = 0; n < (long long)N; ++n) {
    double uu[3] = {u[n], u[N + n], u[2 * N + n]}, fe[19];
    const double r = rho ? rho[n] : 1.0;
    feq_poly(r, uu, fe);
    for (int i = 0; i < 19; ++i) f[(size_t)i * N + n] = fe[i] + (pert ? eps * t.W[i] * pert[(size_t)i * N + n] : 0.0);
  }
  if (hist)
    for (int k = 0; k < 5; ++k)
      for (int y = 0; y < ny; ++y)
        for (int z = 0; z < nz; ++z)
          hist[((size_t)k * ny + y) * nz + z] = f[(size_t)OUT5[k] * N + ((size_t)(nx - 1) * ny + y) * nz + z];
  return OR_OK;
}

/* Streaming with wall rules only; unset populations (outside the x range) are -1. */
int oracle_stream_only(const oracle_cfg* cfg, const double* fin, double* fout) {
  if (!cfg_ok(cfg)) return OR_ERR_ARG;
  Ctx c{cfg, fin, nullptr, nullptr, (size_t)cfg->nx * cfg->ny * cfg->nz, cfg->nx, cfg->ny, cfg->nz};
#pragma omp parallel for collapse(2) schedule(static)
  for (int x = 0; x < c.nx; ++x)
    for (int y = 0; y < c.ny; ++y)
      for (int z = 0; z < c.nz; ++z)
        for (int i = 0; i < 19; ++i) {
          double v;
          fout[c.at(i, x, y, z)] = pulled(c, i, x, y, z, &v) ? v : -1.0;
        }
  return OR_OK;
}

/*
 * One full step s_n -> s_{n+1} (Algorithm 1) with the inlet velocity plane
 * given (uin [3][ny][nz], used when xbc = 1).  hist_in/hist_out: outlet
 * history (may not alias).  Statistics: for each x in planes[],
 * acc[p][y][0..8] += sum over z of (u, v, w, uu, vv, ww, uv, uw, vw) with the
 * force-corrected velocity.
 */
int step_core(const oracle_cfg* cfg, const double* uin, const double* fin, double* fout, const double* hist_in,
              double* hist_out, const int32_t* planes, int32_t n_planes, double* acc, double* wall_acc) {
  const int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
  Ctx c{cfg, fin, hist_in, uin, (size_t)nx * ny * nz, nx, ny, nz};
  std::vector<int> plane_of(nx, -1);
  for (int p = 0; p < n_planes; ++p)
    if (planes[p] >= 0 && planes[p] < nx) plane_of[planes[p]] = p;
  int st_err = OR_OK;
  std::vector<double> line;
  if (line_mode(*cfg)) {
    st_err = wall_lines(c, line);
    c.line = line.data();
  }
#pragma omp parallel for collapse(2) schedule(static)
  for (int x = 0; x < nx; ++x)
    for (int y = 0; y < ny; ++y) {
      double sums[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, ut_sum = 0.0;
      int st_local = OR_OK;
      for (int z = 0; z < nz; ++z) {
        double out[19], hn[5], u[3], ut;
        bool is_out;
        int st = node_update(c, x, y, z, out, hn, &is_out, u, &ut);
        ut_sum += ut;
        if (st != OR_OK) st_local = st;
        for (int i = 0; i < 19; ++i) fout[c.at(i, x, y, z)] = out[i];
        if (is_out)
          for (int k = 0; k < 5; ++k) hist_out[((size_t)k * ny + y) * nz + z] = hn[k];
        sums[0] += u[0];
        sums[1] += u[1];
        sums[2] += u[2];
        sums[3] += u[0] * u[0];
        sums[4] += u[1] * u[1];
        sums[5] += u[2] * u[2];
        sums[6] += u[0] * u[1];
        sums[7] += u[0] * u[2];
        sums[8] += u[1] * u[2];
      }
      if (plane_of[x] >= 0 && acc)
        for (int k = 0; k < 9; ++k) acc[((size_t)plane_of[x] * ny + y) * 9 + k] += sums[k];
      /* wall statistics: sum over z of u_tau in the first off-wall rows [bottom, top][x] */
      if (wall_acc && is_wall_cell(*cfg, y)) wall_acc[(y == ny - 1 ? nx : 0) + x] += ut_sum;
      if (st_local != OR_OK) {
#pragma omp critical
        st_err = st_local;
      }
    }
  return st_err;
}

int oracle_step(const oracle_cfg* cfg, const oracle_stg* stg, double t_next, const double* fin, double* fout,
                const double* hist_in, double* hist_out, const int32_t* planes, int32_t n_planes, double* acc,
                double* wall_acc) {
  if (!cfg_ok(cfg) || !fin || !fout) return OR_ERR_ARG;
  if (cfg->xbc == 1 && (!stg || !hist_in || !hist_out)) return OR_ERR_ARG;
  std::vector<double> uin;
  int st_all = OR_OK;
  if (cfg->xbc == 1) {
    uin.resize((size_t)3 * cfg->ny * cfg->nz);
    st_all = stg_plane(*cfg, *stg, t_next, uin.data(), nullptr);
  }
  int st = step_core(cfg, uin.empty() ? nullptr : uin.data(), fin, fout, hist_in, hist_out, planes, n_planes, acc,
                     wall_acc);
  return st != OR_OK ? st : st_all;
}

/* The same step with the inlet velocity plane given instead of generated. */
int oracle_step_uin(const oracle_cfg* cfg, const double* uin, const double* fin, double* fout,
                    const double* hist_in, double* hist_out, const int32_t* planes, int32_t n_planes, double* acc) {
  if (!cfg_ok(cfg) || !fin || !fout) return OR_ERR_ARG;
  if (cfg->xbc == 1 && (!uin || !hist_in || !hist_out)) return OR_ERR_ARG;
  return step_core(cfg, uin, fin, fout, hist_in, hist_out, planes, n_planes, acc, nullptr);
}

/*
 * Discrete adjoint of one step s_n -> s_{n+1} (the transpose of the step's
 * linearisation).  Given the loss sensitivities to the step's outputs --
 * lam_next = dL/ds_{n+1} [19][N], eta_next = dL/dhist_{n+1} [5][ny][nz] and
 * the statistics weights coef [n_planes][ny][9] (dL/d of each accumulated sum
 * of this step, NULL when the step is not sampled) -- it returns
 * lam_prev = dL/ds_n, eta_prev = dL/dhist_n, g_uin = dL/du_in(t_next)
 * [3][ny][nz] (overwritten) and adds dL/dC_s to *g_cs and, with STG inputs,
 * dL/ds_b = sum over the bin's rows of g_uin . (a v') to g_amp[b].
 *
 * Method: every node's update is split into its boundary rules (pulled
 * populations, outlet history and upstream values, inlet velocity -> the
 * post-boundary populations) and its core (post-boundary populations of the
 * node and, in a first off-wall cell, of the next row, and C_s -> the new
 * populations and velocity).  The local Jacobians of both come from dual
 * numbers; pass 1 pulls the output sensitivities back to the post-boundary
 * populations of every node, pass 2 pulls those back through the boundary
 * rules and adds them to the source of every pulled value.
 */
int oracle_adjoint_step(const oracle_cfg* cfg, const oracle_stg* stg, double t_next, const double* uin_given,
                        const double* s_n, const double* hist_n, const double* lam_next, const double* eta_next,
                        const int32_t* planes, int32_t n_planes, const double* coef, double* lam_prev,
                        double* eta_prev, double* g_uin, double* g_cs, double* g_amp) {
  if (!cfg_ok(cfg) || !s_n || !lam_next || !lam_prev) return OR_ERR_ARG;
  const int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
  const bool open = cfg->xbc == 1;
  if (open && (!hist_n || !eta_next || !eta_prev || (!uin_given && !stg))) return OR_ERR_ARG;
  if (g_amp && !stg) return OR_ERR_ARG;
  const size_t N = (size_t)nx * ny * nz, P = (size_t)ny * nz;
  std::vector<double> uin, fluct;
  int st_all = OR_OK;
  if (open) {
    uin.resize(3 * P);
    if (stg) {
      fluct.resize(3 * P);
      st_all = stg_plane(*cfg, *stg, t_next, uin.data(), fluct.data());
    }
    if (uin_given) std::memcpy(uin.data(), uin_given, 3 * P * sizeof(double));
  }
  Ctx c{cfg, s_n, hist_n, open ? uin.data() : nullptr, N, nx, ny, nz};
  std::vector<int> plane_of(nx, -1);
  for (int p = 0; p < n_planes; ++p)
    if (planes && planes[p] >= 0 && planes[p] < nx) plane_of[planes[p]] = p;
  int st_err = OR_OK;
  const bool lines = line_mode(*cfg);
  std::vector<double> line, gline(lines ? 2 * (size_t)nx : 0, 0.0);
  if (lines) {
    st_err = wall_lines(c, line);
    c.line = line.data();
  }

  /* pass 1: dL/d(post-boundary populations) of every node, dL/dC_s and, with
     line-averaged u_tau, dL/d(line u_tau) (slot 39) */
  typedef Dual<40> D1;
  std::vector<double> G(19 * N, 0.0), gcs_x(nx, 0.0);
#pragma omp parallel for schedule(static)
  for (int x = 0; x < nx; ++x) {
    for (int y = 0; y < ny; ++y)
      for (int z = 0; z < nz; ++z) {
        double fo[19], f2[19], hn[5];
        bool is_out;
        post_boundary(c, x, y, z, fo, hn, &is_out);
        const bool wall = is_wall_cell(*cfg, y);
        const int y2 = wall ? wall_neighbour_row(*cfg, y) : y;
        if (wall) {
          double h2[5];
          bool o2;
          post_boundary(c, x, y2, z, f2, h2, &o2);
        }
        D1 fd[19], f2d[19], out[19], u[3];
        for (int i = 0; i < 19; ++i) {
          fd[i] = D1::seed(fo[i], i);
          f2d[i] = wall ? D1::seed(f2[i], 19 + i) : D1(0.0);
        }
        const D1 cs = D1::seed(cfg->cs_smag, 38);
        const size_t li = (size_t)(y == ny - 1 ? nx : 0) + x;
        const D1 ld = (lines && wall) ? D1::seed(line[li], 39) : D1(0.0);
        int st = node_core(*cfg, x, y, fd, f2d, cs, out, u, (D1*)nullptr, (lines && wall) ? &ld : nullptr);
        if (st != OR_OK) {
#pragma omp critical
          st_err = st;
        }
        D1 J(0.0);
        for (int i = 0; i < 19; ++i) J = J + lam_next[c.at(i, x, y, z)] * out[i];
        if (coef && plane_of[x] >= 0) {
          const double* A = coef + ((size_t)plane_of[x] * ny + y) * 9;
          const D1 prod[9] = {u[0], u[1], u[2], u[0] * u[0], u[1] * u[1], u[2] * u[2],
                              u[0] * u[1], u[0] * u[2], u[1] * u[2]};
          for (int k = 0; k < 9; ++k) J = J + A[k] * prod[k];
        }
        for (int i = 0; i < 19; ++i) G[c.at(i, x, y, z)] += J.d[i];
        if (wall && g_mutation != 8)
          for (int i = 0; i < 19; ++i) G[c.at(i, x, y2, z)] += J.d[19 + i];
        gcs_x[x] += J.d[38];
        if (lines && wall) gline[li] += J.d[39];
        if (is_out && g_mutation != 9)
          for (int k = 0; k < 5; ++k) G[c.at(OUT5[k], x, y, z)] += eta_next[(size_t)k * P + (size_t)y * nz + z];
      }
  }
  if (g_cs)
    for (int x = 0; x < nx; ++x) *g_cs += gcs_x[x];

  /* pass 1b (R23): each line's u_tau depends on the mean u_hat of its cells,
     so dL/d(line u_tau) goes back to the post-boundary populations of every
     first and second off-wall cell of the line */
  if (lines) {
    typedef Dual<38> D3;
    typedef Dual<1> D0;
    for (int w = 0; w < 2; ++w)
#pragma omp parallel for schedule(static)
      for (int x = 0; x < nx; ++x) {
        const double gl = gline[(size_t)w * nx + x];
        if (gl == 0.0) continue;
        const int y = w ? ny - 1 : 0, y2 = wall_neighbour_row(*cfg, y);
        double sum = 0.0;
        for (int z = 0; z < nz; ++z) sum += cell_uhat(c, x, w, z);
        D0 l;
        line_utau(*cfg, D0::seed(sum / nz, 0), &l);
        const double gu = gl * l.d[0] / nz; /* dL/du_hat of each cell */
        for (int z = 0; z < nz; ++z) {
          double f[19], f2[19], h[5];
          bool o;
          post_boundary(c, x, y, z, f, h, &o);
          post_boundary(c, x, y2, z, f2, h, &o);
          D3 fd[19], f2d[19], rho, rho2, uw[3], u2[3];
          for (int i = 0; i < 19; ++i) {
            fd[i] = D3::seed(f[i], i);
            f2d[i] = D3::seed(f2[i], 19 + i);
          }
          pre_force_velocity(fd, &rho, uw);
          pre_force_velocity(f2d, &rho2, u2);
          const D3 uh = wall_uhat(uw, u2, w);
          for (int i = 0; i < 19; ++i) {
            G[c.at(i, x, y, z)] += gu * uh.d[i];
            if (g_mutation != 16) G[c.at(i, x, y2, z)] += gu * uh.d[19 + i];
          }
        }
      }
  }

  /* pass 2: through the boundary rules to the pulled sources, history and inlet velocity */
  typedef Dual<32> D2;
  std::memset(lam_prev, 0, 19 * N * sizeof(double));
  if (open) std::memset(eta_prev, 0, 5 * P * sizeof(double));
  std::vector<double> gu(open ? 3 * P : 0, 0.0);
  for (int x = 0; x < nx; ++x)
    for (int y = 0; y < ny; ++y)
      for (int z = 0; z < nz; ++z) {
        NodeIn in;
        gather_inputs(c, x, y, z, &in);
        D2 pv[19], hist[5], up[5], ui[3], fo[19], hn[5];
        for (int i = 0; i < 19; ++i) pv[i] = D2::seed(in.pv[i], i);
        for (int k = 0; k < 5; ++k) {
          hist[k] = D2::seed(in.hist[k], 19 + k);
          up[k] = D2::seed(in.up[k], 24 + k);
        }
        for (int a = 0; a < 3; ++a) ui[a] = D2::seed(in.uin[a], 29 + a);
        boundary_rules(*cfg, in.outlet, in.inlet, pv, hist, up, ui, fo, hn);
        D2 J(0.0);
        for (int i = 0; i < 19; ++i) J = J + G[c.at(i, x, y, z)] * fo[i];
        for (int i = 0; i < 19; ++i) {
          const long long k = pull_src(c, i, x, y, z);
          if (k >= 0) lam_prev[k] += J.d[i];
        }
        if (in.outlet)
          for (int k = 0; k < 5; ++k) {
            eta_prev[(size_t)k * P + (size_t)y * nz + z] += J.d[19 + k];
            const long long s = pull_src(c, OUT5[k], x - 1, y, z);
            if (s >= 0 && g_mutation != 10) lam_prev[s] += J.d[24 + k];
          }
        if (in.inlet)
          for (int a = 0; a < 3; ++a) gu[(size_t)a * P + (size_t)y * nz + z] += J.d[29 + a];
      }
  if (open && g_uin) std::memcpy(g_uin, gu.data(), 3 * P * sizeof(double));
  if (open && g_amp && !fluct.empty())
    for (int y = 0; y < ny; ++y)
      for (int z = 0; z < nz; ++z)
        for (int a = 0; a < 3; ++a)
          g_amp[stg->bin_of_y[y]] += gu[(size_t)a * P + (size_t)y * nz + z] * fluct[(size_t)a * P + (size_t)y * nz + z];
  return st_err != OR_OK ? st_err : st_all;
}

/*
 * The same update evaluated at a list of nodes only (for comparisons at full
 * lattice sizes): out[19][n_nodes], u_out[3][n_nodes] (force-corrected u).
 */
/* Reading R23, for the pins: the signed line u_tau line[2][nx] and the u_hat
   of every first off-wall cell uhat[2][nx][nz] of the step s_n -> s_{n+1}. */
int oracle_wall_lines(const oracle_cfg* cfg, const oracle_stg* stg, double t_next, const double* fin,
                      const double* hist_in, double* line, double* uhat) {
  if (!cfg_ok(cfg) || !fin || cfg->wall_model != 1 || cfg->ywall == 0) return OR_ERR_ARG;
  if (cfg->xbc == 1 && (!stg || !hist_in)) return OR_ERR_ARG;
  const int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
  std::vector<double> uin;
  if (cfg->xbc == 1) {
    uin.resize((size_t)3 * ny * nz);
    stg_plane(*cfg, *stg, t_next, uin.data(), nullptr);
  }
  Ctx c{cfg, fin, hist_in, uin.empty() ? nullptr : uin.data(), (size_t)nx * ny * nz, nx, ny, nz};
  std::vector<double> l;
  const int st = wall_lines(c, l);
  std::memcpy(line, l.data(), l.size() * sizeof(double));
  for (int w = 0; w < 2; ++w)
    for (int x = 0; x < nx; ++x)
      for (int z = 0; z < nz; ++z) uhat[((size_t)w * nx + x) * nz + z] = cell_uhat(c, x, w, z);
  return st;
}

int oracle_step_nodes(const oracle_cfg* cfg, const oracle_stg* stg, double t_next, const double* fin,
                      const double* hist_in, int64_t n_nodes, const int64_t* nodes, double* out, double* u_out) {
  if (!cfg_ok(cfg) || !fin) return OR_ERR_ARG;
  if (cfg->xbc == 1 && (!stg || !hist_in)) return OR_ERR_ARG;
  const int nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
  std::vector<double> uin;
  int st_all = OR_OK;
  if (cfg->xbc == 1) {
    uin.resize((size_t)3 * ny * nz);
    st_all = stg_plane(*cfg, *stg, t_next, uin.data(), nullptr);
  }
  Ctx c{cfg, fin, hist_in, uin.empty() ? nullptr : uin.data(), (size_t)nx * ny * nz, nx, ny, nz};
  int st_err = OR_OK;
  std::vector<double> line;
  if (line_mode(*cfg)) {
    st_err = wall_lines(c, line);
    c.line = line.data();
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (long long k = 0; k < (long long)n_nodes; ++k) {
    const int64_t n = nodes[k];
    const int z = (int)(n % nz), y = (int)((n / nz) % ny), x = (int)(n / ((int64_t)nz * ny));
    double o[19], hn[5], u[3];
    bool is_out;
    int st = node_update(c, x, y, z, o, hn, &is_out, u);
    if (st != OR_OK) {
#pragma omp critical
      st_err = st;
    }
    for (int i = 0; i < 19; ++i) out[(size_t)i * n_nodes + k] = o[i];
    if (u_out)
      for (int a = 0; a < 3; ++a) u_out[(size_t)a * n_nodes + k] = u[a];
  }
  return st_err != OR_OK ? st_err : st_all;
}

/* Macroscopic fields without force: rho = sum f, u = sum f c / rho. */
void oracle_macro(const oracle_cfg* cfg, const double* f, double* rho, double* u) {
  const size_t N = (size_t)cfg->nx * cfg->ny * cfg->nz;
#pragma omp parallel for schedule(static)
  for (long long n = 0; n < (long long)N; ++n) {
    double fl[19], r, uu[3];
    for (int i = 0; i < 19; ++i) fl[i] = f[(size_t)i * N + n];
    pre_force_velocity(fl, &r, uu);
    rho[n] = r;
    for (int a = 0; a < 3; ++a) u[(size_t)a * N + n] = uu[a];
  }
}

}  // extern "C"

extern "C" {
/* nsteps steps from t0 (STG time t0 + n + 1 for step n); f and hist updated in place. */
int oracle_run(const oracle_cfg* cfg, const oracle_stg* stg, double t0, int32_t nsteps, double* f, double* hist,
               const int32_t* planes, int32_t n_planes, double* acc, double* wall_acc) {
  if (!cfg_ok(cfg) || !f) return OR_ERR_ARG;
  const size_t N = (size_t)cfg->nx * cfg->ny * cfg->nz;
  std::vector<double> tmp(19 * N), htmp(hist ? (size_t)5 * cfg->ny * cfg->nz : 0);
  int st_all = OR_OK;
  for (int n = 0; n < nsteps; ++n) {
    if (hist) std::memcpy(htmp.data(), hist, htmp.size() * sizeof(double));
    int st = oracle_step(cfg, stg, t0 + n + 1, f, tmp.data(), hist, hist ? htmp.data() : nullptr, planes,
                         n_planes, acc, wall_acc);
    if (st != OR_OK) st_all = st;
    std::memcpy(f, tmp.data(), 19 * N * sizeof(double));
    if (hist) std::memcpy(hist, htmp.data(), htmp.size() * sizeof(double));
  }
  return st_all;
}
}  // extern "C"

#ifdef _OPENMP
#include <omp.h>
#endif
extern "C" int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the following parallel loops (n >= 1); no effect without OpenMP. */
extern "C" void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
