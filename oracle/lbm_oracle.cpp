// FP64 reference implementation of the VANSE Carreau-Yasuda lattice Boltzmann
// step (D3Q19).  TEST INFRASTRUCTURE ONLY: it is used by the test-suite, the
// smoke check and the CPU-baseline timing; the product path never calls it.
//
// Every function follows the paper's method section in the paper's order:
//   moments and pressure ........ method section, definitions of rho, u, p
//   explicit velocity ........... method section, closed form of u with C0, C1
//   drag and permeability ....... model section, Darcy/Forchheimer force and
//                                 the Kozeny-Carman relation
//   collide and stream .......... method section, update f + Omega^phi +
//                                 dt*Omega^f + Omega^SRT and the four
//                                 definitions that follow it
//   relaxation rate ............. method section, omega from mu; Carreau-Yasuda
//                                 law (model section, eq. carreau); semi-explicit
//                                 shear rate from the corrected second moment Pi
//   boundaries .................. simulation section: halfway bounce-back walls,
//                                 Zou-He velocity inflow, Poiseuille profile,
//                                 extrapolation outflow.
// Where the paper is silent the reading is stated at the point of use.
//
// Lattice units throughout: dx = dt = 1, c_s^2 = 1/3.  State = pre-collision,
// post-streaming populations f_i at the fluid cells (cells in ascending box
// index order, box index = x + nx*(y + ny*z)), plus the relaxation rate of the
// previous step at every fluid cell.  Populations that arrive from outside an
// open (inflow/outflow) face are unknown; the state holds 0 there and the
// Zou-He fill of the next step replaces them.  An extrapolation outflow instead
// keeps its unknowns in the state (see extrapolate_outlet).
//
// The scalar type is a template parameter so that forward-mode dual numbers give
// exact derivatives of the discrete map (used by the gradient checks).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

// ---------------------------------------------------------------------------
// Velocity set, chosen at compile time (ORACLE_Q = 19 or 27; the paper's
// method section uses D3Q27).  D3Q19: rest (1/3), 6 axis neighbours (1/18),
// 12 edge neighbours (1/36).  D3Q27: rest (8/27), axis (2/27), edges (1/54),
// 8 corners (1/216).  Each odd-numbered moving direction is followed by its
// opposite; the first 19 directions are the same in both sets.
// ---------------------------------------------------------------------------
#ifndef ORACLE_Q
#define ORACLE_Q 19
#endif
const int Q = ORACLE_Q;
const int CV[27][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};
#if ORACLE_Q == 19
const double WT[Q] = {1.0 / 3.0,
                      1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                      1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                      1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
#elif ORACLE_Q == 27
const double WT[Q] = {8.0 / 27.0,
                      2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0,
                      1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0,
                      1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0,
                      1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0,
                      1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0};
#else
#error "ORACLE_Q must be 19 or 27"
#endif
const double CS2 = 1.0 / 3.0;

int opposite(int i) {
  for (int j = 0; j < Q; ++j)
    if (CV[j][0] == -CV[i][0] && CV[j][1] == -CV[i][1] && CV[j][2] == -CV[i][2]) return j;
  return -1;
}

// ---------------------------------------------------------------------------
// Forward-mode dual numbers with N derivative components.
// ---------------------------------------------------------------------------
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0) { for (int k = 0; k < N; ++k) d[k] = 0; }
  Dual(double x) : v(x) { for (int k = 0; k < N; ++k) d[k] = 0; }
};
template <int N> Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v + b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v - b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a) { Dual<N> r; r.v = -a.v; for (int k = 0; k < N; ++k) r.d[k] = -a.d[k]; return r; }
template <int N> Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v * b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
template <int N> Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v / b.v; for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v; return r; }
template <int N> Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> Dual<N> operator*(const Dual<N>& a, double b) { Dual<N> r; r.v = a.v * b; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b; return r; }
template <int N> Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N> Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }

double val(double x) { return x; }
template <int N> double val(const Dual<N>& x) { return x.v; }

double Sqrt(double x) { return std::sqrt(x); }
template <int N> Dual<N> Sqrt(const Dual<N>& x) {
  Dual<N> r; r.v = std::sqrt(x.v);
  // derivative taken as 0 at x = 0 (non-smooth point convention)
  double s = (x.v > 0) ? 0.5 / r.v : 0.0;
  for (int k = 0; k < N; ++k) r.d[k] = s * x.d[k];
  return r;
}
// x^p for x >= 0 and a constant exponent p; derivative 0 at x = 0.
double Pow(double x, double p) { return (x > 0) ? std::pow(x, p) : (p == 0 ? 1.0 : 0.0); }
template <int N> Dual<N> Pow(const Dual<N>& x, double p) {
  Dual<N> r; r.v = Pow(x.v, p);
  double s = (x.v > 0) ? p * std::pow(x.v, p - 1.0) : 0.0;
  for (int k = 0; k < N; ++k) r.d[k] = s * x.d[k];
  return r;
}

}  // namespace

// ---------------------------------------------------------------------------
// Case description (C ABI for the Python test harness).
// ---------------------------------------------------------------------------
extern "C" {
typedef struct {
  int nx, ny, nz;
  int periodic[3];
  const uint8_t* solid;        // nx*ny*nz, 1 = solid
  const double* phi;           // nx*ny*nz, porosity in (0, 1] on fluid
  const uint8_t* sac;          // nx*ny*nz or NULL: objective region
  int inlet, outlet;           // velocity inflow at x = 0; outflow at x = nx-1: 1 density, 2 extrapolation
  const double* inlet_shape;   // ny*nz (index y + ny*z): u_x/amplitude on the x = 0 face
  double a0, a1, period;       // amplitude(t) = a0 (1 + a1 sin(2 pi t / period))
  double rho_out;
  double nu0, nu_inf, lam, n, a;     // Carreau-Yasuda (kinematic, lattice units)
  double nu_d, kc, d;                // Darcy viscosity, Kozeny-Carman constant, grain size
  int forchheimer;                   // 0: C_F = 0; 1: Ergun C_F = 1.75/sqrt(150 phi^3)
  double g[3];                       // body force per unit mass
  int ramp;                          // pre-run length R (0: none)
  const double* wave_table;          // NULL: sine waveform; else samples of one period
  int table_len;
  double aniso[6];                   // permeability shape M (xx yy zz xy xz yz); all 0: isotropic
  int aniso_iters;                   // fixed-point iterations of the anisotropic velocity
} oracle_case;
}

namespace {

// ---------------------------------------------------------------------------
// Anisotropic permeability (the Remark of the method section).  Reading: the
// paper leaves open how K varies; here K(x) = k(phi(x)) M with k the
// Kozeny-Carman permeability and M a fixed symmetric positive definite shape,
// so K^-1 = (1/k) M^-1 and K^-1/2 = (1/k)^1/2 M^-1/2.  M = 0 means isotropic.
// M^-1 and M^-1/2 come from the eigen-decomposition M = V diag(l) V^T by
// cyclic Jacobi rotations.
// ---------------------------------------------------------------------------
struct Shape {
  bool on = false;
  double Minv[3][3], Mhi[3][3];
};

Shape shape_of(const oracle_case& c) {
  Shape S;
  const double* a = c.aniso;
  S.on = false;
  for (int k = 0; k < 6; ++k) S.on = S.on || a[k] != 0.0;
  if (!S.on) return S;
  double A[3][3] = {{a[0], a[3], a[4]}, {a[3], a[1], a[5]}, {a[4], a[5], a[2]}};
  double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = std::fabs(A[0][1]) + std::fabs(A[0][2]) + std::fabs(A[1][2]);
    if (off < 1e-300) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        // rotation angle that annihilates A[p][q]
        const double th = 0.5 * std::atan2(2.0 * A[p][q], A[q][q] - A[p][p]);
        const double cs = std::cos(th), sn = std::sin(th);
        for (int k = 0; k < 3; ++k) {  // A <- A J
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = cs * akp - sn * akq;
          A[k][q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < 3; ++k) {  // A <- J^T A
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = cs * apk - sn * aqk;
          A[q][k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < 3; ++k) {  // V <- V J
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = cs * vkp - sn * vkq;
          V[k][q] = sn * vkp + cs * vkq;
        }
      }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s1 = 0.0, s2 = 0.0;
      for (int k = 0; k < 3; ++k) {
        s1 += V[i][k] * V[j][k] / A[k][k];
        s2 += V[i][k] * V[j][k] / std::sqrt(A[k][k]);
      }
      S.Minv[i][j] = s1;
      S.Mhi[i][j] = s2;
    }
  return S;
}

// Solve X u = v for a 3x3 matrix X (Cramer's rule).
template <class T>
void solve3(const T X[3][3], const T v[3], T u[3]) {
  const T c00 = X[1][1] * X[2][2] - X[1][2] * X[2][1];
  const T c01 = X[1][2] * X[2][0] - X[1][0] * X[2][2];
  const T c02 = X[1][0] * X[2][1] - X[1][1] * X[2][0];
  const T det = X[0][0] * c00 + X[0][1] * c01 + X[0][2] * c02;
  T Y[3][3];  // X with column j replaced by v, determinant by cofactors
  for (int j = 0; j < 3; ++j) {
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) Y[i][k] = k == j ? v[i] : X[i][k];
    const T d = Y[0][0] * (Y[1][1] * Y[2][2] - Y[1][2] * Y[2][1]) - Y[0][1] * (Y[1][0] * Y[2][2] - Y[1][2] * Y[2][0]) +
                Y[0][2] * (Y[1][0] * Y[2][1] - Y[1][1] * Y[2][0]);
    u[j] = d / det;
  }
}

const int NB_WALL = -1;  // halfway bounce-back
const int NB_OPEN = -2;  // leaves through an open face: dropped

struct Ctx {
  oracle_case c;
  std::vector<uint8_t> solid, sac;
  std::vector<double> phi_box, shape, wave;
  std::vector<int64_t> cells;          // fluid -> box index
  std::vector<int64_t> box2f;          // box -> fluid (or -1)
  std::vector<int> nbr;                // [Q][nf]: fluid index of x + c_i, or NB_WALL/NB_OPEN
  std::vector<int> xc, yc, zc;         // coordinates of fluid cells
  std::vector<uint8_t> kind;           // 0 interior, 1 inlet, 2 outlet
  Shape shape_m;                       // anisotropic permeability shape
  std::vector<double> nrm;             // [nf][3]: outer wall normal (0 off the wall)
  std::vector<uint8_t> wall;           // 1: the cell has a wall normal
  int64_t nf = 0;
  long nsac = 0;
  long nwss = 0;                       // objective-region cells on the wall
};

// Inflow waveform at time s of its period: the sine a0 (1 + a1 sin(2 pi s / T)),
// or the sampled period (sample k at s = k T / n), read by linear
// interpolation between neighbouring samples and repeated every T steps.
double waveform(const Ctx& C, double s) {
  const oracle_case& c = C.c;
  if (C.wave.empty()) {
    const double pi = 3.14159265358979323846;
    return c.a0 * (1.0 + c.a1 * std::sin(2.0 * pi * s / c.period));
  }
  const int n = (int)C.wave.size();
  double phase = s / c.period;
  phase -= std::floor(phase);
  const double pos = phase * n;
  int k = (int)pos;
  if (k >= n) k = n - 1;
  const int k1 = (k + 1) % n;
  return C.wave[k] + (pos - k) * (C.wave[k1] - C.wave[k]);
}

// Inflow amplitude at step t.  The simulation section starts from rest with a
// pre-run in which the inflow grows linearly to the waveform's starting value;
// the waveform runs from the end of the pre-run.
double amplitude(const Ctx& C, int t) {
  const int R = C.c.ramp;
  if (t < R) return ((double)t / (double)R) * waveform(C, 0.0);
  return waveform(C, (double)(t - R));
}

// Which fluid cell (or wall / open face) lies at x + c_i.
int classify(const Ctx& C, int x, int y, int z, int i) {
  const oracle_case& c = C.c;
  int p[3] = {x + CV[i][0], y + CV[i][1], z + CV[i][2]};
  const int dims[3] = {c.nx, c.ny, c.nz};
  bool out_wall = false, out_open = false;
  for (int a = 0; a < 3; ++a) {
    if (p[a] >= 0 && p[a] < dims[a]) continue;
    if (c.periodic[a]) { p[a] = (p[a] + dims[a]) % dims[a]; continue; }
    if (a == 0 && ((p[a] < 0 && c.inlet) || (p[a] >= dims[a] && c.outlet))) out_open = true;
    else out_wall = true;
  }
  if (out_wall) return NB_WALL;
  if (out_open) return NB_OPEN;
  int64_t b = p[0] + (int64_t)c.nx * (p[1] + (int64_t)c.ny * p[2]);
  int64_t f = C.box2f[b];
  return f < 0 ? NB_WALL : (int)f;
}

// ---------------------------------------------------------------------------
// Open-face fill (Zou-He).  Inflow on x = 0 with prescribed velocity u_in: the
// unknowns are the five populations with c_x = +1; density from mass and normal
// momentum, tangential momentum balanced by the transverse corrections N_y, N_z.
// Outflow on x = nx-1 with prescribed density and zero tangential velocity: the
// unknowns are the five populations with c_x = -1.
// ---------------------------------------------------------------------------
#if ORACLE_Q == 27
// D3Q27 (nine unknowns per face).  Reading: the closure of the D3Q19 version
// generalised with weight-proportional transverse corrections,
//   f_i = f_opp(i) + 2 w_i rho (c_i . u) / c_s^2 - 18 w_i (c_iy N_y + c_iz N_z),
// N_a = sum_{c_x = 0} f c_a - (2/3) rho u_a, which imposes rho and the whole
// velocity and reduces to the D3Q19 closure above on the D3Q19 set.
template <class T>
void zouhe_face(T f[Q], int side, T rho, T ux, T uy, T uz) {
  T sy = 0, sz = 0;
  for (int i = 0; i < Q; ++i)
    if (CV[i][0] == 0) { sy += f[i] * (double)CV[i][1]; sz += f[i] * (double)CV[i][2]; }
  const T Ny = sy - (2.0 / 3.0) * rho * uy, Nz = sz - (2.0 / 3.0) * rho * uz;
  for (int i = 0; i < Q; ++i) {
    if (CV[i][0] != side) continue;
    const int o = opposite(i);
    const T cu = (double)CV[i][0] * ux + (double)CV[i][1] * uy + (double)CV[i][2] * uz;
    f[i] = f[o] + 2.0 * WT[i] * rho * cu / CS2 - 18.0 * WT[i] * ((double)CV[i][1] * Ny + (double)CV[i][2] * Nz);
  }
}
template <class T>
void zouhe_inlet(T f[Q], double ux, double uy, double uz) {
  T s0 = 0, sm = 0;
  for (int i = 0; i < Q; ++i) {
    if (CV[i][0] == 0) s0 += f[i];
    if (CV[i][0] == -1) sm += f[i];
  }
  zouhe_face(f, 1, (s0 + 2.0 * sm) / (1.0 - ux), T(ux), T(uy), T(uz));
}
template <class T>
void zouhe_outlet(T f[Q], double rho_out) {
  T s0 = 0, sp = 0;
  for (int i = 0; i < Q; ++i) {
    if (CV[i][0] == 0) s0 += f[i];
    if (CV[i][0] == 1) sp += f[i];
  }
  T ux = (s0 + 2.0 * sp) / rho_out - 1.0;
  zouhe_face(f, -1, T(rho_out), ux, T(0.0), T(0.0));
}
#else
template <class T>
void zouhe_inlet(T f[Q], double ux, double uy, double uz) {
  T s0 = 0, sm = 0, sy = 0, sz = 0;
  for (int i = 0; i < Q; ++i) {
    if (CV[i][0] == 0) { s0 += f[i]; sy += f[i] * (double)CV[i][1]; sz += f[i] * (double)CV[i][2]; }
    if (CV[i][0] == -1) sm += f[i];
  }
  T rho = (s0 + 2.0 * sm) / (1.0 - ux);
  T Ny = 0.5 * sy - rho * uy / 3.0;
  T Nz = 0.5 * sz - rho * uz / 3.0;
  // f(+x) = f(-x) + rho ux/3; edge populations with the transverse corrections
  for (int i = 0; i < Q; ++i) {
    if (CV[i][0] != 1) continue;
    int o = opposite(i);
    int cy = CV[i][1], cz = CV[i][2];
    if (cy == 0 && cz == 0) f[i] = f[o] + rho * ux / 3.0;
    else if (cy != 0) f[i] = f[o] + rho * (ux + cy * uy) / 6.0 - (double)cy * Ny;
    else f[i] = f[o] + rho * (ux + cz * uz) / 6.0 - (double)cz * Nz;
  }
}

template <class T>
void zouhe_outlet(T f[Q], double rho_out) {
  T s0 = 0, sp = 0, sy = 0, sz = 0;
  for (int i = 0; i < Q; ++i) {
    if (CV[i][0] == 0) { s0 += f[i]; sy += f[i] * (double)CV[i][1]; sz += f[i] * (double)CV[i][2]; }
    if (CV[i][0] == 1) sp += f[i];
  }
  T ux = (s0 + 2.0 * sp) / rho_out - 1.0;
  T Ny = 0.5 * sy, Nz = 0.5 * sz;  // tangential velocity 0
  for (int i = 0; i < Q; ++i) {
    if (CV[i][0] != -1) continue;
    int o = opposite(i);
    int cy = CV[i][1], cz = CV[i][2];
    if (cy == 0 && cz == 0) f[i] = f[o] - rho_out * ux / 3.0;
    else if (cy != 0) f[i] = f[o] - rho_out * ux / 6.0 - (double)cy * Ny;
    else f[i] = f[o] - rho_out * ux / 6.0 - (double)cz * Nz;
  }
}
#endif

// Everything one cell computes in one step.
template <class T>
struct CellResult {
  T rho, u[3], F[3], feq[Q], Pi[6], shear, nu, omega, q[Q];
};

// One cell: moments, velocity, force, equilibrium, second moment, rheology and
// collision.  f holds the cell's pre-collision populations after the open-face
// fill; phit[i] is the porosity at x + c_i (the cell's own porosity where that
// neighbour is solid or outside: no porosity jump across walls).
template <class T>
void cell_update(const oracle_case& c, const Shape& S, const T f[Q], T omega_prev, T phi, const T phit[Q],
                 CellResult<T>& r) {
  // moments: rho = phi^-1 sum f, momentum sum f c
  T sumf = 0, m[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i) {
    sumf += f[i];
    for (int a = 0; a < 3; ++a) m[a] += f[i] * (double)CV[i][a];
  }
  T rho = sumf / phi;
  // preliminary velocity v = (phi rho)^-1 sum f c, plus half the body force
  // (the body force enters u the same way as the drag; a reading: the paper
  // has no body force, the channel configuration adds one)
  T v[3];
  for (int a = 0; a < 3; ++a) v[a] = m[a] / (phi * rho) + c.g[a] / (2.0 * phi);
  // Kozeny-Carman permeability k = phi^3 d^2 / (K_c (1-phi)^2), used as 1/k so
  // that phi = 1 (no medium) gives 1/k = 0
  T om = 1.0 - phi;
  T invk = c.kc * om * om / (c.d * c.d * phi * phi * phi);
  // sqrt(1/k), written for 0 < phi <= 1 as sqrt(K_c) (1 - phi) / (d phi^(3/2)):
  // the same value, and differentiable at phi = 1 from below (the square root
  // of (1 - phi)^2 has a kink there, which the dual numbers would flatten)
  T sik = std::sqrt(c.kc) * om / (c.d * phi * Sqrt(phi));
  T CF = 0;
  if (c.forchheimer) CF = 1.75 / Sqrt(150.0 * phi * phi * phi);
  if (!S.on) {
    // explicit velocity: u = v / (C0 + sqrt(C0^2 + C1 |v|))
    T C0 = 0.5 + phi * c.nu_d * invk / 4.0;
    T C1 = phi * phi * CF * sik / 2.0;
    T vn = Sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    T den = C0 + Sqrt(C0 * C0 + C1 * vn);
    for (int a = 0; a < 3; ++a) r.u[a] = v[a] / den;
    // force density rho f(u): body force, Darcy and Forchheimer drag
    T un = Sqrt(r.u[0] * r.u[0] + r.u[1] * r.u[1] + r.u[2] * r.u[2]);
    for (int a = 0; a < 3; ++a)
      r.F[a] = rho * (c.g[a] - phi * phi * c.nu_d * invk * r.u[a] - phi * phi * phi * CF * sik * un * r.u[a]);
  } else {
    // anisotropic: A = Id + (phi nu / 2) K^-1, B = (phi^2 C_F / 2) K^-1/2,
    // u_{m+1} = (A + |u_m| B)^-1 v from u_0 = v (the Remark's fixed point)
    T Ki[3][3], Kh[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        Ki[i][j] = invk * S.Minv[i][j];
        Kh[i][j] = sik * S.Mhi[i][j];
      }
    T A[3][3], B[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        A[i][j] = (i == j ? 1.0 : 0.0) + 0.5 * phi * c.nu_d * Ki[i][j];
        B[i][j] = 0.5 * phi * phi * CF * Kh[i][j];
      }
    T u[3] = {v[0], v[1], v[2]};
    for (int m = 0; m < c.aniso_iters; ++m) {
      T un = Sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      T X[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) X[i][j] = A[i][j] + un * B[i][j];
      solve3(X, v, u);
    }
    for (int a = 0; a < 3; ++a) r.u[a] = u[a];
    // force density: body force and the tensor drag -phi^2 nu K^-1 u - phi^3 C_F |u| K^-1/2 u
    T un = Sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int a = 0; a < 3; ++a) {
      T kd = 0, kf = 0;
      for (int b = 0; b < 3; ++b) {
        kd += Ki[a][b] * u[b];
        kf += Kh[a][b] * u[b];
      }
      r.F[a] = rho * (c.g[a] - phi * phi * c.nu_d * kd - phi * phi * phi * CF * un * kf);
    }
  }
  r.rho = rho;
  // equilibrium with porosity
  T uu = r.u[0] * r.u[0] + r.u[1] * r.u[1] + r.u[2] * r.u[2];
  for (int i = 0; i < Q; ++i) {
    T cu = r.u[0] * (double)CV[i][0] + r.u[1] * (double)CV[i][1] + r.u[2] * (double)CV[i][2];
    r.feq[i] = WT[i] * phi * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
  // corrected second moment Pi = sum (f - feq) c c + (1/2)(F u + u F); order xx yy zz xy xz yz
  const int PA[6] = {0, 1, 2, 0, 0, 1}, PB[6] = {0, 1, 2, 1, 2, 2};
  for (int k = 0; k < 6; ++k) {
    T s = 0;
    for (int i = 0; i < Q; ++i) s += (f[i] - r.feq[i]) * (double)(CV[i][PA[k]] * CV[i][PB[k]]);
    r.Pi[k] = s + 0.5 * (r.F[PA[k]] * r.u[PB[k]] + r.u[PA[k]] * r.F[PB[k]]);
  }
  T pn2 = 0;
  for (int k = 0; k < 6; ++k) pn2 += (k < 3 ? 1.0 : 2.0) * r.Pi[k] * r.Pi[k];
  // semi-explicit shear rate: previous relaxation rate times |Pi|_F / (c_s^2 rho)
  r.shear = omega_prev * Sqrt(pn2) / (CS2 * rho);
  // Carreau-Yasuda viscosity (kinematic; dynamic mu = rho_0 nu with rho_0 = 1)
  T la = c.lam * r.shear;
  r.nu = c.nu_inf + (c.nu0 - c.nu_inf) * Pow(1.0 + Pow(la, c.a), (c.n - 1.0) / c.a);
  T mu = r.nu;  // rho_0 = 1
  // relaxation rate from viscosity: omega = 2 rho c_s^2 / (2 mu + rho c_s^2)
  r.omega = 2.0 * rho * CS2 / (2.0 * mu + rho * CS2);
  // collision: f + Omega^phi + Omega^f + Omega^SRT
  for (int i = 0; i < Q; ++i) {
    T cu = r.u[0] * (double)CV[i][0] + r.u[1] * (double)CV[i][1] + r.u[2] * (double)CV[i][2];
    T guo = 0;
    for (int a = 0; a < 3; ++a)
      guo += (((double)CV[i][a] - r.u[a]) / CS2 + cu * (double)CV[i][a] / (CS2 * CS2)) * r.F[a];
    guo = WT[i] * (1.0 - r.omega / 2.0) * guo;
    T omphi = WT[i] * rho * (phit[i] - phi);
    T srt = -r.omega * (f[i] - r.feq[i]);
    r.q[i] = f[i] + omphi + guo + srt;
  }
}

// ---------------------------------------------------------------------------
// Extrapolation outflow (the simulation section's non-reflecting outflow after
// Geier et al.).  Reading: every population is treated as a field carried out
// through the outflow face at the speed of sound c_s, and the advection is
// discretised upwind in space and forward in time, so an unknown population i
// (c_x = -1) of an outflow cell x_b at the next step is
//   f_i(t+1, x_b) = (1 - c_s) f_i(t, x_b) + c_s f_i(t, x_b - e_x),
// both pre-collision values of step t (f_i(t, x_b) being the previous
// extrapolated value).  The state therefore keeps these unknowns: the rest
// state holds their rest value, and each step writes them while streaming.
// If x_b - e_x is not a fluid cell the upstream term is the cell's own.
// ---------------------------------------------------------------------------
template <class T>
void extrapolate_outlet(const Ctx& C, const T* f, int64_t x, T* fn) {
  const int64_t nf = C.nf;
  const double cs = std::sqrt(CS2);
  const int up = C.nbr[2 * nf + x];  // direction 2 is -x
  for (int i = 0; i < Q; ++i) {
    if (CV[i][0] != -1 || C.nbr[opposite(i) * nf + x] != NB_OPEN) continue;
    const T own = f[i * nf + x];
    const T ups = up >= 0 ? f[i * nf + up] : own;
    fn[i * nf + x] = (1.0 - cs) * own + cs * ups;
  }
}

// ---------------------------------------------------------------------------
// Wall shear stress (the simulation section's WSS, here on the voxel wall).
// Reading: the paper extrapolates the deviatoric stress to a wall mesh and
// projects it on the tangential plane; with no mesh, the wall is the set of
// fluid cells that have a bounce-back link, the outer normal of such a cell is
// the lattice-weighted mean direction of its wall links,
//   n = m / |m|,  m = sum over {i : x + c_i is wall} of w_i c_i,
// and tau = sigma n - (n . sigma n) n with the cell's deviatoric stress
// sigma = (omega/2 - 1) Pi (omega the relaxation rate the cell computes in
// this step).  A cell whose wall links cancel (m = 0) has no normal and no WSS.
// Open-face links are not wall.
// ---------------------------------------------------------------------------
bool wall_normal(const Ctx& C, int64_t x, double n[3]) {
  double m[3] = {0.0, 0.0, 0.0};
  for (int i = 1; i < Q; ++i)
    if (C.nbr[i * C.nf + x] == NB_WALL)
      for (int a = 0; a < 3; ++a) m[a] += WT[i] * CV[i][a];
  const double len = std::sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
  for (int a = 0; a < 3; ++a) n[a] = len > 0.0 ? m[a] / len : 0.0;
  return len > 0.0;
}

template <class T>
void wall_shear(const CellResult<T>& r, const double n[3], T tau[3]) {
  const T s = r.omega / 2.0 - 1.0;
  // full symmetric tensor from the stored xx yy zz xy xz yz
  const T P[3][3] = {{r.Pi[0], r.Pi[3], r.Pi[4]}, {r.Pi[3], r.Pi[1], r.Pi[5]}, {r.Pi[4], r.Pi[5], r.Pi[2]}};
  T sn[3];
  for (int a = 0; a < 3; ++a) sn[a] = s * (P[a][0] * n[0] + P[a][1] * n[1] + P[a][2] * n[2]);
  const T nsn = sn[0] * n[0] + sn[1] * n[1] + sn[2] * n[2];
  for (int a = 0; a < 3; ++a) tau[a] = sn[a] - nsn * n[a];
}

// Per-cell term of the objective e(t): kind 0 the kinetic energy rho |u|^2 / 2
// on region cells, kind 1 the WSS magnitude |tau| on region cells of the wall.
template <class T>
T objective_term(const Ctx& C, int64_t x, const CellResult<T>& r, int kind) {
  if (!C.sac[x]) return T(0.0);
  if (kind == 0) return 0.5 * r.rho * (r.u[0] * r.u[0] + r.u[1] * r.u[1] + r.u[2] * r.u[2]);
  if (!C.wall[x]) return T(0.0);
  T tau[3];
  wall_shear(r, &C.nrm[3 * x], tau);
  return Sqrt(tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2]);
}

// Number of cells e(t) averages over.
long objective_count(const Ctx& C, int kind) { return std::max(1L, kind == 0 ? C.nsac : C.nwss); }

// Gather a cell's inputs: its populations (after the open-face fill at step t)
// and the porosity of its neighbours.
template <class T>
void cell_inputs(const Ctx& C, const T* f, int64_t x, int t, const T* phi_f, T fl[Q], T phit[Q]) {
  const int64_t nf = C.nf;
  for (int i = 0; i < Q; ++i) fl[i] = f[i * nf + x];
  if (C.kind[x] == 1) {
    double ux = amplitude(C, t) * C.shape[C.yc[x] + (int64_t)C.c.ny * C.zc[x]];
    zouhe_inlet(fl, ux, 0.0, 0.0);
  } else if (C.kind[x] == 2 && C.c.outlet == 1) {
    zouhe_outlet(fl, C.c.rho_out);
  }
  for (int i = 0; i < Q; ++i) {
    int nb = C.nbr[i * nf + x];
    phit[i] = (i > 0 && nb >= 0) ? phi_f[nb] : phi_f[x];
  }
}

// Push the post-collision populations along the links.
template <class T>
void stream_out(const Ctx& C, int64_t x, const T q[Q], T* fn) {
  const int64_t nf = C.nf;
  for (int i = 0; i < Q; ++i) {
    int nb = C.nbr[i * nf + x];
    if (nb >= 0) fn[i * nf + nb] = q[i];
    else if (nb == NB_WALL) fn[opposite(i) * nf + x] = q[i];
    // NB_OPEN: leaves the domain
  }
}

// One full step in place: f (pre-collision, [Q][nf]) and omega (previous rate).
// If ke is non-null, also returns the sac-averaged kinetic energy of step t.
template <class T>
void step(const Ctx& C, std::vector<T>& f, std::vector<T>& omega, const std::vector<T>& phi_f, int t, T* ke,
          int kind = 0) {
  const int64_t nf = C.nf;
  std::vector<T> fn((size_t)Q * nf, T(0.0));
  std::vector<T> keloc(ke ? nf : 0, T(0.0));
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < nf; ++x) {
    T fl[Q], phit[Q];
    cell_inputs(C, f.data(), x, t, phi_f.data(), fl, phit);
    CellResult<T> r;
    cell_update(C.c, C.shape_m, fl, omega[x], phi_f[x], phit, r);
    omega[x] = r.omega;
    if (ke) keloc[x] = objective_term(C, x, r, kind);
    stream_out(C, x, r.q, fn.data());
    if (C.kind[x] == 2 && C.c.outlet == 2) extrapolate_outlet(C, f.data(), x, fn.data());
  }
  f.swap(fn);
  if (ke) {
    T s = 0;
    for (int64_t x = 0; x < nf; ++x) if (C.sac[x]) s += keloc[x];
    *ke = s / (double)objective_count(C, kind);
  }
}

double omega_rest(const oracle_case& c) { return 2.0 * CS2 / (2.0 * c.nu0 + CS2); }

template <class T>
void rest_state(const Ctx& C, const std::vector<T>& phi_f, std::vector<T>& f, std::vector<T>& omega) {
  const int64_t nf = C.nf;
  f.assign((size_t)Q * nf, T(0.0));
  omega.assign(nf, T(omega_rest(C.c)));
  for (int64_t x = 0; x < nf; ++x)
    for (int i = 0; i < Q; ++i) {
      bool unknown = false;
      int o = opposite(i);
      // population i arrives from x - c_i = x + c_o; unknown if that is an open
      // face, except on an extrapolation outflow, whose state keeps them
      if (C.nbr[o * nf + x] == NB_OPEN && !(C.kind[x] == 2 && C.c.outlet == 2)) unknown = true;
      f[i * nf + x] = unknown ? T(0.0) : WT[i] * phi_f[x];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// C API
// ---------------------------------------------------------------------------
extern "C" {

void* oracle_new(const oracle_case* c) {
  Ctx* C = new Ctx();
  C->c = *c;
  const int64_t nb = (int64_t)c->nx * c->ny * c->nz;
  C->solid.assign(c->solid, c->solid + nb);
  C->phi_box.assign(c->phi, c->phi + nb);
  C->sac.clear();
  if (c->inlet_shape) C->shape.assign(c->inlet_shape, c->inlet_shape + (int64_t)c->ny * c->nz);
  else C->shape.assign((int64_t)c->ny * c->nz, 0.0);
  if (c->wave_table && c->table_len > 0) C->wave.assign(c->wave_table, c->wave_table + c->table_len);
  C->c.solid = nullptr; C->c.phi = nullptr; C->c.sac = nullptr; C->c.inlet_shape = nullptr;
  C->c.wave_table = nullptr;
  C->box2f.assign(nb, -1);
  for (int64_t b = 0; b < nb; ++b)
    if (!c->solid[b]) { C->box2f[b] = (int64_t)C->cells.size(); C->cells.push_back(b); }
  C->nf = (int64_t)C->cells.size();
  const int64_t nf = C->nf;
  C->xc.resize(nf); C->yc.resize(nf); C->zc.resize(nf); C->kind.assign(nf, 0); C->sac.assign(nf, 0);
  for (int64_t x = 0; x < nf; ++x) {
    int64_t b = C->cells[x];
    C->xc[x] = (int)(b % c->nx);
    C->yc[x] = (int)((b / c->nx) % c->ny);
    C->zc[x] = (int)(b / ((int64_t)c->nx * c->ny));
    if (c->inlet && C->xc[x] == 0) C->kind[x] = 1;
    else if (c->outlet && C->xc[x] == c->nx - 1) C->kind[x] = 2;
    if (c->sac && c->sac[b]) { C->sac[x] = 1; C->nsac++; }
  }
  C->nbr.assign((size_t)Q * nf, 0);
  for (int64_t x = 0; x < nf; ++x)
    for (int i = 0; i < Q; ++i) C->nbr[i * nf + x] = classify(*C, C->xc[x], C->yc[x], C->zc[x], i);
  C->shape_m = shape_of(C->c);
  C->nrm.assign((size_t)3 * nf, 0.0);
  C->wall.assign(nf, 0);
  for (int64_t x = 0; x < nf; ++x) {
    C->wall[x] = wall_normal(*C, x, &C->nrm[3 * x]) ? 1 : 0;
    if (C->wall[x] && C->sac[x]) C->nwss++;
  }
  return C;
}

void oracle_free(void* h) { delete (Ctx*)h; }
int64_t oracle_nfluid(void* h) { return ((Ctx*)h)->nf; }
void oracle_cells(void* h, int64_t* out) { Ctx* C = (Ctx*)h; std::copy(C->cells.begin(), C->cells.end(), out); }
void oracle_neighbours(void* h, int32_t* out) { Ctx* C = (Ctx*)h; std::copy(C->nbr.begin(), C->nbr.end(), out); }
double oracle_amplitude(void* h, int t) { return amplitude(*(Ctx*)h, t); }

static std::vector<double> fluid_phi(const Ctx& C) {
  std::vector<double> p(C.nf);
  for (int64_t x = 0; x < C.nf; ++x) p[x] = C.phi_box[C.cells[x]];
  return p;
}

void oracle_set_phi(void* h, const double* phi_box) {
  Ctx* C = (Ctx*)h;
  std::copy(phi_box, phi_box + C->phi_box.size(), C->phi_box.begin());
}

void oracle_init(void* h, double* f, double* omega) {
  Ctx* C = (Ctx*)h;
  std::vector<double> ff, oo, ph = fluid_phi(*C);
  rest_state(*C, ph, ff, oo);
  std::copy(ff.begin(), ff.end(), f);
  std::copy(oo.begin(), oo.end(), omega);
}

// Advance nsteps from step index t0; f ([19][nf]) and omega ([nf]) in place.
// ke_out (nullable, [nsteps]) receives the sac-averaged kinetic energy per step.
void oracle_run(void* h, double* f, double* omega, int t0, int nsteps, double* ke_out) {
  Ctx* C = (Ctx*)h;
  std::vector<double> ff(f, f + (size_t)Q * C->nf), oo(omega, omega + C->nf), ph = fluid_phi(*C);
  for (int s = 0; s < nsteps; ++s) {
    double ke = 0;
    step(*C, ff, oo, ph, t0 + s, ke_out ? &ke : nullptr);
    if (ke_out) ke_out[s] = ke;
  }
  std::copy(ff.begin(), ff.end(), f);
  std::copy(oo.begin(), oo.end(), omega);
}

// Macroscopic fields of the state at step t (fill, moments, velocity, Pi,
// shear rate, new relaxation rate, deviatoric stress sigma = (omega/2 - 1) Pi,
// wall shear stress tau [3][nf], 0 off the wall), per fluid cell.  Any output
// may be NULL.
void oracle_moments(void* h, const double* f, const double* omega, int t, double* rho, double* u,
                    double* shear, double* omega_new, double* sigma, double* tau) {
  Ctx* C = (Ctx*)h;
  const int64_t nf = C->nf;
  std::vector<double> ph = fluid_phi(*C);
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < nf; ++x) {
    double fl[Q], phit[Q];
    cell_inputs(*C, f, x, t, ph.data(), fl, phit);
    CellResult<double> r;
    cell_update(C->c, C->shape_m, fl, omega[x], ph[x], phit, r);
    if (rho) rho[x] = r.rho;
    if (u) for (int a = 0; a < 3; ++a) u[a * nf + x] = r.u[a];
    if (shear) shear[x] = r.shear;
    if (omega_new) omega_new[x] = r.omega;
    if (sigma) for (int k = 0; k < 6; ++k) sigma[k * nf + x] = (r.omega / 2.0 - 1.0) * r.Pi[k];
    if (tau) {
      double tw[3] = {0.0, 0.0, 0.0};
      if (C->wall[x]) wall_shear(r, &C->nrm[3 * x], tw);
      for (int a = 0; a < 3; ++a) tau[a * nf + x] = tw[a];
    }
  }
}

// Single-cell evaluation for identity tests.  f: 19 populations (no fill is
// applied), phit: porosity at x + c_i.  Outputs (any may be NULL): rho, u[3],
// F[3], feq[19], Pi[6], shear, nu, omega, q[19].
void oracle_cell(const oracle_case* c, const double* f, double omega_prev, double phi, const double* phit,
                 double* rho, double* u, double* F, double* feq, double* Pi, double* shear, double* nu,
                 double* omega, double* q) {
  CellResult<double> r;
  double pt[Q];
  for (int i = 0; i < Q; ++i) pt[i] = phit[i];
  cell_update(*c, shape_of(*c), f, omega_prev, phi, pt, r);
  if (rho) *rho = r.rho;
  for (int a = 0; a < 3; ++a) { if (u) u[a] = r.u[a]; if (F) F[a] = r.F[a]; }
  for (int i = 0; i < Q; ++i) { if (feq) feq[i] = r.feq[i]; if (q) q[i] = r.q[i]; }
  for (int k = 0; k < 6; ++k) if (Pi) Pi[k] = r.Pi[k];
  if (shear) *shear = r.shear;
  if (nu) *nu = r.nu;
  if (omega) *omega = r.omega;
}

void oracle_zouhe_inlet(double* f, double ux, double uy, double uz) { zouhe_inlet(f, ux, uy, uz); }
void oracle_zouhe_outlet(double* f, double rho_out) { zouhe_outlet(f, rho_out); }

void oracle_lattice(int* c, double* w) {
  for (int i = 0; i < Q; ++i) { for (int a = 0; a < 3; ++a) c[3 * i + a] = CV[i][a]; w[i] = WT[i]; }
}

// Objective: J = (1/(te-tb)) sum_{t=tb}^{te-1} e(t), e(t) = sac mean of
// (1/2) rho |u|^2 (kind 0) or of the WSS magnitude over the sac's wall cells
// (kind 1) from step t's moments, starting at rest and running T steps.
double oracle_objective(void* h, int T, int tb, int te, int kind) {
  Ctx* C = (Ctx*)h;
  std::vector<double> ph = fluid_phi(*C), f, om;
  rest_state(*C, ph, f, om);
  double J = 0;
  for (int t = 0; t < T; ++t) {
    double ke = 0;
    bool in = (t >= tb && t < te);
    step(*C, f, om, ph, t, in ? &ke : nullptr, kind);
    if (in) J += ke;
  }
  return J / (double)(te - tb);
}

// Exact discrete derivative dJ/dphi at up to 16 cells (box indices) by
// forward-mode dual numbers (one derivative component per cell).
void oracle_grad_dual(void* h, int T, int tb, int te, const int64_t* boxcells, int ncells, double* J,
                      double* grads, int kind) {
  const int N = 16;
  typedef Dual<N> D;
  Ctx* C = (Ctx*)h;
  std::vector<double> ph0 = fluid_phi(*C);
  std::vector<D> ph(C->nf);
  for (int64_t x = 0; x < C->nf; ++x) ph[x] = D(ph0[x]);
  for (int k = 0; k < ncells && k < N; ++k) {
    int64_t fi = C->box2f[boxcells[k]];
    if (fi >= 0) ph[fi].d[k] = 1.0;
  }
  std::vector<D> f, om;
  rest_state(*C, ph, f, om);
  D acc = 0;
  for (int t = 0; t < T; ++t) {
    D ke;
    bool in = (t >= tb && t < te);
    step(*C, f, om, ph, t, in ? &ke : nullptr, kind);
    if (in) acc += ke;
  }
  acc = acc / (double)(te - tb);
  *J = acc.v;
  for (int k = 0; k < ncells && k < N; ++k) grads[k] = acc.d[k];
}

// Full gradient dJ/dphi (box layout, 0 outside the fluid) by a reverse sweep.
// The forward trajectory is checkpointed every `ckpt` steps and recomputed per
// segment.  For each cell and step the local Jacobian of
//   (19 pre-collision populations, previous omega, phi(x), 18 neighbour phi)
//   -> (19 post-collision populations, new omega, kinetic-energy term)
// is taken with 39-component dual numbers and its transpose applied to the
// output adjoints; the streaming transpose gathers along +c_i.  With the
// extrapolation outflow the outflow cells' unknowns are state that step n
// computes linearly from step n-1's values (see extrapolate_outlet); that map
// is transposed after the local maps.
void oracle_grad_reverse(void* h, int T, int tb, int te, int ckpt, double* J, double* grad_box, int kind) {
  const int NI = 2 * Q + 1;
  typedef Dual<NI> D;
  Ctx* C = (Ctx*)h;
  const int64_t nf = C->nf;
  const bool extrap = C->c.outlet == 2;
  std::vector<double> ph = fluid_phi(*C), f, om;
  rest_state(*C, ph, f, om);
  // forward with checkpoints
  int nseg = (T + ckpt - 1) / ckpt;
  std::vector<std::vector<double>> cf(nseg), co(nseg);
  double acc = 0;
  for (int t = 0; t < T; ++t) {
    if (t % ckpt == 0) { cf[t / ckpt] = f; co[t / ckpt] = om; }
    double ke = 0;
    bool in = (t >= tb && t < te);
    step(*C, f, om, ph, t, in ? &ke : nullptr, kind);
    if (in) acc += ke;
  }
  *J = acc / (double)(te - tb);
  const double ew = 1.0 / ((double)(te - tb) * (double)objective_count(*C, kind));

  std::vector<double> fh((size_t)Q * nf, 0.0), fh_new((size_t)Q * nf, 0.0);  // adjoint of f_{n+1}, f_n
  std::vector<double> oh(nf, 0.0), oh_new(nf, 0.0);                           // adjoint of omega_n, omega_{n-1}
  std::vector<double> phh(nf, 0.0);
  std::vector<double> nbcontrib((size_t)Q * nf, 0.0);  // adjoint for phi at x + c_i
  for (int s = nseg - 1; s >= 0; --s) {
    int t0 = s * ckpt, t1 = std::min(T, t0 + ckpt);
    // recompute the segment's states
    std::vector<std::vector<double>> sf(t1 - t0), so(t1 - t0);
    std::vector<double> ff = cf[s], oo = co[s];
    for (int t = t0; t < t1; ++t) {
      sf[t - t0] = ff; so[t - t0] = oo;
      step(*C, ff, oo, ph, t, (double*)nullptr);
    }
    for (int t = t1 - 1; t >= t0; --t) {
      const std::vector<double>& fs = sf[t - t0];
      const std::vector<double>& os = so[t - t0];
      bool in = (t >= tb && t < te);
#pragma omp parallel for schedule(static)
      for (int64_t x = 0; x < nf; ++x) {
        // seed inputs
        D fl[Q], phit[Q], phx, omp;
        for (int i = 0; i < Q; ++i) { fl[i] = D(fs[i * nf + x]); fl[i].d[i] = 1.0; }
        omp = D(os[x]); omp.d[Q] = 1.0;
        phx = D(ph[x]); phx.d[Q + 1] = 1.0;
        for (int i = 0; i < Q; ++i) {
          int nb = C->nbr[i * nf + x];
          if (i > 0 && nb >= 0) { phit[i] = D(ph[nb]); phit[i].d[Q + 1 + i] = 1.0; }
          else phit[i] = phx;
        }
        // open-face fill (inside the local map)
        if (C->kind[x] == 1) {
          double ux = amplitude(*C, t) * C->shape[C->yc[x] + (int64_t)C->c.ny * C->zc[x]];
          zouhe_inlet(fl, ux, 0.0, 0.0);
        } else if (C->kind[x] == 2 && !extrap) {
          zouhe_outlet(fl, C->c.rho_out);
        }
        CellResult<D> r;
        cell_update(C->c, C->shape_m, fl, omp, phx, phit, r);
        D e = objective_term(*C, x, r, kind);
        // output adjoints
        double qh[Q];
        for (int i = 0; i < Q; ++i) {
          int nb = C->nbr[i * nf + x];
          if (nb >= 0) qh[i] = fh[i * nf + nb];
          else if (nb == NB_WALL) qh[i] = fh[opposite(i) * nf + x];
          else qh[i] = 0.0;
        }
        double wh = oh[x];
        double eh = (in && C->sac[x]) ? ew : 0.0;
        double g[NI];
        for (int k = 0; k < NI; ++k) {
          double s2 = wh * r.omega.d[k] + eh * e.d[k];
          for (int i = 0; i < Q; ++i) s2 += qh[i] * r.q[i].d[k];
          g[k] = s2;
        }
        for (int i = 0; i < Q; ++i) fh_new[i * nf + x] = g[i];
        oh_new[x] = g[Q];
        phh[x] += g[Q + 1];
        for (int i = 1; i < Q; ++i) nbcontrib[i * nf + x] = g[Q + 1 + i];
      }
      // scatter neighbour-porosity adjoints (serial: plain and race-free)
      for (int64_t x = 0; x < nf; ++x)
        for (int i = 1; i < Q; ++i) {
          int nb = C->nbr[i * nf + x];
          if (nb >= 0) phh[nb] += nbcontrib[i * nf + x];
        }
      // transpose of the extrapolation: f_i(t+1, x_b) = (1 - c_s) f_i(t, x_b) + c_s f_i(t, x_b - e_x)
      if (extrap) {
        const double cs = std::sqrt(CS2);
        for (int64_t x = 0; x < nf; ++x) {
          if (C->kind[x] != 2) continue;
          const int up = C->nbr[2 * nf + x];
          for (int i = 0; i < Q; ++i) {
            if (CV[i][0] != -1 || C->nbr[opposite(i) * nf + x] != NB_OPEN) continue;
            const double a = fh[i * nf + x];
            fh_new[i * nf + x] += (up >= 0 ? 1.0 - cs : 1.0) * a;
            if (up >= 0) fh_new[i * nf + up] += cs * a;
          }
        }
      }
      fh.swap(fh_new);
      oh.swap(oh_new);
    }
  }
  // initial state f_i(0, x) = w_i phi(x) on the known links (and on the
  // extrapolation outflow's unknowns, which are state)
  for (int64_t x = 0; x < nf; ++x)
    for (int i = 0; i < Q; ++i) {
      int o = opposite(i);
      if (C->nbr[o * nf + x] == NB_OPEN && !(C->kind[x] == 2 && extrap)) continue;
      phh[x] += WT[i] * fh[i * nf + x];
    }
  const int64_t nb = (int64_t)C->c.nx * C->c.ny * C->c.nz;
  std::fill(grad_box, grad_box + nb, 0.0);
  for (int64_t x = 0; x < nf; ++x) grad_box[C->cells[x]] = phh[x];
}

int oracle_threads(void) { return omp_get_max_threads(); }
// Thread count of later parallel loops (n < 1: one per processor); returns the previous count.
int oracle_set_threads(int n) {
  const int prev = omp_get_max_threads();
  omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
  return prev;
}
int oracle_q(void) { return Q; }

}  // extern "C"
