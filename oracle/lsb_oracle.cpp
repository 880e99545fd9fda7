// lsb_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, FP64 CPU oracle of the coupled level-set lattice Boltzmann
// two-fluid method (Vorspohl et al., "Coupled Level-Set Lattice Boltzmann
// Method on Adaptive Cartesian Grids").  Only the tests, the smoke check and
// the CPU-baseline leg of the benchmark may load this library; the product
// path never does.  It shares no code, header or table with the HIP library.
//
// Every routine is written as plain nested loops over the cells of a dense
// uniform grid, in the order the method states.  The whole state update is a
// template over the scalar type T; T = double is the oracle proper and
// T = Dual (value + tangent) differentiates the identical discrete program.
// All branches are taken on the primal value, so the Dual instantiation gives
// the derivative with every discrete decision frozen.
//
// Paper passages followed (section / equation):
//   Sec. 2.1  LB evolution equation (Eq. 1), moments (eq:macro), BGK
//             collision, equilibrium (eq:feq), relaxation frequency
//             (eq:omega), gravity forcing, interpolated bounce-back (eq:bb)
//             with the moving-wall momentum term.
//   Sec. 2.2  level-set sign convention, transport equation, narrow band,
//             hyperbolic velocity extension (eq:hyperbolicExtension),
//             constrained reinitialisation, normal and curvature.
//   Sec. 2.3  interface bounce-back momentum term (eq:bb_cc), stress-jump
//             decomposition (eq:Sdecomp), wall distance from the level set
//             (radiation theorem).
//   Sec. 2.4  refilling of newly activated cells (e_min, f^neq copy,
//             quadratic extrapolation of rho and u).
//   Sec. 3.2  Heaviside-weighted gas centroid and bubble velocity; the
//             interface kept on the finest level of a two-level grid
//             (with the Sec. 2.1 refinement: lattice units and relaxation
//             time rescaled, Dupuis-Chopard coupling of the levels).
// Where the paper is silent or garbled, the reading taken is stated at the
// place it is used; the same readings are listed in the repository's design
// notes.
//
// Parity status: every part is pinned by the CPU tests (closed forms,
// invariants, brute force) except where a function header says
// "parity unpinned".

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <vector>

namespace orc {

// --------------------------------------------------------------------------
// Dual number: value and one tangent component.  Comparisons are deliberately
// not defined: every decision must go through val().
// --------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double a) : v(a), d(0.0) {}
  Dual(double a, double b) : v(a), d(b) {}
  Dual& operator+=(const Dual& o) { v += o.v; d += o.d; return *this; }
  Dual& operator-=(const Dual& o) { v -= o.v; d -= o.d; return *this; }
  Dual& operator*=(const Dual& o) { d = d * o.v + v * o.d; v *= o.v; return *this; }
  Dual& operator/=(const Dual& o) { double r = v / o.v; d = (d - r * o.d) / o.v; v = r; return *this; }
};
inline Dual operator+(Dual a, const Dual& b) { return a += b; }
inline Dual operator-(Dual a, const Dual& b) { return a -= b; }
inline Dual operator*(Dual a, const Dual& b) { return a *= b; }
inline Dual operator/(Dual a, const Dual& b) { return a /= b; }
inline Dual operator-(const Dual& a) { return Dual(-a.v, -a.d); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(double a, const Dual& b) { return Dual(a * b.v, a * b.d); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator*(const Dual& a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator/(const Dual& a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual sqrt(const Dual& a) { double s = std::sqrt(a.v); return Dual(s, s > 0 ? 0.5 * a.d / s : 0.0); }
inline Dual sin(const Dual& a) { return Dual(std::sin(a.v), std::cos(a.v) * a.d); }
inline Dual fabs(const Dual& a) { return a.v < 0 ? -a : a; }

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
using std::sqrt;
using std::sin;
using std::fabs;

// --------------------------------------------------------------------------
// Lattices.  Direction order follows the paper's velocity-set figure (rest
// direction last).  D3Q19 is not in the paper: it is the textbook set made of
// the paper's D3Q27 directions 0..17 plus rest.  Weights are the standard
// ones quoted under eq:feq (D2Q9, D3Q27) and the textbook D3Q19 weights.
// --------------------------------------------------------------------------
struct Lattice {
  int D = 0, Q = 0;
  int c[27][3] = {};
  double w[27] = {};
  int opp[27] = {};
};

static Lattice make_lattice(int id) {
  Lattice L;
  static const int d2q9[9][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}, {-1, -1},
                                 {-1, 1}, {1, 1}, {1, -1}, {0, 0}};
  static const int d3q27[27][3] = {
      {-1, 0, 0},   {1, 0, 0},   {0, -1, 0},  {0, 1, 0},   {0, 0, -1},  {0, 0, 1},
      {-1, -1, 0},  {-1, 1, 0},  {1, -1, 0},  {1, 1, 0},   {-1, 0, -1}, {-1, 0, 1},
      {1, 0, -1},   {1, 0, 1},   {0, -1, -1}, {0, -1, 1},  {0, 1, -1},  {0, 1, 1},
      {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1}, {1, -1, 1},
      {1, 1, -1},   {1, 1, 1},   {0, 0, 0}};
  if (id == 0) {
    L.D = 2; L.Q = 9;
    for (int i = 0; i < 9; ++i) { L.c[i][0] = d2q9[i][0]; L.c[i][1] = d2q9[i][1]; L.c[i][2] = 0; }
  } else if (id == 1) {
    L.D = 3; L.Q = 19;
    for (int i = 0; i < 18; ++i) for (int a = 0; a < 3; ++a) L.c[i][a] = d3q27[i][a];
    for (int a = 0; a < 3; ++a) L.c[18][a] = 0;
  } else {
    L.D = 3; L.Q = 27;
    for (int i = 0; i < 27; ++i) for (int a = 0; a < 3; ++a) L.c[i][a] = d3q27[i][a];
  }
  for (int i = 0; i < L.Q; ++i) {
    int n2 = L.c[i][0] * L.c[i][0] + L.c[i][1] * L.c[i][1] + L.c[i][2] * L.c[i][2];
    if (id == 0) L.w[i] = (n2 == 0) ? 4.0 / 9.0 : (n2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
    else if (id == 1) L.w[i] = (n2 == 0) ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    else L.w[i] = (n2 == 0) ? 8.0 / 27.0 : (n2 == 1 ? 2.0 / 27.0 : (n2 == 2 ? 1.0 / 54.0 : 1.0 / 216.0));
  }
  for (int i = 0; i < L.Q; ++i)
    for (int j = 0; j < L.Q; ++j)
      if (L.c[j][0] == -L.c[i][0] && L.c[j][1] == -L.c[i][1] && L.c[j][2] == -L.c[i][2]) L.opp[i] = j;
  return L;
}

static int find_dir(const Lattice& L, int cx, int cy, int cz) {
  for (int i = 0; i < L.Q; ++i)
    if (L.c[i][0] == cx && L.c[i][1] == cy && L.c[i][2] == cz) return i;
  return -1;
}

static const double CS2 = 1.0 / 3.0;  // lattice speed of sound squared

// Equilibrium eq:feq.
template <class T>
static void equilibrium(const Lattice& L, const T& rho, const T u[3], T* feq) {
  T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < L.Q; ++i) {
    T cu = L.c[i][0] * u[0] + L.c[i][1] * u[1] + L.c[i][2] * u[2];
    feq[i] = L.w[i] * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
  }
}

// --------------------------------------------------------------------------
// Cumulant collision (Sec. 2.1, D3Q27): the populations are transformed into
// cumulants, every cumulant relaxes towards its value for the Maxwell
// distribution, c' = c + omega_alpha (c_eq - c), with the shear rate
// omega_1 = omega_BGK and every other rate one, and the result is
// transformed back.  The paper takes the operator from Geier et al. (2015);
// here it is written from the definitions:
//   * the 27 moments m_abc = sum_i c_ix^a c_iy^b c_iz^c f_i, a, b, c in
//     {0, 1, 2}, determine the 27 populations (a 27 x 27 linear system);
//   * the cumulant of index (a, b, c) is the joint cumulant of the variable
//     list (x a times, y b times, z c times) under the normalised
//     distribution f / rho, by the moment-cumulant formula over the set
//     partitions pi of the list,
//       kappa = sum_pi (-1)^(|pi| - 1) (|pi| - 1)! prod_{B in pi} E[prod_{j in B} X_j],
//     inverted by E[X_1 ... X_n] = sum_pi prod_{B in pi} kappa(B);
//   * the Maxwell distribution has first cumulants u, second cumulants
//     cs^2 delta_ab and no others.
// Relaxation groups: rho and u are conserved; the deviatoric part of the
// second-order cumulants relaxes with omega_1 (shear), their trace with
// omega_2 (bulk) and every cumulant of order three or more with its own
// rate; the paper sets every rate except omega_1 to one.  Reading: the body
// force enters as in the BGK operator (only the collision operator is
// exchanged, the discrete Boltzmann equation is kept).
// --------------------------------------------------------------------------
inline int midx(int a, int b, int c) { return 9 * a + 3 * b + c; }

// For every cumulant index (a, b, c), the moment-cumulant formula collected
// into terms coef * prod_j moment[idx_j] (partitions with the same multiset of
// block moments merged), and the inverse formula likewise.
struct CumulantTables {
  struct Term {
    double coef;
    std::vector<int> idx;
  };
  std::vector<Term> to_cum[27], to_mom[27];
  double Minv[27][27];  // populations from moments (D3Q27 directions)
};

static void set_partitions(int n, std::vector<std::vector<int>>& out) {
  // restricted growth strings: label[0] = 0, label[j] <= 1 + max(label[0..j-1])
  std::vector<int> lab(n, 0);
  std::function<void(int, int)> rec = [&](int j, int mx) {
    if (j == n) { out.push_back(lab); return; }
    for (int v = 0; v <= mx + 1; ++v) { lab[j] = v; rec(j + 1, std::max(mx, v)); }
  };
  if (n == 0) { out.push_back(lab); return; }
  lab[0] = 0;
  rec(1, 0);
}

static const CumulantTables& cumulant_tables() {
  static const CumulantTables T = [] {
    CumulantTables t;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c) {
          std::vector<int> var;
          for (int k = 0; k < a; ++k) var.push_back(0);
          for (int k = 0; k < b; ++k) var.push_back(1);
          for (int k = 0; k < c; ++k) var.push_back(2);
          const int n = (int)var.size();
          std::vector<std::vector<int>> parts;
          set_partitions(n, parts);
          std::map<std::vector<int>, double> cum, mom;
          for (const auto& lab : parts) {
            const int nb = n == 0 ? 0 : 1 + *std::max_element(lab.begin(), lab.end());
            std::vector<int> blocks;
            for (int B = 0; B < nb; ++B) {
              int cnt[3] = {0, 0, 0};
              for (int j = 0; j < n; ++j)
                if (lab[j] == B) ++cnt[var[j]];
              blocks.push_back(midx(cnt[0], cnt[1], cnt[2]));
            }
            std::sort(blocks.begin(), blocks.end());
            double fact = 1.0;
            for (int k = 2; k < nb; ++k) fact *= k;
            cum[blocks] += ((nb - 1) % 2 ? -1.0 : 1.0) * fact;
            mom[blocks] += 1.0;
          }
          const int m = midx(a, b, c);
          for (const auto& kv : cum)
            if (kv.second != 0.0) t.to_cum[m].push_back({kv.second, kv.first});
          for (const auto& kv : mom) t.to_mom[m].push_back({kv.second, kv.first});
        }
    // moment matrix of D3Q27 and its inverse (Gauss-Jordan, partial pivoting)
    const Lattice L = make_lattice(2);
    double M[27][54];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c)
          for (int i = 0; i < 27; ++i) {
            const int r = midx(a, b, c);
            M[r][i] = std::pow(L.c[i][0], a) * std::pow(L.c[i][1], b) * std::pow(L.c[i][2], c);
            M[r][27 + i] = (r == i) ? 1.0 : 0.0;
          }
    for (int col = 0; col < 27; ++col) {
      int piv = col;
      for (int r = col + 1; r < 27; ++r)
        if (std::fabs(M[r][col]) > std::fabs(M[piv][col])) piv = r;
      for (int k = 0; k < 54; ++k) std::swap(M[col][k], M[piv][k]);
      const double d = M[col][col];
      for (int k = 0; k < 54; ++k) M[col][k] /= d;
      for (int r = 0; r < 27; ++r) {
        if (r == col || M[r][col] == 0.0) continue;
        const double e = M[r][col];
        for (int k = 0; k < 54; ++k) M[r][k] -= e * M[col][k];
      }
    }
    for (int i = 0; i < 27; ++i)
      for (int r = 0; r < 27; ++r) t.Minv[i][r] = M[i][27 + r];
    return t;
  }();
  return T;
}

// Joint cumulants (index midx) of a normalised moment set m (m[0] = 1).
template <class T>
static void cumulants_from_moments(const T* m, T* kap) {
  const CumulantTables& t = cumulant_tables();
  kap[0] = m[0];
  for (int r = 1; r < 27; ++r) {
    T s = T(0.0);
    for (const auto& term : t.to_cum[r]) {
      T p = T(term.coef);
      for (int j : term.idx) p = p * m[j];
      s += p;
    }
    kap[r] = s;
  }
}

// Normalised moments from joint cumulants (kap[0] is ignored; m[0] = 1).
template <class T>
static void moments_from_cumulants(const T* kap, T* m) {
  const CumulantTables& t = cumulant_tables();
  for (int r = 0; r < 27; ++r) {
    T s = T(0.0);
    for (const auto& term : t.to_mom[r]) {
      T p = T(term.coef);
      for (int j : term.idx) p = p * kap[j];
      s += p;
    }
    m[r] = r == 0 ? T(1.0) : s;
  }
}

// Cumulant collision of one D3Q27 cell (rates: omega1 shear, omega2 bulk,
// omega3 every higher order; the paper's operator is omega2 = omega3 = 1)
// plus the first-order body force w_i rho (c_i . a) / cs^2.
template <class T>
static void cumulant_collide(const Lattice& L, const T* f, double omega1, double omega2, double omega3,
                             const double* acc, T* out) {
  const CumulantTables& t = cumulant_tables();
  T rho = T(0.0);
  for (int i = 0; i < 27; ++i) rho += f[i];
  T m[27], kap[27];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        T s = T(0.0);
        for (int i = 0; i < 27; ++i) {
          const double w = std::pow(L.c[i][0], a) * std::pow(L.c[i][1], b) * std::pow(L.c[i][2], c);
          if (w != 0.0) s += w * f[i];
        }
        m[midx(a, b, c)] = s / rho;
      }
  cumulants_from_moments(m, kap);
  // second order: trace (bulk) and deviatoric (shear) parts
  const int dg[3] = {midx(2, 0, 0), midx(0, 2, 0), midx(0, 0, 2)};
  const int od[3] = {midx(1, 1, 0), midx(1, 0, 1), midx(0, 1, 1)};
  const T tr = (kap[dg[0]] + kap[dg[1]] + kap[dg[2]]) / 3.0;
  T post[27];
  for (int r = 0; r < 27; ++r) post[r] = kap[r];
  const T tr_post = tr + omega2 * (CS2 - tr);
  for (int k = 0; k < 3; ++k) post[dg[k]] = tr_post + (1.0 - omega1) * (kap[dg[k]] - tr);
  for (int k = 0; k < 3; ++k) post[od[k]] = (1.0 - omega1) * kap[od[k]];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c)
        if (a + b + c >= 3) post[midx(a, b, c)] = (1.0 - omega3) * kap[midx(a, b, c)];
  T mp[27];
  moments_from_cumulants(post, mp);
  for (int i = 0; i < 27; ++i) {
    T s = T(0.0);
    for (int r = 0; r < 27; ++r) s += t.Minv[i][r] * mp[r];
    const double ca = L.c[i][0] * acc[0] + L.c[i][1] * acc[1] + L.c[i][2] * acc[2];
    out[i] = rho * s + L.w[i] * rho * ca / CS2;
  }
}

// --------------------------------------------------------------------------
// Parameters (layout mirrored by the Python ctypes binding of the oracle).
// Faces are ordered -x,+x,-y,+y,-z,+z.  Phase 0 is the liquid (phi < 0),
// phase 1 the gas (phi >= 0).
// --------------------------------------------------------------------------
enum { BC_PERIODIC = 0, BC_NOSLIP = 1, BC_FREESLIP = 2 };
// A face of a refined box: beyond it lies the coarser grid, which supplies
// the populations that cross the face (Sim::ghost); only the refinement
// driver below creates it.
constexpr int BC_INJECT = 3;
constexpr double BAND_SNAP = 1e-3;  // width of the band edge held at +-B (cells)

struct Params {
  int lattice, storage, nx, ny, nz;
  int bc[6];
  double wall_u[6][3];
  double rho_phys[2], tau[2];
  double accel[2][3];
  double sigma;
  double band;
  int n_ext;
  double ext_dtau;
  int reinit_every, n_reinit;
  double reinit_dtau;
  double heaviside_eps;
  int use_pb;
  double pb0;
  int init_hydrostatic;
  int fp16_scale_log2;
  int collision[2];  // per phase: 0 BGK, 1 cumulant (D3Q27 only)
};

// Tag bits used when exporting the classification.
enum { TAG_GAS = 1, TAG_ACTIVE = 2, TAG_IFACE = 4 };

// Heaviside smoothed over +-eps (the gas indicator of the integral
// quantities, Sec. 3.2); the smoothed form is the classical one of
// Sussman, Smereka and Osher (1994).
template <class T>
static T heaviside_mid(const T& phi, double eps) {
  const double pi = 3.14159265358979323846;
  return 0.5 * (1.0 + phi / eps + sin(pi * phi / eps) / pi);
}
template <class T>
static T heaviside(const T& phi, double eps) {
  if (val(phi) < -eps) return T(0.0);
  if (val(phi) > eps) return T(1.0);
  return heaviside_mid(phi, eps);
}

// --------------------------------------------------------------------------
// The simulation state and the step.
// --------------------------------------------------------------------------
template <class T>
struct Sim {
  Params P;
  Lattice L;
  int nx, ny, nz, D, Q;
  long N;
  double omega[2], eta[2];
  std::vector<T> A, An;                 // post-collision populations [i*N + cell]
  std::vector<T> phi;                   // level set
  std::vector<unsigned char> gas, act;  // phase and LS-active flag of the current step
  std::vector<unsigned char> gas1, act1;
  std::vector<T> Mr, Mu, MS;            // (rho, u, S) of the last collision, LS-active cells
  std::vector<T> Mr1, Mu1, MS1;         // the ones being written this step
  std::vector<T> nrm, kap;              // interface normal and curvature (LS-active cells)
  std::vector<T> ut, ut2;               // extension velocity
  std::vector<T> ghost;                 // [i*N + cell]: populations crossing an injected face
  T sig, Pb;
  // several bubbles (use_pb = 2): component of each cell in the support of
  // the smoothed Heaviside (-1 outside), the baseline of each cell's
  // component, and per component volume, centroid and baseline
  std::vector<int> bub;
  std::vector<T> pbc;
  std::vector<T> bvol, bxc, bpb;
  T xc0[3];
  long nstep = 0;
  bool all_active = false;              // component tests: treat every cell as LS-active
  // Decisions, for finite-difference checks of the frozen-decision
  // derivative.  Every branch that a value decides (tags, bounce-back
  // branch, upwind directions, clamp, refill direction and fallback,
  // Heaviside region, bubble labels, Godunov branches and subcell-fix set
  // of the reinitialisation) goes through decide(): its (site, outcome) is
  // folded into the deciding cell's word (each word is written by one
  // thread only), and the end of init and of every step folds the words and
  // the tags into one hash.  In record mode the outcomes and tags are also
  // kept; in replay mode a recorded run's outcomes and tags are imposed, so
  // a perturbed run takes exactly the recorded branches.
  struct DStep {
    std::vector<int> cells, start;  // cells with decisions, their first entry
    std::vector<unsigned char> site;
    std::vector<int> out;
    std::vector<unsigned char> tags;  // phase + 2 LS-active, one byte per cell
  };
  int dmode = 0;  // 0 hash only, 1 record, 2 replay
  mutable std::vector<uint64_t> dcell;
  mutable std::vector<std::vector<std::pair<unsigned char, int>>> dcur;
  std::shared_ptr<std::vector<DStep>> rlog;
  size_t rstep = 0;
  mutable std::vector<int> rcur, rend;
  mutable std::atomic<bool> rbad{false};
  std::vector<uint64_t> dlog;
  long decide(long c, unsigned site, long outcome) const {
    if (dmode == 2) {
      const DStep& d = (*rlog)[rstep];
      if (rcur[c] < rend[c] && d.site[rcur[c]] == site) outcome = d.out[rcur[c]++];
      else rbad = true;
    } else if (dmode == 1) {
      dcur[c].push_back({(unsigned char)site, (int)outcome});
    }
    dcell[c] = dcell[c] * 0x100000001B3ull + (uint64_t)site * 0x9E3779B97F4A7C15ull + (uint64_t)(outcome + 7);
    return outcome;
  }
  void begin_decisions() {
    if (dmode != 2) return;
    if (rstep >= rlog->size()) { rbad = true; return; }
    const DStep& d = (*rlog)[rstep];
    for (size_t k = 0; k < d.cells.size(); ++k) {
      rcur[d.cells[k]] = d.start[k];
      rend[d.cells[k]] = (k + 1 < d.cells.size()) ? d.start[k + 1] : (int)d.out.size();
    }
  }
  // tags of the classification: recorded, or imposed from the record
  void decide_tags(std::vector<unsigned char>& g, std::vector<unsigned char>& a) {
    if (dmode == 1) {
      dtags.resize(N);
      for (long c = 0; c < N; ++c) dtags[c] = (unsigned char)(g[c] + 2 * a[c]);
    } else if (dmode == 2 && rstep < rlog->size()) {
      const std::vector<unsigned char>& t = (*rlog)[rstep].tags;
      for (long c = 0; c < N; ++c) { g[c] = t[c] & 1; a[c] = (t[c] >> 1) & 1; }
    }
  }
  std::vector<unsigned char> dtags;
  void fold_decisions() {
    uint64_t h = 0xCBF29CE484222325ull;
    for (long c = 0; c < N; ++c) {
      h = (h ^ dcell[c]) * 0x100000001B3ull;
      h = (h ^ (uint64_t)(gas[c] + 2 * act[c])) * 0x100000001B3ull;
      dcell[c] = 0;
    }
    dlog.push_back(h);
    if (dmode == 1) {
      DStep d;
      for (long c = 0; c < N; ++c) {
        if (dcur[c].empty()) continue;
        d.cells.push_back((int)c);
        d.start.push_back((int)d.out.size());
        for (auto& e : dcur[c]) { d.site.push_back(e.first); d.out.push_back(e.second); }
        dcur[c].clear();
      }
      d.tags.swap(dtags);
      rlog->push_back(std::move(d));
    } else if (dmode == 2 && rstep < rlog->size()) {
      const DStep& d = (*rlog)[rstep];
      for (size_t k = 0; k < d.cells.size(); ++k) {
        const long c = d.cells[k];
        if (rcur[c] != rend[c]) rbad = true;  // recorded decisions left over
        rcur[c] = rend[c] = 0;
      }
      ++rstep;
    }
  }
  void set_decision_mode(int mode, const std::shared_ptr<std::vector<DStep>>& src) {
    dmode = mode;
    if (mode == 1) { rlog = std::make_shared<std::vector<DStep>>(); dcur.assign(N, {}); }
    if (mode == 2) { rlog = src; rstep = 0; rcur.assign(N, 0); rend.assign(N, 0); }
  }

  explicit Sim(const Params& p) : P(p) {
    L = make_lattice(p.lattice);
    nx = p.nx; ny = p.ny; nz = p.nz;
    D = L.D; Q = L.Q;
    N = (long)nx * ny * nz;
    for (int k = 0; k < 2; ++k) {
      // eq:omega with dt = dx = 1: omega = cs^2 / (nu + cs^2 / 2) = 1 / tau.
      double nu = CS2 * (p.tau[k] - 0.5);
      omega[k] = CS2 / (nu + 0.5 * CS2);
      eta[k] = p.rho_phys[k] * nu;  // dynamic viscosity eta = rho nu (Sec. 2.3)
    }
    A.assign((size_t)Q * N, T(0.0)); An = A;
    phi.assign(N, T(0.0));
    gas.assign(N, 0); act.assign(N, 0); gas1 = gas; act1 = act;
    Mr.assign(N, T(1.0)); Mu.assign(3 * N, T(0.0)); MS.assign(6 * N, T(0.0));
    Mr1 = Mr; Mu1 = Mu; MS1 = MS;
    nrm.assign(3 * N, T(0.0)); kap.assign(N, T(0.0));
    ut.assign(3 * N, T(0.0)); ut2 = ut;
    dcell.assign(N, 0);
    sig = T(p.sigma); Pb = T(p.pb0);
    for (int a = 0; a < 3; ++a) xc0[a] = T(0.0);
  }

  long idx(int x, int y, int z) const { return ((long)z * ny + y) * nx + x; }
  void coords(long c, int& x, int& y, int& z) const {
    x = (int)(c % nx); y = (int)((c / nx) % ny); z = (int)(c / ((long)nx * ny));
  }
  int ext(int a) const { return a == 0 ? nx : (a == 1 ? ny : nz); }

  // Lattice neighbour c + d.  Periodic axes wrap; returns false when the
  // displacement leaves the domain through a wall face.
  bool nb(int x, int y, int z, int dx, int dy, int dz, long& out) const {
    int s[3] = {x + dx, y + dy, z + dz};
    for (int a = 0; a < 3; ++a) {
      int n = ext(a);
      if (s[a] < 0 || s[a] >= n) {
        if (P.bc[2 * a] != BC_PERIODIC) return false;
        s[a] = (s[a] % n + n) % n;
      }
    }
    out = idx(s[0], s[1], s[2]);
    return true;
  }

  // Level-set stencil neighbour: periodic axes wrap, wall faces mirror the
  // level set evenly about the face (reading, the paper does not say).
  long ls_nb(int x, int y, int z, int dx, int dy, int dz) const {
    int s[3] = {x + dx, y + dy, z + dz};
    for (int a = 0; a < 3; ++a) {
      int n = ext(a);
      if (s[a] >= 0 && s[a] < n) continue;
      if (P.bc[2 * a] == BC_PERIODIC) s[a] = (s[a] % n + n) % n;
      else if (s[a] < 0) s[a] = -1 - s[a];
      else s[a] = 2 * n - 1 - s[a];
    }
    return idx(s[0], s[1], s[2]);
  }

  bool is_act(long c) const { return all_active || act[c]; }

  // Phase pressures.  Each phase solver keeps its own LB density near 1; the
  // physical density enters through p = rho_phys cs^2 (rho_LB - 1) (reading:
  // the paper does not say how the density ratio is represented).  The gas
  // carries the pressure baseline: Pb, or with several bubbles the baseline
  // of the bubble the cell c belongs to.
  T baseline(long c) const { return P.use_pb == 2 ? pbc[c] : Pb; }
  T pressure(int k, const T& rho, long c) const {
    T p = P.rho_phys[k] * CS2 * (rho - 1.0);
    if (k == 1) p = p + baseline(c);
    return p;
  }

  // ------------------------------------------------------------------
  // Interface bounce-back (eq:bb with the momentum term eq:bb_cc).
  // Own cell c (phase k) pulls direction i from s = c - c_i which lies in
  // the other phase.  The link seen from c points along -c_i; the
  // population travelling towards the interface is A_j(c), j = opp(i), and
  // the missing one is f_i(c).
  // ------------------------------------------------------------------
  T interface_bb(long c, int x, int y, int z, long s, int i, int k) const {
    const int* ci = L.c[i];
    const int j = L.opp[i];
    // Wall distance from the radiation theorem (Sec. 2.3).
    T q = phi[c] / (phi[c] - phi[s]);
    // Interface velocity: linear interpolation between both phases (Sec. 2.3),
    // with the moments of the previous collision.
    T uG[3];
    for (int a = 0; a < 3; ++a) uG[a] = (1.0 - q) * Mu[3 * c + a] + q * Mu[3 * s + a];
    // Geometry at the link point.
    T nG[3], nn = T(0.0);
    for (int a = 0; a < 3; ++a) { nG[a] = (1.0 - q) * nrm[3 * c + a] + q * nrm[3 * s + a]; nn += nG[a] * nG[a]; }
    T nl = sqrt(nn);
    if (val(nl) > 1e-300) for (int a = 0; a < 3; ++a) nG[a] = nG[a] / nl;
    T kG = (1.0 - q) * kap[c] + q * kap[s];
    // Pressures carried to the link point with each phase's own body
    // acceleration (hydrostatic shift; reading).
    const int o = 1 - k;
    T p_own = pressure(k, Mr[c], c);
    T p_oth = pressure(o, Mr[s], s);
    for (int a = 0; a < 3; ++a) {
      p_own = p_own + P.rho_phys[k] * P.accel[k][a] * (-(double)ci[a]) * q;
      p_oth = p_oth + P.rho_phys[o] * P.accel[o][a] * (double)ci[a] * (1.0 - q);
    }
    T p_l = (k == 0) ? p_own : p_oth;
    T p_g = (k == 0) ? p_oth : p_own;
    // Stress-jump (eq:Sdecomp).  Reading: the Laplace term is sigma*kappa
    // with kappa = div n (the total curvature), and the operand missing after
    // [eta]/eta_bar is the phase-averaged strain rate S_bar, so that
    // [eta S] = eta_bar [S] + [eta] S_bar.  The tangential-tangential jump is
    // zero because the velocity is continuous.
    const double eta_bar = 0.5 * (eta[0] + eta[1]);
    const double jeta = eta[1] - eta[0];
    // The pressure part of the normal jump acts as an explicit feedback with
    // a one-step lag (E uses the moments of the previous collision): one step
    // changes an interface cell's pressure by k Delta with
    // k = rho cs^2 q(1-q) sum_i 6 w_i (c_i.n)^2 / (2 eta) <= rho / (24 eta),
    // and the lagged iteration x' = x - k x_prev has roots of modulus sqrt(k),
    // so it can diverge only for k > 1, i.e. eta_bar < rho_max / 24.
    // Reading: where eta_bar >= rho_max / 24 the bound keeps k <= 1 and the
    // divisor is eq:Sdecomp's own eta_bar; below it (every workload with tau
    // near 1/2 and a large density ratio) the divisor is raised to
    // rho_max cs^2 / 4, which bounds k by 1/2 (roots of modulus 0.71).
    const double rho_max = std::max(P.rho_phys[0], P.rho_phys[1]);
    const double eta_p = eta_bar >= rho_max / 24.0 ? eta_bar : rho_max * CS2 / 4.0;
    T E = ((p_g - p_l) + sig * kG) / (2.0 * eta_p);
    T Sb[6];
    for (int m = 0; m < 6; ++m) Sb[m] = 0.5 * (MS[6 * c + m] + MS[6 * s + m]);
    const double acoef = -jeta / eta_bar;
    // full symmetric tensors from (xx, yy, zz, xy, xz, yz)
    T Sm[3][3] = {{Sb[0], Sb[3], Sb[4]}, {Sb[3], Sb[1], Sb[5]}, {Sb[4], Sb[5], Sb[2]}};
    T cn = ci[0] * nG[0] + ci[1] * nG[1] + ci[2] * nG[2];
    T nAn = T(0.0), nAc = T(0.0);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        nAn = nAn + acoef * nG[a] * Sm[a][b] * nG[b];
        nAc = nAc + acoef * nG[a] * Sm[a][b] * (double)ci[b];
      }
    // c.[S].c: normal-normal part E + n.A.n, normal-tangential part from A.
    T cSc = cn * cn * E + 2.0 * cn * nAc - cn * cn * nAn;
    // Momentum term.  Reading of eq:bb_cc: Lambda_i = c_i c_i, and the sign is
    // that of the jump (other - own): +1 seen from the liquid, -1 from the
    // gas.  The reflected population gains 2 w (c_i . u_G)/cs^2 as for a wall
    // moving with u_G.
    const double s_own = (k == 0) ? 1.0 : -1.0;
    T cu = ci[0] * uG[0] + ci[1] * uG[1] + ci[2] * uG[2];
    T W = (2.0 * L.w[i] / CS2) * (cu + q * (1.0 - q) * s_own * cSc);
    // Interpolated bounce-back, eq:bb.  Reading of the q >= 1/2 branch: the
    // second population is the reflected one at the cell itself (Bouzidi's
    // linear interpolation), which keeps both branches equal at q = 1/2.
    long far = 0;
    const bool far_in = nb(x, y, z, ci[0], ci[1], ci[2], far) && gas[far] == k;
    const long br = decide(c, 1, val(q) < 0.5 ? (far_in ? 1 : 2) : 0);
    if (br == 1) return 2.0 * q * A[(size_t)j * N + c] + (1.0 - 2.0 * q) * A[(size_t)j * N + far] + W;
    if (br == 2) return A[(size_t)j * N + c] + W;  // thin film: halfway bounce-back
    return A[(size_t)j * N + c] / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * A[(size_t)i * N + c] +
           W / (2.0 * q);
  }

  // Incoming population f_i at cell c (pull streaming, Eq. 1).
  T pull(long c, int x, int y, int z, int i, int k) const {
    const int* ci = L.c[i];
    int s[3] = {x - ci[0], y - ci[1], z - ci[2]};
    bool cross[3] = {false, false, false};
    int face[3] = {0, 0, 0};
    bool any = false;
    for (int a = 0; a < 3; ++a) {
      int n = ext(a);
      if (s[a] >= 0 && s[a] < n) continue;
      if (P.bc[2 * a] == BC_PERIODIC) { s[a] = (s[a] % n + n) % n; continue; }
      cross[a] = true; face[a] = (s[a] < 0) ? 2 * a : 2 * a + 1; any = true;
    }
    if (any) {
      // Across the face of a refined box: the coarser grid's population.
      for (int a = 0; a < 3; ++a)
        if (cross[a] && P.bc[face[a]] == BC_INJECT) return ghost[(size_t)i * N + c];
      // Walls lie on cell faces: halfway bounce-back (q = 1/2) with the
      // moving-wall term of Sec. 2.1 for no-slip faces, specular reflection
      // for free-slip faces.  A link crossing any no-slip face is no-slip.
      for (int a = 0; a < 3; ++a)
        if (cross[a] && P.bc[face[a]] == BC_NOSLIP) {
          const double* uw = P.wall_u[face[a]];
          double cu = ci[0] * uw[0] + ci[1] * uw[1] + ci[2] * uw[2];
          return A[(size_t)L.opp[i] * N + c] + 2.0 * L.w[i] * cu / CS2;
        }
      int cr[3];
      for (int a = 0; a < 3; ++a) { cr[a] = cross[a] ? -ci[a] : ci[a]; if (cross[a]) s[a] = (a == 0 ? x : (a == 1 ? y : z)); }
      int ir = find_dir(L, cr[0], cr[1], cr[2]);
      long src = idx(s[0], s[1], s[2]);
      if (gas[src] != k) return A[(size_t)L.opp[i] * N + c];  // reflected source across the interface
      return A[(size_t)ir * N + src];
    }
    long src = idx(s[0], s[1], s[2]);
    if (gas[src] == k) return A[(size_t)i * N + src];
    return interface_bb(c, x, y, z, src, i, k);
  }

  // ------------------------------------------------------------------
  // a2-a4: fused collide and stream of each phase with wall and interface
  // bounce-back.  Writes An and, on LS-active cells, M1 = (rho, u, S).
  // ------------------------------------------------------------------
  void lb_step() {
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
      int x, y, z;
      coords(c, x, y, z);
      const int k = gas[c];
      T f[27], feq[27];
      for (int i = 0; i < Q; ++i) f[i] = pull(c, x, y, z, i, k);
      // Moments (eq:macro).
      T rho = T(0.0), m[3] = {T(0.0), T(0.0), T(0.0)};
      for (int i = 0; i < Q; ++i) {
        rho += f[i];
        for (int a = 0; a < 3; ++a) m[a] += (double)L.c[i][a] * f[i];
      }
      T u[3] = {m[0] / rho, m[1] / rho, m[2] / rho};
      equilibrium(L, rho, u, feq);
      const double om = omega[k];
      // Strain rate from the non-equilibrium second moment (textbook
      // Chapman-Enskog relation; the paper does not say how S is found):
      // S_ab = -omega / (2 rho cs^2) sum_i c_ia c_ib (f_i - f_i^eq).
      if (is_act(c)) {
        T Pi[6] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)};
        for (int i = 0; i < Q; ++i) {
          T fn = f[i] - feq[i];
          const int* ci = L.c[i];
          Pi[0] += (double)(ci[0] * ci[0]) * fn; Pi[1] += (double)(ci[1] * ci[1]) * fn;
          Pi[2] += (double)(ci[2] * ci[2]) * fn; Pi[3] += (double)(ci[0] * ci[1]) * fn;
          Pi[4] += (double)(ci[0] * ci[2]) * fn; Pi[5] += (double)(ci[1] * ci[2]) * fn;
        }
        T fac = -om / (2.0 * rho * CS2);
        Mr1[c] = rho;
        for (int a = 0; a < 3; ++a) Mu1[3 * c + a] = u[a];
        for (int mm = 0; mm < 6; ++mm) MS1[6 * c + mm] = fac * Pi[mm];
      }
      // BGK collision plus the first-order body force of Sec. 2.1 written for
      // a general acceleration a_k: F_i = w_i rho (c_i . a_k) / cs^2; or the
      // cumulant collision with the same force.
      const double* acc = P.accel[k];
      if (P.collision[k] == 1) {
        T post[27];
        cumulant_collide(L, f, om, 1.0, 1.0, acc, post);
        for (int i = 0; i < Q; ++i) An[(size_t)i * N + c] = post[i];
        continue;
      }
      for (int i = 0; i < Q; ++i) {
        double ca = L.c[i][0] * acc[0] + L.c[i][1] * acc[1] + L.c[i][2] * acc[2];
        An[(size_t)i * N + c] = f[i] - om * (f[i] - feq[i]) + L.w[i] * rho * ca / CS2;
      }
    }
  }

  // Cell c has a lattice link to a cell of the other phase (interface cell).
  bool is_iface(long c, int x, int y, int z, const std::vector<unsigned char>& ph) const {
    for (int i = 0; i < Q; ++i) {
      if (L.c[i][0] == 0 && L.c[i][1] == 0 && L.c[i][2] == 0) continue;
      long s;
      if (nb(x, y, z, -L.c[i][0], -L.c[i][1], -L.c[i][2], s) && ph[s] != ph[c]) return true;
    }
    return false;
  }

  // ------------------------------------------------------------------
  // a6 part 1: hyperbolic velocity extension (eq:hyperbolicExtension).
  // Seed: on interface cells the mean over their interface links of the
  // linearly interpolated interface velocity; elsewhere in the band the
  // cell's own fluid velocity.  Then n_ext forward-Euler steps of the
  // first-order upwind discretisation with v = S(phi) n, interface cells
  // held fixed, zero gradient towards cells outside the band.  The smoothed
  // sign S(phi) = phi / sqrt(phi^2 + 1) is Peng et al. (1999).
  // ------------------------------------------------------------------
  void extension() {
    std::vector<unsigned char> icell(N, 0);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
      if (!is_act(c)) continue;
      int x, y, z;
      coords(c, x, y, z);
      T acc[3] = {T(0.0), T(0.0), T(0.0)};
      int cnt = 0;
      for (int i = 0; i < Q; ++i) {
        const int* ci = L.c[i];
        if (ci[0] == 0 && ci[1] == 0 && ci[2] == 0) continue;
        long s;
        if (!nb(x, y, z, -ci[0], -ci[1], -ci[2], s) || gas[s] == gas[c]) continue;
        T q = phi[c] / (phi[c] - phi[s]);
        for (int a = 0; a < 3; ++a) acc[a] += (1.0 - q) * Mu1[3 * c + a] + q * Mu1[3 * s + a];
        ++cnt;
      }
      if (cnt > 0) {
        icell[c] = 1;
        for (int a = 0; a < 3; ++a) ut[3 * c + a] = acc[a] / (double)cnt;
      } else {
        for (int a = 0; a < 3; ++a) ut[3 * c + a] = Mu1[3 * c + a];
      }
    }
    extension_iterate(icell);
  }

  // n_ext Jacobi sweeps of the upwind extension; cells with icell set are held.
  void extension_iterate(const std::vector<unsigned char>& icell) {
    for (int it = 0; it < P.n_ext; ++it) {
#pragma omp parallel for schedule(static)
      for (long c = 0; c < N; ++c) {
        if (!is_act(c)) continue;
        for (int a = 0; a < 3; ++a) ut2[3 * c + a] = ut[3 * c + a];
        if (icell[c]) continue;
        int x, y, z;
        coords(c, x, y, z);
        T sg = phi[c] / sqrt(phi[c] * phi[c] + 1.0);
        for (int ax = 0; ax < D; ++ax) {
          T v = sg * nrm[3 * c + ax];
          const long sv = decide(c, 2, val(v) > 0.0 ? 1 : (val(v) < 0.0 ? -1 : 0));
          if (sv == 0) continue;
          const int d = sv > 0 ? -1 : 1;  // towards the upwind neighbour
          int e[3] = {0, 0, 0};
          e[ax] = d;
          long s;
          // Upwind neighbour's velocity.  Across a free-slip face the face is
          // a mirror plane: the neighbour is the cell's own image, with the
          // component normal to the face reversed.  Across a no-slip face,
          // or towards a cell outside the band, the axis is skipped (zero
          // gradient).  (Reading: the paper does not treat walls here.)
          T un[3];
          if (nb(x, y, z, e[0], e[1], e[2], s)) {
            if (!is_act(s)) continue;
            for (int a = 0; a < 3; ++a) un[a] = ut[3 * s + a];
          } else {
            if (P.bc[2 * ax + (d > 0 ? 1 : 0)] != BC_FREESLIP) continue;
            for (int a = 0; a < 3; ++a) un[a] = (a == ax) ? -ut[3 * c + a] : ut[3 * c + a];
          }
          for (int a = 0; a < 3; ++a)
            ut2[3 * c + a] -= P.ext_dtau * v * (d < 0 ? ut[3 * c + a] - un[a] : un[a] - ut[3 * c + a]);
        }
      }
      std::swap(ut, ut2);
    }
  }

  // Fifth-order upwind-biased first derivative along axis ax at cell c
  // ("fifth-order upwind-central", Sec. 2.2; reading: the linear six-point
  // upwind-biased stencil, exact for polynomials of degree five).
  T d_upwind5(const std::vector<T>& ph, int x, int y, int z, int ax, bool positive) const {
    auto at = [&](int o) {
      int e[3] = {0, 0, 0};
      e[ax] = o;
      return ph[ls_nb(x, y, z, e[0], e[1], e[2])];
    };
    if (positive)
      return (-2.0 * at(-3) + 15.0 * at(-2) - 60.0 * at(-1) + 20.0 * at(0) + 30.0 * at(1) - 3.0 * at(2)) / 60.0;
    return (3.0 * at(-2) - 30.0 * at(-1) - 20.0 * at(0) + 60.0 * at(1) - 15.0 * at(2) + 2.0 * at(3)) / 60.0;
  }

  // Right-hand side of the transport equation, L = -u~ . grad phi.
  void advect_rate(const std::vector<T>& ph, std::vector<T>& out) const {
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
      if (!is_act(c)) { out[c] = T(0.0); continue; }
      int x, y, z;
      coords(c, x, y, z);
      T r = T(0.0);
      for (int ax = 0; ax < D; ++ax) {
        T u = ut[3 * c + ax];
        const bool up = decide(c, 3, val(u) >= 0.0) != 0;
        r = r - u * d_upwind5(ph, x, y, z, ax, up);
      }
      out[c] = r;
    }
  }

  // a6 part 2: three-stage TVD Runge-Kutta (Shu and Osher) of the transport
  // equation over one LB time step, on the band only, then the band clamp.
  void advect() {
    std::vector<T> r(N), p1 = phi, p2 = phi;
    advect_rate(phi, r);
    for (long c = 0; c < N; ++c) if (is_act(c)) p1[c] = phi[c] + r[c];
    advect_rate(p1, r);
    for (long c = 0; c < N; ++c) if (is_act(c)) p2[c] = 0.75 * phi[c] + 0.25 * (p1[c] + r[c]);
    advect_rate(p2, r);
    for (long c = 0; c < N; ++c) if (is_act(c)) phi[c] = (1.0 / 3.0) * phi[c] + (2.0 / 3.0) * (p2[c] + r[c]);
    clamp_band();
  }

  // The band's edge is held at exactly +-B: a value beyond B - BAND_SNAP
  // (in magnitude) is set to +-B (reading: the paper's narrow band has an
  // edge; holding it exactly keeps sub-rounding drifts of the edge cells,
  // which a reduced-precision level set cannot follow, out of the
  // reinitialisation stencils that reach the edge).
  void clamp_band() {
    const double B = P.band;
    const double Bs = B - BAND_SNAP;
    for (long c = 0; c < N; ++c) {
      if (!is_act(c)) continue;
      const long cl = decide(c, 4, val(phi[c]) > Bs ? 1 : (val(phi[c]) < -Bs ? -1 : 0));
      if (cl > 0) phi[c] = T(B);
      if (cl < 0) phi[c] = T(-B);
    }
  }

  // HJ-WENO5 one-sided derivative from five consecutive differences
  // (Jiang and Peng 2000, the standard Hamilton-Jacobi WENO weights).
  static T weno5(const T& v1, const T& v2, const T& v3, const T& v4, const T& v5) {
    const double eps = 1e-6;
    T p0 = v1 / 3.0 - 7.0 * v2 / 6.0 + 11.0 * v3 / 6.0;
    T p1 = -v2 / 6.0 + 5.0 * v3 / 6.0 + v4 / 3.0;
    T p2 = v3 / 3.0 + 5.0 * v4 / 6.0 - v5 / 6.0;
    T a0 = v1 - 2.0 * v2 + v3, b0 = v1 - 4.0 * v2 + 3.0 * v3;
    T a1 = v2 - 2.0 * v3 + v4, b1 = v2 - v4;
    T a2 = v3 - 2.0 * v4 + v5, b2 = 3.0 * v3 - 4.0 * v4 + v5;
    T s0 = 13.0 / 12.0 * a0 * a0 + 0.25 * b0 * b0;
    T s1 = 13.0 / 12.0 * a1 * a1 + 0.25 * b1 * b1;
    T s2 = 13.0 / 12.0 * a2 * a2 + 0.25 * b2 * b2;
    T w0 = 0.1 / ((eps + s0) * (eps + s0));
    T w1 = 0.6 / ((eps + s1) * (eps + s1));
    T w2 = 0.3 / ((eps + s2) * (eps + s2));
    return (w0 * p0 + w1 * p1 + w2 * p2) / (w0 + w1 + w2);
  }

  // ------------------------------------------------------------------
  // a7: constrained reinitialisation.  The paper cites Hartmann et al.
  // (2010) without reproducing it.  Reading: pseudo-time integration of
  // phi_tau = -S(phi0)(|grad phi| - 1) with the Godunov Hamiltonian of HJ-WENO5
  // one-sided derivatives and TVD-RK3 in pseudo time; on the cells next to the
  // zero set (an axis neighbour of the other sign in phi0) a forcing term
  // beta (phi~ - phi) holds the zero crossings in place, where
  // phi~_i = mean_j phi0_i (phi_i - phi_j) / (phi0_i - phi0_j) over those
  // neighbours j keeps each crossing ratio phi_i / (phi_i - phi_j) equal to
  // the one of phi0.  A signed-distance field is a fixed point.  phi0, S(phi0)
  // and the constrained cells stay frozen over the n_reinit pseudo steps.
  // ------------------------------------------------------------------
  void reinit() {
    const std::vector<T> p0 = phi;
    const double beta = 0.5;
    std::vector<unsigned char> fix(N, 0);
    std::vector<int> fixmask(N, 0);  // neighbours across the zero set of phi0, per (axis, side)
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
      if (!is_act(c)) continue;
      int x, y, z;
      coords(c, x, y, z);
      bool g0 = val(p0[c]) >= 0.0;
      long mask = 0;
      for (int ax = 0; ax < D; ++ax)
        for (int sgn = -1; sgn <= 1; sgn += 2) {
          int e[3] = {0, 0, 0};
          e[ax] = sgn;
          if ((val(p0[ls_nb(x, y, z, e[0], e[1], e[2])]) >= 0.0) != g0) mask |= 1L << (2 * ax + (sgn > 0));
        }
      fixmask[c] = (int)decide(c, 9, mask);
      fix[c] = fixmask[c] != 0;
    }
    std::vector<T> r(N), p1(N), p2(N);
    auto rate = [&](const std::vector<T>& ph, std::vector<T>& out) {
#pragma omp parallel for schedule(static)
      for (long c = 0; c < N; ++c) {
        if (!is_act(c)) { out[c] = T(0.0); continue; }
        int x, y, z;
        coords(c, x, y, z);
        T S0 = p0[c] / sqrt(p0[c] * p0[c] + 1.0);
        T h2 = T(0.0);
        // Godunov branches, four bits per axis: sign of S(phi0), the kept
        // one-sided derivatives (nonzero or clipped) and the larger one
        T dms[3], dps[3];
        long code = 0;
        for (int ax = 0; ax < D; ++ax) {
          auto at = [&](int o) {
            int e[3] = {0, 0, 0};
            e[ax] = o;
            return ph[ls_nb(x, y, z, e[0], e[1], e[2])];
          };
          T m3 = at(-3), m2 = at(-2), m1 = at(-1), c0 = at(0), p1v = at(1), p2v = at(2), p3 = at(3);
          dms[ax] = weno5(m2 - m3, m1 - m2, c0 - m1, p1v - c0, p2v - p1v);
          dps[ax] = weno5(p3 - p2v, p2v - p1v, p1v - c0, c0 - m1, m1 - m2);
          const bool pos = val(S0) > 0.0;
          const bool ka = pos ? val(dms[ax]) > 0.0 : val(dms[ax]) < 0.0;
          const bool kb = pos ? val(dps[ax]) < 0.0 : val(dps[ax]) > 0.0;
          const double av = ka ? val(dms[ax]) : 0.0, bv = kb ? val(dps[ax]) : 0.0;
          code |= (long)((pos ? 1 : 0) | (ka ? 2 : 0) | (kb ? 4 : 0) | (av * av > bv * bv ? 8 : 0)) << (4 * ax);
        }
        code = decide(c, 8, code);
        for (int ax = 0; ax < D; ++ax) {
          const long bits = (code >> (4 * ax)) & 15;
          T a = (bits & 2) ? dms[ax] : T(0.0);
          T b = (bits & 4) ? dps[ax] : T(0.0);
          h2 = h2 + ((bits & 8) ? a * a : b * b);
        }
        T rt = -S0 * (sqrt(h2) - 1.0);
        if (fix[c]) {
          T acc = T(0.0);
          int cnt = 0;
          for (int ax = 0; ax < D; ++ax)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
              int e[3] = {0, 0, 0};
              e[ax] = sgn;
              long j = ls_nb(x, y, z, e[0], e[1], e[2]);
              if (!(fixmask[c] & (1 << (2 * ax + (sgn > 0))))) continue;
              acc = acc + p0[c] * (ph[c] - ph[j]) / (p0[c] - p0[j]);
              ++cnt;
            }
          rt = rt + beta * (acc / (double)cnt - ph[c]);
        }
        out[c] = rt;
      }
    };
    const double dt = P.reinit_dtau;
    for (int it = 0; it < P.n_reinit; ++it) {
      p1 = phi; p2 = phi;
      rate(phi, r);
      for (long c = 0; c < N; ++c) if (is_act(c)) p1[c] = phi[c] + dt * r[c];
      rate(p1, r);
      for (long c = 0; c < N; ++c) if (is_act(c)) p2[c] = 0.75 * phi[c] + 0.25 * (p1[c] + dt * r[c]);
      rate(p2, r);
      for (long c = 0; c < N; ++c) if (is_act(c)) phi[c] = (1.0 / 3.0) * phi[c] + (2.0 / 3.0) * (p2[c] + dt * r[c]);
    }
    clamp_band();
  }

  // ------------------------------------------------------------------
  // a5: normal n = grad phi / |grad phi| and curvature kappa = div n
  // (Sec. 2.2) with second-order central differences at cell centres.
  // ------------------------------------------------------------------
  void geometry() {
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
      if (!is_act(c)) continue;
      int x, y, z;
      coords(c, x, y, z);
      auto at = [&](int dx, int dy, int dz) { return phi[ls_nb(x, y, z, dx, dy, dz)]; };
      T p = phi[c];
      T gx = 0.5 * (at(1, 0, 0) - at(-1, 0, 0));
      T gy = 0.5 * (at(0, 1, 0) - at(0, -1, 0));
      T gz = T(0.0), zz = T(0.0), xz = T(0.0), yz = T(0.0);
      T xx = at(1, 0, 0) - 2.0 * p + at(-1, 0, 0);
      T yy = at(0, 1, 0) - 2.0 * p + at(0, -1, 0);
      T xy = 0.25 * (at(1, 1, 0) - at(1, -1, 0) - at(-1, 1, 0) + at(-1, -1, 0));
      if (D == 3) {
        gz = 0.5 * (at(0, 0, 1) - at(0, 0, -1));
        zz = at(0, 0, 1) - 2.0 * p + at(0, 0, -1);
        xz = 0.25 * (at(1, 0, 1) - at(1, 0, -1) - at(-1, 0, 1) + at(-1, 0, -1));
        yz = 0.25 * (at(0, 1, 1) - at(0, 1, -1) - at(0, -1, 1) + at(0, -1, -1));
      }
      T g2 = gx * gx + gy * gy + gz * gz;
      T g = sqrt(g2);
      if (val(g) < 1e-12) {
        for (int a = 0; a < 3; ++a) nrm[3 * c + a] = T(0.0);
        kap[c] = T(0.0);
        continue;
      }
      nrm[3 * c + 0] = gx / g; nrm[3 * c + 1] = gy / g; nrm[3 * c + 2] = gz / g;
      T num = xx * (gy * gy + gz * gz) + yy * (gx * gx + gz * gz) + zz * (gx * gx + gy * gy) -
              2.0 * gx * gy * xy - 2.0 * gx * gz * xz - 2.0 * gy * gz * yz;
      kap[c] = num / (g2 * g);
    }
  }

  // Phase and band classification from phi: gas where phi >= 0 (phi = 0
  // counts as gas, reading); LS-active where some cell of the 3^d box around
  // the cell has |phi| < band.
  void classify(std::vector<unsigned char>& g, std::vector<unsigned char>& a) const {
    const double B = P.band;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
      int x, y, z;
      coords(c, x, y, z);
      g[c] = val(phi[c]) >= 0.0 ? 1 : 0;
      bool on = false;
      int zr = (D == 3) ? 1 : 0;
      for (int dz = -zr; dz <= zr && !on; ++dz)
        for (int dy = -1; dy <= 1 && !on; ++dy)
          for (int dx = -1; dx <= 1 && !on; ++dx) {
            long s;
            if (!nb(x, y, z, dx, dy, dz, s)) continue;
            if (std::fabs(val(phi[s])) < B) on = true;
          }
      a[c] = on ? 1 : 0;
    }
  }

  // ------------------------------------------------------------------
  // a8: refill of cells whose phase changed (Sec. 2.4).
  // Readings: e_min is the lattice direction best aligned with the normal
  // pointing into the new phase (the figure and caption; the printed argmin
  // would point out of it), ties to the lowest index; the third Lagrange
  // weight is -q/(q+2) (the printed +2q/(q+2) does not sum to one); the
  // boundary values are the old phase's moments at the cell with the
  // Laplace jump applied to the pressure; f^neq is the stored
  // (post-collision) population minus the equilibrium of the neighbour's
  // last moments.
  // ------------------------------------------------------------------
  static void refill_weights(double q, double Lw[3]) {
    Lw[0] = 2.0 / ((q + 1.0) * (q + 2.0));
    Lw[1] = 2.0 * q / (q + 1.0);
    Lw[2] = -q / (q + 2.0);
  }

  void refill() {
    // Reads An / Mr1,Mu1,MS1 of established cells only and writes flipped
    // cells only, so the cell order is irrelevant.
    for (long c = 0; c < N; ++c) {
      if (gas1[c] == gas[c]) continue;
      int x, y, z;
      coords(c, x, y, z);
      const int knew = gas1[c];
      const int kold = gas[c];
      T m[3];
      for (int a = 0; a < 3; ++a) m[a] = (knew == 1 ? 1.0 : -1.0) * nrm[3 * c + a];
      // Candidate directions sorted by alignment, ties to the lowest index.
      int order[27], nc = 0;
      double score[27];
      for (int i = 0; i < Q; ++i) {
        const int* ci = L.c[i];
        double len = std::sqrt((double)(ci[0] * ci[0] + ci[1] * ci[1] + ci[2] * ci[2]));
        if (len == 0.0) continue;
        double sc = (ci[0] * val(m[0]) + ci[1] * val(m[1]) + ci[2] * val(m[2])) / len;
        if (sc <= 0.0) continue;
        score[i] = sc;
        int p = nc++;
        order[p] = i;
        while (p > 0 && score[order[p - 1]] < sc) { std::swap(order[p - 1], order[p]); --p; }
      }
      // Boundary values: the old phase's moments here, with the normal
      // stress condition reduced to the Laplace jump.
      T rhoO = Mr1[c];
      T uG[3] = {Mu1[3 * c], Mu1[3 * c + 1], Mu1[3 * c + 2]};
      T pold = pressure(kold, rhoO, c);
      T pnew = (knew == 0) ? pold + sig * kap[c] : pold - sig * kap[c];
      T rhoG = 1.0 + (pnew - (knew == 1 ? baseline(c) : T(0.0))) / (P.rho_phys[knew] * CS2);
      auto established = [&](long s) { return gas[s] == knew && gas1[s] == knew; };
      // Wall distance q along e: from the level set across x - e when it
      // changes sign there (branch 0), else the normal distance |phi| / |e.n|
      // along e, capped at one spacing (branches 1-3).
      auto q_branch = [&](const int* e, T& q) {
        long xm = 0;
        if (nb(x, y, z, -e[0], -e[1], -e[2], xm) && ((val(phi[xm]) >= 0.0) != (val(phi[c]) >= 0.0))) {
          q = phi[c] / (phi[c] - phi[xm]);
          return 0;
        }
        double len = std::sqrt((double)(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]));
        T en = (e[0] * nrm[3 * c] + e[1] * nrm[3 * c + 1] + e[2] * nrm[3 * c + 2]) / len;
        T aen = fabs(en);
        if (val(aen) < 1e-12) { q = T(1.0); return 1; }
        q = fabs(phi[c]) / (aen * len);
        if (val(q) > 1.0) { q = T(1.0); return 3; }
        return 2;
      };
      // The choice: the first direction in order of alignment whose
      // neighbour x + e is established, quadratic if x + 2e is too, and the
      // q branch; -1 when no direction qualifies.
      long code = -1;
      for (int t = 0; t < nc; ++t) {
        const int i = order[t];
        const int* e = L.c[i];
        long x1 = 0, x2 = 0;
        if (!nb(x, y, z, e[0], e[1], e[2], x1) || !established(x1)) continue;
        bool two = nb(x, y, z, 2 * e[0], 2 * e[1], 2 * e[2], x2) && established(x2);
        T qd;
        code = 16 * i + 4 * (two ? 1 : 0) + q_branch(e, qd);
        break;
      }
      code = decide(c, 5, code);
      if (code >= 0) {
        const int i = (int)(code / 16);
        const bool two = ((code / 4) % 4) != 0;
        const int qb = (int)(code % 4);
        const int* e = L.c[i];
        long x1 = 0, x2 = 0;
        nb(x, y, z, e[0], e[1], e[2], x1);
        if (two) nb(x, y, z, 2 * e[0], 2 * e[1], 2 * e[2], x2);
        T q;
        if (qb == 0) {
          long xm = 0;
          nb(x, y, z, -e[0], -e[1], -e[2], xm);
          q = phi[c] / (phi[c] - phi[xm]);
        } else if (qb == 2) {
          double len = std::sqrt((double)(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]));
          T en = (e[0] * nrm[3 * c] + e[1] * nrm[3 * c + 1] + e[2] * nrm[3 * c + 2]) / len;
          q = fabs(phi[c]) / (fabs(en) * len);
        } else {
          q = T(1.0);
        }
        T w0, w1, w2 = T(0.0);
        if (two) {
          w0 = 2.0 / ((q + 1.0) * (q + 2.0));
          w1 = 2.0 * q / (q + 1.0);
          w2 = -q / (q + 2.0);
        } else {
          w0 = 1.0 / (1.0 + q);
          w1 = q / (1.0 + q);
        }
        // Converting the old phase's pressure into the density of a lighter
        // new phase multiplies the old phase's pressure fluctuations by
        // rho_old / rho_new in LB density (1000 for liquid -> gas); reading:
        // into the lighter phase the boundary density is that of the nearest
        // established cell of the new phase.
        T rhoB = (P.rho_phys[knew] >= P.rho_phys[kold]) ? rhoG : Mr1[x1];
        T rr = w0 * rhoB + w1 * Mr1[x1] + (two ? w2 * Mr1[x2] : T(0.0));
        T ur[3];
        for (int a = 0; a < 3; ++a)
          ur[a] = w0 * uG[a] + w1 * Mu1[3 * x1 + a] + (two ? w2 * Mu1[3 * x2 + a] : T(0.0));
        T fe[27], fe1[27];
        equilibrium(L, rr, ur, fe);
        T u1[3] = {Mu1[3 * x1], Mu1[3 * x1 + 1], Mu1[3 * x1 + 2]};
        equilibrium(L, Mr1[x1], u1, fe1);
        for (int k = 0; k < Q; ++k) An[(size_t)k * N + c] = fe[k] + (An[(size_t)k * N + x1] - fe1[k]);
        Mr1[c] = rr;
        for (int a = 0; a < 3; ++a) Mu1[3 * c + a] = ur[a];
        for (int mm = 0; mm < 6; ++mm) MS1[6 * c + mm] = MS1[6 * x1 + mm];
      } else {
        T fe[27];
        equilibrium(L, rhoG, uG, fe);
        for (int k = 0; k < Q; ++k) An[(size_t)k * N + c] = fe[k];
        Mr1[c] = rhoG;
        for (int mm = 0; mm < 6; ++mm) MS1[6 * c + mm] = T(0.0);
      }
    }
  }

  // a9: Heaviside-weighted gas volume and centroid (Sec. 3.2).
  void centroid(T& V, T xc[3]) const {
    V = T(0.0);
    T s[3] = {T(0.0), T(0.0), T(0.0)};
    for (long c = 0; c < N; ++c) {
      const double pe = val(phi[c]);
      const long reg = decide(c, 6, pe < -P.heaviside_eps ? -1 : (pe > P.heaviside_eps ? 1 : 0));
      if (reg < 0) continue;
      T h = reg > 0 ? T(1.0) : heaviside_mid(phi[c], P.heaviside_eps);
      if (val(h) == 0.0) continue;
      int x, y, z;
      coords(c, x, y, z);
      V += h;
      s[0] += h * (x + 0.5); s[1] += h * (y + 0.5); s[2] += h * (z + 0.5);
    }
    for (int a = 0; a < 3; ++a) xc[a] = (val(V) > 0.0) ? s[a] / V : T(0.0);
  }

  // Several bubbles (reading; the paper gives no pressure level for the
  // gas of several bubbles): every connected component of the support of
  // the smoothed Heaviside (phi > -eps, cells joined by the lattice links,
  // periodic faces wrapping) is a bubble, numbered by its smallest cell
  // index, with the baseline of the single-bubble case taken at its own
  // centroid: Pb_k = pb0 + rho_l a_l . (x_c,k - x_c0), x_c0 the initial
  // centroid of all gas (the hydrostatic reference of the liquid).
  void update_bubbles() {
    const double eps = P.heaviside_eps;
    bub.assign(N, -1);
    int nb_ = 0;
    std::vector<long> queue;
    for (long c0 = 0; c0 < N; ++c0) {
      if (bub[c0] >= 0 || !(val(phi[c0]) > -eps)) continue;
      const int id = nb_++;
      bub[c0] = id;
      queue.assign(1, c0);
      for (size_t h = 0; h < queue.size(); ++h) {
        int x, y, z;
        coords(queue[h], x, y, z);
        for (int i = 0; i < Q; ++i) {
          if (L.c[i][0] == 0 && L.c[i][1] == 0 && L.c[i][2] == 0) continue;
          long s;
          if (!nb(x, y, z, L.c[i][0], L.c[i][1], L.c[i][2], s)) continue;
          if (bub[s] >= 0 || !(val(phi[s]) > -eps)) continue;
          bub[s] = id;
          queue.push_back(s);
        }
      }
    }
    for (long c = 0; c < N; ++c)
      if (decide(c, 7, bub[c]) != bub[c]) rbad = true;  // labels are checked, not imposed
    bvol.assign(nb_, T(0.0));
    bxc.assign(3 * (size_t)nb_, T(0.0));
    bpb.assign(nb_, T(0.0));
    for (long c = 0; c < N; ++c) {
      if (bub[c] < 0) continue;
      T h = heaviside(phi[c], eps);
      int x, y, z;
      coords(c, x, y, z);
      const int k = bub[c];
      bvol[k] += h;
      bxc[3 * k] += h * (x + 0.5); bxc[3 * k + 1] += h * (y + 0.5); bxc[3 * k + 2] += h * (z + 0.5);
    }
    for (int k = 0; k < nb_; ++k) {
      T pb = T(P.pb0);
      for (int a = 0; a < 3; ++a) {
        bxc[3 * k + a] = val(bvol[k]) > 0.0 ? bxc[3 * k + a] / bvol[k] : T(0.0);
        pb = pb + P.rho_phys[0] * P.accel[0][a] * (bxc[3 * k + a] - xc0[a]);
      }
      bpb[k] = pb;
    }
    pbc.assign(N, T(0.0));
    for (long c = 0; c < N; ++c)
      if (bub[c] >= 0) pbc[c] = bpb[bub[c]];
  }

  void update_pb() {
    if (P.use_pb == 2) {
      update_bubbles();
      return;
    }
    if (!P.use_pb) return;
    T V, xc[3];
    centroid(V, xc);
    // Gas pressure baseline: the liquid's hydrostatic pressure at the
    // bubble centroid relative to the initial one (reading; the paper is
    // silent on how the gas pressure level follows a rising bubble).
    T pb = T(P.pb0);
    for (int a = 0; a < 3; ++a) pb = pb + P.rho_phys[0] * P.accel[0][a] * (xc[a] - xc0[a]);
    Pb = pb;
  }

  // ------------------------------------------------------------------
  // One time step n -> n+1.  Order (the paper gives no sequencing; reading):
  //  1 LB collide-stream with wall and interface bounce-back from
  //    (A_n, phi_n, n_n, kappa_n, M_n, Pb_n), writing A_{n+1} and M_{n+1}
  //  2 velocity extension seeded from M_{n+1}
  //  3 TVD-RK3 advection of phi on the band, clamp
  //  4 reinitialisation every reinit_every steps
  //  5 classification of phase and band from phi_{n+1}
  //  6 geometry (n, kappa) on the new band
  //  7 refill of cells whose phase changed
  //  8 gas centroid and pressure baseline
  // ------------------------------------------------------------------
  void step() {
    begin_decisions();
    lb_step();
    extension();
    advect();
    if (P.reinit_every > 0 && ((nstep + 1) % P.reinit_every) == 0 && P.n_reinit > 0) reinit();
    classify(gas1, act1);
    decide_tags(gas1, act1);
    std::swap(act, act1);  // geometry runs on the new band
    geometry();
    std::swap(act, act1);
    refill();
    std::swap(A, An);
    std::swap(Mr, Mr1); std::swap(Mu, Mu1); std::swap(MS, MS1);
    std::swap(gas, gas1); std::swap(act, act1);
    update_pb();
    fold_decisions();
    ++nstep;
  }

  // Initial state: phi clamped to the band, A = f^eq(rho0, u0), M = (rho0, u0, 0).
  void init(const T* phi0, const double* rho0, const double* u0) {
    const double B = P.band;
    for (long c = 0; c < N; ++c) {
      T p = phi0[c];
      if (val(p) > B - BAND_SNAP) p = T(B);
      if (val(p) < -(B - BAND_SNAP)) p = T(-B);
      phi[c] = p;
    }
    begin_decisions();
    classify(gas, act);
    decide_tags(gas, act);
    geometry();
    T V;
    centroid(V, xc0);
    Pb = T(P.pb0);
    if (P.use_pb == 2) update_bubbles();
    for (long c = 0; c < N; ++c) {
      int x, y, z;
      coords(c, x, y, z);
      const int k = gas[c];
      T rho;
      if (rho0) rho = T(rho0[c]);
      else {
        rho = T(1.0);
        if (P.init_hydrostatic) {
          // Hydrostatic LB density of each phase about the initial centroid
          // (with several bubbles, a gas cell about its own bubble's).
          double pos[3] = {x + 0.5, y + 0.5, z + 0.5};
          const T* ref = xc0;
          if (P.use_pb == 2 && k == 1 && bub[c] >= 0) ref = &bxc[3 * (size_t)bub[c]];
          for (int a = 0; a < 3; ++a) rho = rho + P.accel[k][a] * (pos[a] - ref[a]) / CS2;
        }
      }
      T u[3] = {T(0.0), T(0.0), T(0.0)};
      if (u0) for (int a = 0; a < 3; ++a) u[a] = T(u0[3 * c + a]);
      T fe[27];
      equilibrium(L, rho, u, fe);
      for (int i = 0; i < Q; ++i) A[(size_t)i * N + c] = fe[i];
      Mr[c] = rho;
      for (int a = 0; a < 3; ++a) Mu[3 * c + a] = u[a];
      for (int m = 0; m < 6; ++m) MS[6 * c + m] = T(0.0);
    }
    Mr1 = Mr; Mu1 = Mu; MS1 = MS;
    nstep = 0;
    fold_decisions();
  }

  // Macroscopic output: rho = sum A, u = sum c A / rho - a_k / 2 (the
  // time-centred velocity of the stored post-collision state), phase
  // pressure.
  void fields(long c, T& rho, T u[3], T& p) const {
    rho = T(0.0);
    T m[3] = {T(0.0), T(0.0), T(0.0)};
    for (int i = 0; i < Q; ++i) {
      T a = A[(size_t)i * N + c];
      rho += a;
      for (int d = 0; d < 3; ++d) m[d] += (double)L.c[i][d] * a;
    }
    const int k = gas[c];
    for (int d = 0; d < 3; ++d) u[d] = m[d] / rho - 0.5 * P.accel[k][d];
    p = pressure(k, rho, c);
  }
};


// --------------------------------------------------------------------------
// Two-level refinement of the two-phase step (Sec. 2.1, refinement
// paragraph; Sec. 3.2, adaptive refinement with the interface on the finest
// level, the same level on both of its sides).  Reading (the paper gives
// the coupling of its grid levels only as Dupuis-Chopard interpolation in
// space and time with the collision frequency adapted per level):
//
//   levels   a coarse grid of nodes (I, J, K) in coarse lattice units
//            (periodic, no-slip or free-slip faces, the walls of the
//            one-level step), and one box [ia, ib] x [ja, jb] (x [ka, kb]) of its
//            nodes refined at ratio 2 (fine node (i, j, k) at (ia + i/2,
//            ...)), node-centred as the single-phase refinement.
//   fine     the whole two-phase step (collide-stream with wall and
//            interface bounce-back, level set, refill, baseline) on the box's
//            nodes in fine lattice units: tau_f = 2 tau_c - 1/2 per phase
//            (the viscosity of each phase on both levels), sigma_f = 2
//            sigma_c, a_f = a_c / 2 (dt_f = dx_f = half the coarse ones);
//            pressures and velocities are the same numbers on both levels.
//            The band and the level set live on the fine level only: the box
//            must hold the interface with its band and 3 fine cells to
//            spare (the step refuses otherwise).
//   coarse   every uncovered node is in one phase for good (the interface
//            never leaves the box): pull (with the wall rules), BGK with that phase's
//            tau_c and body force; perimeter nodes keep their pre-collision
//            sets G (t + 1).
//   inject   the fine box's faces are injected faces: a fine node pulls a
//            population from outside the box as the Dupuis-Chopard value
//            of the single-phase refinement, the coarse sets interpolated in
//            time ((G(t) + G(t+1))/2 for the first sub-step, G(t+1) for the
//            second) and space (mean of the 2 or 4 coarse nodes beside an
//            odd fine coordinate), the non-equilibrium part about the
//            equilibrium of the interpolated moments scaled by
//            tau_f,k / (2 tau_c,k) of the node's phase k, plus one fine
//            step of body force.  With the first-order force a pre-collision
//            set lags the physical time by one step of its own level, half a
//            coarse step more on the coarse grid than on the fine level;
//            the fine force closes that gap (the initial coarse set is the
//            initial state less one coarse step of force).
//   restrict after the second sub-step, only the covered coarse nodes
//            next to the perimeter (the only ones the coarse step reads)
//            take the fine node's state: its pre-collision populations of
//            that sub-step (pulled again from the fine state before it; the
//            node is a bulk node of one phase) less one fine step of force,
//            f, e = f_eq(moments of f), the coarse post-collision
//            populations e + 2 (tau_c,k - 1) / tau_f,k (f - e) + the coarse
//            body force.
// --------------------------------------------------------------------------
struct TwoPhaseRef {
  Params Pc;             // coarse parameters (coarse lattice units)
  Lattice L;
  int D = 2, Q = 9;
  int n[3] = {1, 1, 1};  // coarse nodes per axis
  int box[6] = {0, 0, 0, 0, 0, 0};
  double omega_c[2], tau_c[2], tau_f[2];
  std::vector<double> fc;            // coarse post-collision populations [q][node]
  std::vector<unsigned char> kc;     // coarse node phase
  std::vector<double> g0, g1;        // coarse pre-collision sets over the box nodes
  Sim<double>* fine = nullptr;
  long nstep = 0;

  ~TwoPhaseRef() { delete fine; }
  long nc() const { return (long)n[0] * n[1] * n[2]; }
  long cidx(int I, int J, int K) const { return ((long)K * n[1] + J) * n[0] + I; }
  int bext(int a) const { return box[2 * a + 1] - box[2 * a] + 1; }
  long nbox() const { return (long)bext(0) * bext(1) * (D == 3 ? bext(2) : 1); }
  long bidx(int I, int J, int K) const {
    return ((long)(D == 3 ? K - box[4] : 0) * bext(1) + (J - box[2])) * bext(0) + (I - box[0]);
  }
  bool covered(int I, int J, int K) const {
    return I > box[0] && I < box[1] && J > box[2] && J < box[3] && (D == 2 || (K > box[4] && K < box[5]));
  }
  bool in_box(int I, int J, int K) const {
    return I >= box[0] && I <= box[1] && J >= box[2] && J <= box[3] && (D == 2 || (K >= box[4] && K <= box[5]));
  }
  bool perimeter(int I, int J, int K) const { return in_box(I, J, K) && !covered(I, J, K); }
  // covered and next to the perimeter: the nodes the coarse step reads
  bool inner_ring(int I, int J, int K) const {
    if (!covered(I, J, K)) return false;
    bool r = I == box[0] + 1 || I == box[1] - 1 || J == box[2] + 1 || J == box[3] - 1;
    if (D == 3) r = r || K == box[4] + 1 || K == box[5] - 1;
    return r;
  }

  void moments(const double* f, double& rho, double u[3]) const {
    rho = 0.0;
    double m[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < Q; ++q) {
      rho += f[q];
      for (int a = 0; a < 3; ++a) m[a] += (double)L.c[q][a] * f[q];
    }
    for (int a = 0; a < 3; ++a) u[a] = m[a] / rho;
  }
  void force(int k, double rho, const double* acc, double* F) const {
    for (int q = 0; q < Q; ++q) {
      double ca = 0.0;
      for (int a = 0; a < 3; ++a) ca += (double)L.c[q][a] * acc[a];
      F[q] = L.w[q] * rho * ca / CS2;
    }
  }

  // coarse parameters Pc (bc all periodic), box in coarse nodes
  bool create(const Params& p, const int* b) {
    Pc = p;
    L = make_lattice(p.lattice);
    D = L.D;
    Q = L.Q;
    n[0] = p.nx; n[1] = p.ny; n[2] = p.nz;
    for (int a = 0; a < 6; ++a) box[a] = (a < 2 * D) ? b[a] : 0;
    for (int a = 0; a < D; ++a)
      if (box[2 * a] < 1 || box[2 * a + 1] > n[a] - 2 || box[2 * a + 1] - box[2 * a] < 4) return false;
    for (int k = 0; k < 2; ++k) {
      tau_c[k] = p.tau[k];
      omega_c[k] = 1.0 / tau_c[k];
      tau_f[k] = 2.0 * tau_c[k] - 0.5;
    }
    Params pf = p;
    pf.nx = 2 * (box[1] - box[0]) + 1;
    pf.ny = 2 * (box[3] - box[2]) + 1;
    pf.nz = D == 3 ? 2 * (box[5] - box[4]) + 1 : 1;
    for (int a = 0; a < 6; ++a) pf.bc[a] = (a < 2 * D) ? BC_INJECT : BC_PERIODIC;
    for (int k = 0; k < 2; ++k) {
      pf.tau[k] = tau_f[k];
      for (int a = 0; a < 3; ++a) pf.accel[k][a] = 0.5 * p.accel[k][a];
    }
    pf.sigma = 2.0 * p.sigma;
    pf.init_hydrostatic = 0;
    fine = new Sim<double>(pf);
    fine->ghost.assign((size_t)Q * fine->N, 0.0);
    return true;
  }

  // equilibrium initial state on both levels from the caller's fields at
  // the coarse nodes (phi_c, rho_c, u_c) and at the fine nodes (phi_f,
  // rho_f, u_f); u arrays hold 3 components per node
  void init(const double* phi_c, const double* rho_c, const double* u_c, const double* phi_f, const double* rho_f,
            const double* u_f) {
    const long N = nc();
    fc.assign((size_t)Q * N, 0.0);
    kc.assign(N, 0);
    double e[27];
    for (long c = 0; c < N; ++c) {
      kc[c] = phi_c[c] >= 0.0 ? 1 : 0;
      double u[3] = {u_c[3 * c], u_c[3 * c + 1], u_c[3 * c + 2]};
      equilibrium(L, rho_c[c], u, e);
      for (int q = 0; q < Q; ++q) fc[(size_t)q * N + c] = e[q];
    }
    fine->init(phi_f, rho_f, u_f);
    g0.assign((size_t)Q * nbox(), 0.0);
    g1 = g0;
    for (int K = box[4]; K <= (D == 3 ? box[5] : 0); ++K)
      for (int J = box[2]; J <= box[3]; ++J)
        for (int I = box[0]; I <= box[1]; ++I)
          if (perimeter(I, J, K)) {
            // the pre-collision set one coarse step before the start: the
            // initial state less one step of body force
            const long c = cidx(I, J, K);
            double rho = 0.0, F[27];
            for (int q = 0; q < Q; ++q) rho += fc[(size_t)q * N + c];
            force(kc[c], rho, Pc.accel[kc[c]], F);
            for (int q = 0; q < Q; ++q) g0[(size_t)q * nbox() + bidx(I, J, K)] = fc[(size_t)q * N + c] - F[q];
          }
    nstep = 0;
  }

  // The coarse population entering node (I, J, K) along c_q: pull
  // streaming with the wall rules of the one-level step (walls on cell
  // faces; halfway bounce-back with the moving-wall term across a no-slip
  // face, specular reflection across a free-slip face) and periodic wrap.
  // The coarse grid holds no interface.
  double coarse_pull(int I, int J, int K, int q) const {
    const long N = nc();
    const int* ci = L.c[q];
    const int pos[3] = {I, J, K};
    int s[3];
    bool cross[3] = {false, false, false};
    int face[3] = {0, 0, 0};
    bool any = false;
    for (int a = 0; a < 3; ++a) {
      s[a] = pos[a] - ci[a];
      if (s[a] >= 0 && s[a] < n[a]) continue;
      if (Pc.bc[2 * a] == BC_PERIODIC) { s[a] = (s[a] + n[a]) % n[a]; continue; }
      cross[a] = true;
      face[a] = s[a] < 0 ? 2 * a : 2 * a + 1;
      any = true;
    }
    if (!any) return fc[(size_t)q * N + cidx(s[0], s[1], s[2])];
    for (int a = 0; a < 3; ++a)
      if (cross[a] && Pc.bc[face[a]] == BC_NOSLIP) {
        const double* uw = Pc.wall_u[face[a]];
        const double cu = ci[0] * uw[0] + ci[1] * uw[1] + ci[2] * uw[2];
        return fc[(size_t)L.opp[q] * N + cidx(I, J, K)] + 2.0 * L.w[q] * cu / CS2;
      }
    int cr[3];
    for (int a = 0; a < 3; ++a) {
      cr[a] = cross[a] ? -ci[a] : ci[a];
      if (cross[a]) s[a] = pos[a];
    }
    return fc[(size_t)find_dir(L, cr[0], cr[1], cr[2]) * N + cidx(s[0], s[1], s[2])];
  }

  // coarse step: uncovered nodes pull, keep G at the perimeter, collide
  std::vector<double> coarse_step() {
    const long N = nc();
    std::vector<double> out = fc;
    for (int K = 0; K < n[2]; ++K)
      for (int J = 0; J < n[1]; ++J)
        for (int I = 0; I < n[0]; ++I) {
          if (covered(I, J, K)) continue;
          const long c = cidx(I, J, K);
          double f[27], e[27], F[27];
          for (int q = 0; q < Q; ++q) f[q] = coarse_pull(I, J, K, q);
          if (perimeter(I, J, K))
            for (int q = 0; q < Q; ++q) g1[(size_t)q * nbox() + bidx(I, J, K)] = f[q];
          const int k = kc[c];
          double rho, u[3];
          moments(f, rho, u);
          equilibrium(L, rho, u, e);
          force(k, rho, Pc.accel[k], F);
          for (int q = 0; q < Q; ++q) out[(size_t)q * N + c] = f[q] - omega_c[k] * (f[q] - e[q]) + F[q];
        }
    return out;
  }

  // the populations entering the fine box across its faces, for a sub-step
  // with time weights a (G(t)) and b (G(t+1))
  void inject(double a, double b) {
    Sim<double>& s = *fine;
    const int m[3] = {s.nx - 1, s.ny - 1, s.nz - 1};
    for (long c = 0; c < s.N; ++c) {
      int i, j, k;
      s.coords(c, i, j, k);
      const bool surf = i == 0 || i == m[0] || j == 0 || j == m[1] || (D == 3 && (k == 0 || k == m[2]));
      if (!surf) continue;
      double H[27] = {0.0}, eh[27], rho, u[3];
      const int o[3] = {i & 1, j & 1, D == 3 ? (k & 1) : 0};
      const double w = (o[0] ? 0.5 : 1.0) * (o[1] ? 0.5 : 1.0) * (o[2] ? 0.5 : 1.0);
      for (int dz = 0; dz <= o[2]; ++dz)
        for (int dy = 0; dy <= o[1]; ++dy)
          for (int dx = 0; dx <= o[0]; ++dx) {
            const long bx = bidx(box[0] + (i - o[0]) / 2 + dx, box[2] + (j - o[1]) / 2 + dy,
                                 (D == 3 ? box[4] + (k - o[2]) / 2 + dz : 0));
            for (int q = 0; q < Q; ++q)
              H[q] += w * (a * g0[(size_t)q * nbox() + bx] + b * g1[(size_t)q * nbox() + bx]);
          }
      moments(H, rho, u);
      equilibrium(L, rho, u, eh);
      const int ph = s.gas[c];
      const double r = tau_f[ph] / (2.0 * tau_c[ph]);
      double Ff[27];
      force(ph, rho, s.P.accel[ph], Ff);
      for (int q = 0; q < Q; ++q) {
        const int si = i - L.c[q][0], sj = j - L.c[q][1], sk = k - L.c[q][2];
        const bool out = si < 0 || si > m[0] || sj < 0 || sj > m[1] || (D == 3 && (sk < 0 || sk > m[2]));
        if (out) s.ghost[(size_t)q * s.N + c] = eh[q] + r * (H[q] - eh[q]) + Ff[q];
      }
    }
  }

  // restriction of every covered node from the fine state (see above; the
  // coarse step reads only the ring next to the perimeter, the others keep
  // the coarse state complete for output and re-meshing); prev is the fine
  // post-collision state before the second sub-step
  void restrict_into(std::vector<double>& out, const std::vector<double>& prev) {
    Sim<double>& s = *fine;
    const long N = nc();
    for (int K = box[4]; K <= (D == 3 ? box[5] : 0); ++K)
      for (int J = box[2]; J <= box[3]; ++J)
        for (int I = box[0]; I <= box[1]; ++I) {
          if (!covered(I, J, K)) continue;
          const int fi = 2 * (I - box[0]), fj = 2 * (J - box[2]), fk = D == 3 ? 2 * (K - box[4]) : 0;
          const long fcell = s.idx(fi, fj, fk);
          double f[27], e[27], F[27], rho, u[3];
          const int k = s.gas[fcell];
          double Ff[27], rf = 0.0;
          for (int q = 0; q < Q; ++q) {
            f[q] = prev[(size_t)q * s.N + s.idx(fi - L.c[q][0], fj - L.c[q][1], fk - L.c[q][2])];
            rf += f[q];
          }
          force(k, rf, s.P.accel[k], Ff);
          for (int q = 0; q < Q; ++q) f[q] -= Ff[q];  // back to the coarse pre-collision time
          moments(f, rho, u);
          equilibrium(L, rho, u, e);
          force(k, rho, Pc.accel[k], F);
          const long c = cidx(I, J, K);
          kc[c] = (unsigned char)k;
          for (int q = 0; q < Q; ++q)
            out[(size_t)q * N + c] = e[q] + 2.0 * (tau_c[k] - 1.0) / tau_f[k] * (f[q] - e[q]) + F[q];
        }
  }

  // the band keeps 3 fine cells away from the box faces
  bool band_inside() const {
    const Sim<double>& s = *fine;
    const int m[3] = {s.nx - 1, s.ny - 1, s.nz - 1};
    for (long c = 0; c < s.N; ++c) {
      if (!s.act[c]) continue;
      int i, j, k;
      s.coords(c, i, j, k);
      if (i < 3 || i > m[0] - 3 || j < 3 || j > m[1] - 3 || (D == 3 && (k < 3 || k > m[2] - 3))) return false;
    }
    return true;
  }

  // The perimeter's pre-collision sets at the current time, inverted from
  // the coarse post-collision populations f of each perimeter node: with
  // u = m/rho - a_c the pre-collision velocity and e = f_eq(rho, u),
  // G = e + tau_c / (tau_c - 1) (f - F_c - e) (e at tau_c = 1).
  void perimeter_sets_from_state() {
    const long N = nc();
    g0.assign((size_t)Q * nbox(), 0.0);
    for (int K = box[4]; K <= (D == 3 ? box[5] : 0); ++K)
      for (int J = box[2]; J <= box[3]; ++J)
        for (int I = box[0]; I <= box[1]; ++I) {
          if (!perimeter(I, J, K)) continue;
          const long c = cidx(I, J, K);
          const int k = kc[c];
          double f[27], e[27], F[27], rho, u[3];
          for (int q = 0; q < Q; ++q) f[q] = fc[(size_t)q * N + c];
          moments(f, rho, u);
          for (int a = 0; a < 3; ++a) u[a] -= Pc.accel[k][a];
          equilibrium(L, rho, u, e);
          force(k, rho, Pc.accel[k], F);
          const double r = tau_c[k] == 1.0 ? 0.0 : tau_c[k] / (tau_c[k] - 1.0);
          for (int q = 0; q < Q; ++q) g0[(size_t)q * nbox() + bidx(I, J, K)] = e[q] + r * (f[q] - F[q] - e[q]);
        }
  }

  // Re-meshing onto the box nb of the same extents, between coarse steps
  // (reading).  Fine nodes inside the old box keep their state
  // (populations, level set, moments of the last collision); the others take
  // the coarse post-collision populations H interpolated as at the
  // perimeter (mean of 2, 4 or 8 nodes) at the same time level: with u =
  // m/rho, e_c = f_eq(rho, u - a_c) and e_f = f_eq(rho, u - a_f), the fine
  // post-collision populations e_f + (tau_f - 1) / (2 (tau_c - 1)) (H - F_c -
  // e_c) + F_f (the coarse non-equilibrium part rescaled to the fine level;
  // none at tau_c = 1), the level set at +-band by the coarse phase, the
  // moments (rho, u, 0).  The level set's tags, band and geometry are
  // classified again, bubbles relabelled, the initial centroid moved with
  // the fine coordinates (the baseline is unchanged); the covered coarse
  // nodes already hold the restricted fine state, and the new perimeter's
  // pre-collision sets are inverted from the coarse state.  Returns -1 for
  // a box of other extents or outside the grid, -2 if the band is not
  // inside the new box.
  int remesh(const int* nbx) {
    int d[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
      if (nbx[2 * a + 1] - nbx[2 * a] != box[2 * a + 1] - box[2 * a]) return -1;
      if (nbx[2 * a] < 1 || nbx[2 * a + 1] > n[a] - 2) return -1;
      d[a] = nbx[2 * a] - box[2 * a];
    }
    Sim<double>& s = *fine;
    const long Nf = s.N, N = nc();
    std::vector<double> A2((size_t)Q * Nf), phi2(Nf), Mr2(Nf), Mu2(3 * (size_t)Nf), MS2(6 * (size_t)Nf);
    const double B = s.P.band;
    for (long c = 0; c < Nf; ++c) {
      int i, j, k;
      s.coords(c, i, j, k);
      const int oi = i + 2 * d[0], oj = j + 2 * d[1], ok = k + 2 * d[2];
      if (oi >= 0 && oi < s.nx && oj >= 0 && oj < s.ny && ok >= 0 && ok < s.nz) {
        const long o = s.idx(oi, oj, ok);
        for (int q = 0; q < Q; ++q) A2[(size_t)q * Nf + c] = s.A[(size_t)q * Nf + o];
        phi2[c] = s.phi[o];
        Mr2[c] = s.Mr[o];
        for (int a = 0; a < 3; ++a) Mu2[3 * c + a] = s.Mu[3 * o + a];
        for (int m = 0; m < 6; ++m) MS2[6 * c + m] = s.MS[6 * o + m];
        continue;
      }
      const int o3[3] = {i & 1, j & 1, D == 3 ? (k & 1) : 0};
      const double w = (o3[0] ? 0.5 : 1.0) * (o3[1] ? 0.5 : 1.0) * (o3[2] ? 0.5 : 1.0);
      double H[27] = {0.0};
      int kk = 0;
      for (int dz = 0; dz <= o3[2]; ++dz)
        for (int dy = 0; dy <= o3[1]; ++dy)
          for (int dx = 0; dx <= o3[0]; ++dx) {
            const long cc = cidx(nbx[0] + (i - o3[0]) / 2 + dx, nbx[2] + (j - o3[1]) / 2 + dy,
                                 D == 3 ? nbx[4] + (k - o3[2]) / 2 + dz : 0);
            kk = kc[cc];
            for (int q = 0; q < Q; ++q) H[q] += w * fc[(size_t)q * N + cc];
          }
      double rho, u[3], uc[3], uf[3], ec[27], ef[27], Fc[27], Ff[27];
      moments(H, rho, u);
      for (int a = 0; a < 3; ++a) {
        uc[a] = u[a] - Pc.accel[kk][a];
        uf[a] = u[a] - s.P.accel[kk][a];
      }
      equilibrium(L, rho, uc, ec);
      equilibrium(L, rho, uf, ef);
      force(kk, rho, Pc.accel[kk], Fc);
      force(kk, rho, s.P.accel[kk], Ff);
      const double ratio = tau_c[kk] == 1.0 ? 0.0 : (tau_f[kk] - 1.0) / (2.0 * (tau_c[kk] - 1.0));
      for (int q = 0; q < Q; ++q) A2[(size_t)q * Nf + c] = ef[q] + ratio * (H[q] - Fc[q] - ec[q]) + Ff[q];
      phi2[c] = kk ? B : -B;
      Mr2[c] = rho;
      for (int a = 0; a < 3; ++a) Mu2[3 * c + a] = u[a];
      for (int m = 0; m < 6; ++m) MS2[6 * c + m] = 0.0;
    }
    s.A.swap(A2);
    s.An = s.A;
    s.phi.swap(phi2);
    s.Mr.swap(Mr2);
    s.Mu.swap(Mu2);
    s.MS.swap(MS2);
    s.Mr1 = s.Mr;
    s.Mu1 = s.Mu;
    s.MS1 = s.MS;
    for (int a = 0; a < D; ++a) s.xc0[a] = s.xc0[a] - 2.0 * d[a];
    for (int a = 0; a < 6; ++a) box[a] = a < 2 * D ? nbx[a] : 0;
    s.classify(s.gas, s.act);
    s.geometry();
    if (s.P.use_pb == 2) s.update_bubbles();
    perimeter_sets_from_state();
    return band_inside() ? 0 : -2;
  }

  // Level-set sensor for the box (reading; liquid phi < 0, gas phi >= 0 as
  // everywhere here): the fine cells with phi >= -d_ref (the gas and a band
  // of width d_ref around it) are tagged; the box keeps its extents and is
  // moved so that the centre of the tagged cells' bounding box (fine
  // indices lo, hi) falls on its centre, rounded half up to whole coarse
  // nodes, clamped one node inside the grid faces.  The current box when no
  // cell is tagged.
  void sensor(double d_ref, int* out) const {
    const Sim<double>& s = *fine;
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-1, -1, -1};
    for (long c = 0; c < s.N; ++c) {
      if (!(s.phi[c] >= -d_ref)) continue;
      int ijk[3];
      s.coords(c, ijk[0], ijk[1], ijk[2]);
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], ijk[a]);
        hi[a] = std::max(hi[a], ijk[a]);
      }
    }
    for (int a = 0; a < 6; ++a) out[a] = box[a];
    if (hi[0] < 0) return;
    for (int a = 0; a < D; ++a) {
      const int E = box[2 * a + 1] - box[2 * a];
      // new origin: round(box0 + (lo + hi) / 4 - E / 2), in quarter nodes
      const long q4 = 4L * box[2 * a] + lo[a] + hi[a] - 2L * E + 2;
      long b0 = q4 >= 0 ? q4 / 4 : -((-q4 + 3) / 4);
      b0 = std::max<long>(1, std::min<long>(b0, n[a] - 2 - E));
      out[2 * a] = (int)b0;
      out[2 * a + 1] = (int)b0 + E;
    }
  }

  bool step() {
    std::vector<double> out = coarse_step();
    inject(0.5, 0.5);
    fine->step();
    inject(0.0, 1.0);
    fine->step();
    restrict_into(out, fine->An);  // after the swap, An holds the state before the second sub-step
    fc.swap(out);
    g0.swap(g1);
    ++nstep;
    return band_inside();
  }
};

}  // namespace orc

// ==========================================================================
// C interface (double instantiation, plus the tangent entry points).
// ==========================================================================
using orc::Dual;
using orc::Sim;

extern "C" {

struct orc_params_c {  // identical layout to orc::Params
  orc::Params p;
};

int orc_lattice(int lattice, int* D, int* Q, int* c, double* w, int* opp) {
  if (lattice < 0 || lattice > 2) return -1;
  orc::Lattice L = orc::make_lattice(lattice);
  *D = L.D; *Q = L.Q;
  for (int i = 0; i < L.Q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
    w[i] = L.w[i];
    opp[i] = L.opp[i];
  }
  return 0;
}

int orc_feq(int lattice, double rho, const double* u, double* out) {
  if (lattice < 0 || lattice > 2) return -1;
  orc::Lattice L = orc::make_lattice(lattice);
  orc::equilibrium(L, rho, u, out);
  return 0;
}

// Joint cumulants kappa[9a + 3b + c] (a, b, c in {0, 1, 2}) of the
// normalised weighted point set (pts [n][3], weights w); kappa[0] = sum w.
int orc_cumulants_points(int n, const double* pts, const double* w, double* kappa) {
  if (n < 1) return -1;
  double W = 0.0, m[27] = {};
  for (int j = 0; j < n; ++j) W += w[j];
  if (!(W > 0.0)) return -1;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int j = 0; j < n; ++j)
          s += w[j] * std::pow(pts[3 * j], a) * std::pow(pts[3 * j + 1], b) * std::pow(pts[3 * j + 2], c);
        m[orc::midx(a, b, c)] = s / W;
      }
  orc::cumulants_from_moments(m, kappa);
  kappa[0] = W;
  return 0;
}

// Normalised moments m[9a + 3b + c] from joint cumulants (kappa[0] ignored).
void orc_moments_from_cumulants(const double* kappa, double* m) { orc::moments_from_cumulants(kappa, m); }

// One D3Q27 cell through the cumulant collision (rates omega1, omega2,
// omega3; the paper's operator is omega2 = omega3 = 1) with acceleration acc.
int orc_cumulant_collide(const double* f, double omega1, double omega2, double omega3, const double* acc,
                         double* out) {
  const orc::Lattice L = orc::make_lattice(2);
  orc::cumulant_collide(L, f, omega1, omega2, omega3, acc, out);
  return 0;
}

void orc_refill_weights(double q, double* Lw) { Sim<double>::refill_weights(q, Lw); }

double orc_heaviside(double phi, double eps) { return orc::heaviside(phi, eps); }

static int check_params(const orc::Params* p) {
  if (p->lattice < 0 || p->lattice > 2) return -1;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
  if (p->lattice == 0 && p->nz != 1) return -1;
  for (int a = 0; a < 3; ++a)
    if ((p->bc[2 * a] == orc::BC_PERIODIC) != (p->bc[2 * a + 1] == orc::BC_PERIODIC)) return -1;
  if (p->tau[0] <= 0.5 || p->tau[1] <= 0.5) return -1;
  if (p->use_pb < 0 || p->use_pb > 2) return -1;
  for (int k = 0; k < 2; ++k)
    if (p->collision[k] != 0 && (p->collision[k] != 1 || p->lattice != 2)) return -1;
  return 0;
}

void* orc_create(const orc::Params* p) {
  if (check_params(p)) return nullptr;
  return new Sim<double>(*p);
}
void orc_destroy(void* h) { delete static_cast<Sim<double>*>(h); }

int orc_init(void* h, const double* phi0, const double* rho0, const double* u0) {
  static_cast<Sim<double>*>(h)->init(phi0, rho0, u0);
  return 0;
}

int orc_step(void* h, int n) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  for (int k = 0; k < n; ++k) s->step();
  return 0;
}

long orc_nstep(void* h) { return static_cast<Sim<double>*>(h)->nstep; }

// Populations A[i*N + cell].
// Decision record / replay (finite differences of the frozen-decision
// program): mode 1 records the decisions of the run that follows (call
// before orc_init), mode 2 imposes those recorded by src.  Returns -1 for a
// replay without a record.
int orc_set_decisions(void* h, int mode, void* src) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  if (mode == 2) {
    Sim<double>* r = static_cast<Sim<double>*>(src);
    if (!r || r->dmode != 1 || !r->rlog) return -1;
    s->set_decision_mode(2, r->rlog);
  } else {
    s->set_decision_mode(mode, nullptr);
  }
  return 0;
}

// 1 if a replayed run met a decision site the record does not hold (the
// runs took different paths), else 0.
int orc_replay_failed(void* h) { return static_cast<Sim<double>*>(h)->rbad ? 1 : 0; }

// Decision trace: one hash for the initial state and one per step taken
// (see Sim::decide); returns the count, writes at most max hashes.
long orc_decisions(void* h, uint64_t* out, long max) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  const long n = (long)s->dlog.size();
  for (long k = 0; k < n && k < max; ++k) out[k] = s->dlog[k];
  return n;
}

int orc_get_pop(void* h, double* out) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  std::memcpy(out, s->A.data(), sizeof(double) * s->A.size());
  return 0;
}

// Populations (deviations f - w, as stored) and level set of a list of cells
// (sampled comparisons on grids too large to copy out whole):
// pop[i * n + k] = A_i(cells[k]), phi[k], tags[k] as in orc_get_interface.
int orc_get_sample(void* h, const long* cells, int n, double* pop, double* phi, unsigned char* tags) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  for (int k = 0; k < n; ++k) {
    const long c = cells[k];
    if (c < 0 || c >= s->N) return -1;
    if (pop) for (int i = 0; i < s->Q; ++i) pop[(size_t)i * n + k] = s->A[(size_t)i * s->N + c];
    if (phi) phi[k] = s->phi[c];
    if (tags) {
      int x, y, z;
      s->coords(c, x, y, z);
      unsigned char t = s->gas[c] ? orc::TAG_GAS : 0;
      if (s->act[c]) t |= orc::TAG_ACTIVE;
      if (s->is_iface(c, x, y, z, s->gas)) t |= orc::TAG_IFACE;
      tags[k] = t;
    }
  }
  return 0;
}

int orc_get_fields(void* h, double* rho, double* u, double* p, unsigned char* phase) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  for (long c = 0; c < s->N; ++c) {
    double r, uu[3], pp;
    s->fields(c, r, uu, pp);
    if (rho) rho[c] = r;
    if (u) for (int a = 0; a < s->D; ++a) u[(size_t)s->D * c + a] = uu[a];
    if (p) p[c] = pp;
    if (phase) phase[c] = s->gas[c];
  }
  return 0;
}

// Level set, normal (D per cell), curvature and tag bits.
int orc_get_interface(void* h, double* phi, double* normal, double* kappa, unsigned char* tags) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  for (long c = 0; c < s->N; ++c) {
    if (phi) phi[c] = s->phi[c];
    if (normal) for (int a = 0; a < s->D; ++a) normal[(size_t)s->D * c + a] = s->nrm[3 * c + a];
    if (kappa) kappa[c] = s->kap[c];
    if (tags) {
      int x, y, z;
      s->coords(c, x, y, z);
      unsigned char t = s->gas[c] ? orc::TAG_GAS : 0;
      if (s->act[c]) t |= orc::TAG_ACTIVE;
      if (s->is_iface(c, x, y, z, s->gas)) t |= orc::TAG_IFACE;
      tags[c] = t;
    }
  }
  return 0;
}

// Moments of the last collision (rho, u[3], S[6]) per cell, valid on LS-active cells.
int orc_get_moments(void* h, double* out) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  for (long c = 0; c < s->N; ++c) {
    out[10 * c] = s->Mr[c];
    for (int a = 0; a < 3; ++a) out[10 * c + 1 + a] = s->Mu[3 * c + a];
    for (int m = 0; m < 6; ++m) out[10 * c + 4 + m] = s->MS[6 * c + m];
  }
  return 0;
}

// Integral quantities: mass[2], gas volume, centroid[3], bubble velocity[3],
// Pb, max |u|, step.
// Bubbles (use_pb = 2): count, and per bubble (numbered by smallest cell)
// volume, centroid[3], baseline; labels[N] the bubble of each cell (-1
// outside the Heaviside support).  Either output may be NULL.
int orc_get_bubbles(void* h, int max, int* count, double* out, int* labels) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  if (s->P.use_pb != 2) return -1;
  const int n = (int)s->bvol.size();
  *count = n;
  if (out)
    for (int k = 0; k < n && k < max; ++k) {
      out[5 * k] = s->bvol[k];
      for (int a = 0; a < 3; ++a) out[5 * k + 1 + a] = s->bxc[3 * k + a];
      out[5 * k + 4] = s->bpb[k];
    }
  if (labels)
    for (long c = 0; c < s->N; ++c) labels[c] = s->bub[c];
  return 0;
}

int orc_get_integrals(void* h, double* out) {
  Sim<double>* s = static_cast<Sim<double>*>(h);
  double mass[2] = {0, 0}, V = 0, xs[3] = {0, 0, 0}, us[3] = {0, 0, 0}, umax = 0;
  for (long c = 0; c < s->N; ++c) {
    double r, uu[3], pp;
    s->fields(c, r, uu, pp);
    mass[s->gas[c]] += r;
    double hh = orc::heaviside(s->phi[c], s->P.heaviside_eps);
    int x, y, z;
    s->coords(c, x, y, z);
    V += hh;
    xs[0] += hh * (x + 0.5); xs[1] += hh * (y + 0.5); xs[2] += hh * (z + 0.5);
    for (int a = 0; a < 3; ++a) us[a] += hh * uu[a];
    double un = std::sqrt(uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]);
    if (un > umax) umax = un;
  }
  out[0] = mass[0]; out[1] = mass[1]; out[2] = V;
  for (int a = 0; a < 3; ++a) { out[3 + a] = V > 0 ? xs[a] / V : 0.0; out[6 + a] = V > 0 ? us[a] / V : 0.0; }
  out[9] = s->Pb; out[10] = umax; out[11] = (double)s->nstep;
  return 0;
}

// ---- component entry points for the pins -------------------------------
// Each treats every cell as LS-active.

int orc_geometry(const orc::Params* p, const double* phi, double* normal, double* kappa) {
  if (check_params(p)) return -1;
  Sim<double> s(*p);
  s.all_active = true;
  for (long c = 0; c < s.N; ++c) s.phi[c] = phi[c];
  s.geometry();
  for (long c = 0; c < s.N; ++c) {
    for (int a = 0; a < s.D; ++a) normal[(size_t)s.D * c + a] = s.nrm[3 * c + a];
    kappa[c] = s.kap[c];
  }
  return 0;
}

// Transport right-hand side -u.grad phi (upwind-5) with a given velocity field u[3N].
int orc_advect_rate(const orc::Params* p, const double* phi, const double* u, double* out) {
  if (check_params(p)) return -1;
  Sim<double> s(*p);
  s.all_active = true;
  for (long c = 0; c < s.N; ++c) s.phi[c] = phi[c];
  for (long c = 0; c < 3 * s.N; ++c) s.ut[c] = u[c];
  std::vector<double> r(s.N);
  s.advect_rate(s.phi, r);
  for (long c = 0; c < s.N; ++c) out[c] = r[c];
  return 0;
}

// nsteps TVD-RK3 transport steps (dt = 1) with a frozen velocity u[3N]; no clamp.
int orc_advect(const orc::Params* p, double* phi, const double* u, int nsteps) {
  if (check_params(p)) return -1;
  Sim<double> s(*p);
  s.all_active = true;
  s.P.band = 1e300;
  for (long c = 0; c < s.N; ++c) s.phi[c] = phi[c];
  for (long c = 0; c < 3 * s.N; ++c) s.ut[c] = u[c];
  for (int k = 0; k < nsteps; ++k) s.advect();
  for (long c = 0; c < s.N; ++c) phi[c] = s.phi[c];
  return 0;
}

// Reinitialisation with p->n_reinit pseudo steps, repeated `calls` times.
int orc_reinit(const orc::Params* p, double* phi, int calls) {
  if (check_params(p)) return -1;
  Sim<double> s(*p);
  s.all_active = true;
  s.P.band = 1e300;
  for (long c = 0; c < s.N; ++c) s.phi[c] = phi[c];
  for (int k = 0; k < calls; ++k) s.reinit();
  for (long c = 0; c < s.N; ++c) phi[c] = s.phi[c];
  return 0;
}

// Velocity extension on a given level set: seed u (3N), frozen cells
// (nonzero in fixed) keep their seed; n_ext iterations of p.
int orc_extend(const orc::Params* p, const double* phi, const unsigned char* fixed, double* u) {
  if (check_params(p)) return -1;
  Sim<double> s(*p);
  s.all_active = true;
  for (long c = 0; c < s.N; ++c) s.phi[c] = phi[c];
  s.geometry();
  for (long c = 0; c < 3 * s.N; ++c) s.ut[c] = u[c];
  std::vector<unsigned char> icell(fixed, fixed + s.N);
  s.extension_iterate(icell);
  for (long c = 0; c < 3 * s.N; ++c) u[c] = s.ut[c];
  return 0;
}

// Refill (Sec. 2.4) on a crafted state, through the step's own refill():
// phi_new (N) is the level set after transport (its sign gives the new phase,
// its geometry the normal and curvature), old_gas (N) the phase tags before
// it (0 liquid, 1 gas), pop (Q*N, [i*N + cell]) the post-collision
// populations of the step, rho (N), u (3N) and S (6N) the moments of the
// step's collision, pb the gas pressure baseline.  Cells whose tag changes
// are refilled in place in pop, rho, u and S.
int orc_refill(const orc::Params* p, const double* phi_new, const unsigned char* old_gas, double* pop,
               double* rho, double* u, double* S, double pb) {
  if (check_params(p)) return -1;
  Sim<double> s(*p);
  s.all_active = true;
  for (long c = 0; c < s.N; ++c) {
    s.phi[c] = phi_new[c];
    s.gas[c] = old_gas[c] ? 1 : 0;
    s.gas1[c] = phi_new[c] >= 0.0 ? 1 : 0;
    s.Mr1[c] = rho[c];
  }
  s.geometry();
  for (long c = 0; c < 3 * s.N; ++c) s.Mu1[c] = u[c];
  for (long c = 0; c < 6 * s.N; ++c) s.MS1[c] = S[c];
  for (long c = 0; c < (long)s.Q * s.N; ++c) s.An[c] = pop[c];
  s.Pb = pb;
  s.refill();
  for (long c = 0; c < (long)s.Q * s.N; ++c) pop[c] = s.An[c];
  for (long c = 0; c < s.N; ++c) rho[c] = s.Mr1[c];
  for (long c = 0; c < 3 * s.N; ++c) u[c] = s.Mu1[c];
  for (long c = 0; c < 6 * s.N; ++c) S[c] = s.MS1[c];
  return 0;
}

// ---- two-level refinement of the two-phase step ---------------------------
// p: coarse parameters (periodic, no-slip or free-slip faces; z periodic in
// 2D; BGK in both phases), box: 6 ints in coarse nodes.
void* orc_r2_create(const orc::Params* p, const int* box) {
  if (check_params(p)) return nullptr;
  for (int a = 0; a < 6; ++a)
    if (p->bc[a] != orc::BC_PERIODIC && p->bc[a] != orc::BC_NOSLIP && p->bc[a] != orc::BC_FREESLIP) return nullptr;
  if (p->lattice == 0 && p->bc[4] != orc::BC_PERIODIC) return nullptr;
  if (p->collision[0] != 0 || p->collision[1] != 0) return nullptr;
  orc::TwoPhaseRef* r = new orc::TwoPhaseRef();
  if (!r->create(*p, box)) {
    delete r;
    return nullptr;
  }
  return r;
}
void orc_r2_destroy(void* h) { delete static_cast<orc::TwoPhaseRef*>(h); }
// fine-level node counts per axis
void orc_r2_fine_shape(void* h, int* nf) {
  orc::TwoPhaseRef* r = static_cast<orc::TwoPhaseRef*>(h);
  nf[0] = r->fine->nx; nf[1] = r->fine->ny; nf[2] = r->fine->nz;
}
int orc_r2_init(void* h, const double* phi_c, const double* rho_c, const double* u_c, const double* phi_f,
                const double* rho_f, const double* u_f) {
  static_cast<orc::TwoPhaseRef*>(h)->init(phi_c, rho_c, u_c, phi_f, rho_f, u_f);
  return 0;
}
// -2 when the band came within 3 fine cells of the box faces
int orc_r2_step(void* h, int nsteps) {
  orc::TwoPhaseRef* r = static_cast<orc::TwoPhaseRef*>(h);
  for (int s = 0; s < nsteps; ++s)
    if (!r->step()) return -2;
  return 0;
}
// coarse populations [q][node] (covered nodes: the last restriction or the
// initial state), coarse phase [node]; either may be NULL
int orc_r2_get_coarse(void* h, double* pop, unsigned char* phase) {
  orc::TwoPhaseRef* r = static_cast<orc::TwoPhaseRef*>(h);
  if (pop) std::memcpy(pop, r->fc.data(), sizeof(double) * r->fc.size());
  if (phase) std::memcpy(phase, r->kc.data(), r->kc.size());
  return 0;
}
// the fine level as an oracle simulation (populations, fields, interface, integrals)
void* orc_r2_fine(void* h) { return static_cast<orc::TwoPhaseRef*>(h)->fine; }

// Box of the level-set sensor (6 ints) and re-meshing onto a box of the
// same extents (0; -1 for an invalid box, -2 if the band is not inside it).
void orc_r2_sensor(void* h, double d_ref, int* box) { static_cast<orc::TwoPhaseRef*>(h)->sensor(d_ref, box); }
int orc_r2_remesh(void* h, const int* box) { return static_cast<orc::TwoPhaseRef*>(h)->remesh(box); }
void orc_r2_box(void* h, int* box) {
  for (int a = 0; a < 6; ++a) box[a] = static_cast<orc::TwoPhaseRef*>(h)->box[a];
}

// ---- tangent (forward mode, frozen decisions) ---------------------------
// Seeds: dphi0 (N values, may be null) and dsigma.  Output: the tangent of
// the gas centroid component `axis` after the steps taken.
void* orc_tan_create(const orc::Params* p) {
  if (check_params(p)) return nullptr;
  return new Sim<Dual>(*p);
}
void orc_tan_destroy(void* h) { delete static_cast<Sim<Dual>*>(h); }

int orc_tan_init(void* h, const double* phi0, const double* dphi0, double dsigma, const double* rho0,
                 const double* u0) {
  Sim<Dual>* s = static_cast<Sim<Dual>*>(h);
  std::vector<Dual> p0(s->N);
  for (long c = 0; c < s->N; ++c) p0[c] = Dual(phi0[c], dphi0 ? dphi0[c] : 0.0);
  s->sig = Dual(s->P.sigma, dsigma);
  s->init(p0.data(), rho0, u0);
  return 0;
}

int orc_tan_step(void* h, int n) {
  Sim<Dual>* s = static_cast<Sim<Dual>*>(h);
  for (int k = 0; k < n; ++k) s->step();
  return 0;
}

int orc_tan_centroid(void* h, int axis, double* value, double* tangent) {
  Sim<Dual>* s = static_cast<Sim<Dual>*>(h);
  Dual V, xc[3];
  s->centroid(V, xc);
  *value = xc[axis].v;
  *tangent = xc[axis].d;
  return 0;
}

int orc_tan_get_pop(void* h, double* val, double* tan) {
  Sim<Dual>* s = static_cast<Sim<Dual>*>(h);
  for (size_t k = 0; k < s->A.size(); ++k) { val[k] = s->A[k].v; if (tan) tan[k] = s->A[k].d; }
  return 0;
}

}  // extern "C"
