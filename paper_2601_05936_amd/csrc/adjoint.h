// adjoint.h -- reverse mode of the time step (differentiation pattern) for
// the two-dimensional lattice (D2Q9), FP64 or FP32 state, FP64 adjoints.
//
// The step is reversed sub-step by sub-step under the decisions of the
// recorded forward step (phase and band tags, cut and wall links, Bouzidi
// branch, upwind directions, the clamp at +-B, refill events, the Godunov
// branches and subcell-fix set of the reinitialisation).  Every reverse
// kernel takes one output unit (a cell), evaluates the forward arithmetic of
// that unit once to enumerate the inputs it reads, then once per input with
// a dual number seeded on that input, and adds the transposed Jacobian
// column times the output adjoint to the input's adjoint (FP64 atomics).
// The per-unit functions below restate the forward kernels' arithmetic for
// dual numbers; the forward states come from snapshots recorded while the
// forward kernels themselves re-run a checkpoint segment.
#pragma once

#include "kernels.h"

namespace lsb {
namespace adj {

// ---------------------------------------------------------------------------
// Dual number (value and one derivative).  Comparisons act on the value, so
// every branch follows the recorded forward decision.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  __device__ Dual() : v(0.0), d(0.0) {}
  __device__ Dual(double a) : v(a), d(0.0) {}
  __device__ Dual(double a, double b) : v(a), d(b) {}
};
__device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ inline Dual operator/(Dual a, Dual b) {
  const double r = a.v / b.v;
  return Dual(r, (a.d - r * b.d) / b.v);
}
__device__ inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ inline Dual& operator+=(Dual& a, Dual b) { return a = a + b; }
__device__ inline Dual& operator-=(Dual& a, Dual b) { return a = a - b; }
__device__ inline Dual dsqrt(Dual a) {
  const double s = sqrt(a.v);
  return Dual(s, s > 0.0 ? 0.5 * a.d / s : 0.0);
}
__device__ inline Dual dfabs(Dual a) { return a.v < 0.0 ? -a : a; }

// ---------------------------------------------------------------------------
// Arrays a reverse kernel may read (primal value) and accumulate into
// (adjoint).  Step n maps the state (A_n, M_n, phi_n, G_n, Pb_n) to step
// n + 1; MNEW / ANEW are the collide-stream outputs of step n (before the
// refill), UT the extension velocity after a given sweep.
// ---------------------------------------------------------------------------
enum ArrId {
  AR_AIN = 0, AR_MIN, AR_PHI0, AR_GIN, AR_PB, AR_SIG, AR_MNEW, AR_ANEW, AR_PHI1, AR_GNEW, AR_UT, AR_UTOUT, AR_S1, AR_S2,
  AR_XC0,
  // reinitialisation: level set before it (after the advection), and the
  // pseudo step's level set and RK3 stage values
  AR_P0, AR_RPHI, AR_RS1, AR_RS2, AR_NUM
};

template <class R>
struct View {
  const R* val[AR_NUM];        // primal arrays (scalars: see sval)
  double* bar[AR_NUM];         // adjoint accumulators
  const double* sval[AR_NUM];  // scalar primal values (AR_PB, AR_SIG, AR_XC0)
  const uint8_t* tag0;         // tags of step n
  const uint8_t* tag1;         // tags of step n + 1
  int nx, ny, nz, N;
  int per[3], bcf[6];
  double wall_u[6][3];
  double omega[2], acc[2][3], rho_phys[2], eta[2];
  double band, band_snap, ext_dtau, heps, reinit_dtau;
};

constexpr int KSLOT = 3;           // list entries per lane
constexpr int KMAX = 64 * KSLOT;   // inputs of one unit
static_assert(KSLOT == 3, "reverse_unit selects among three slots");

// Accessor: enumeration (records the distinct inputs read) or seeded
// evaluation (derivative 1 on the target input).  All 64 lanes of a
// wavefront evaluate the same unit, so the list of inputs is held across
// the wave's registers: entry e sits on lane e % 64 in slot e / 64, a lookup
// is one comparison per slot and a ballot, and in the seeded pass each lane
// takes its own entries as targets.
template <class R>
struct Acc {
  const View<R>* v;
  int mode;  // 0 enumerate, 1 seeded
  int tarr;
  long tidx;
  int n;     // entries recorded (uniform over the wave)
  int lane;
  bool overflow;
  int sarr[KSLOT];
  int sidx[KSLOT];

  __device__ double load(int arr, long idx) const {
    if (arr == AR_PB || arr == AR_SIG || arr == AR_XC0) return v->sval[arr][idx];
    return (double)v->val[arr][idx];
  }
  __device__ Dual get(int arr, long idx) {
    // the stage values of the advection and the reinitialisation equal
    // phi_n outside the band of step n (those cells are not updated)
    if ((arr == AR_S1 || arr == AR_S2 || arr >= AR_P0) && !(v->tag0[idx] & T_ACT)) arr = AR_PHI0;
    const double x = load(arr, idx);
    if (mode == 0) {
      bool hit = false;
#pragma unroll
      for (int k = 0; k < KSLOT; ++k) hit = hit || (lane + 64 * k < n && sarr[k] == arr && sidx[k] == (int)idx);
      if (__ballot(hit) == 0) {
        if (n < KMAX) {
          if (lane == (n & 63)) {
#pragma unroll
            for (int k = 0; k < KSLOT; ++k)
              if (k == (n >> 6)) { sarr[k] = arr; sidx[k] = (int)idx; }
          }
          ++n;
        } else {
          overflow = true;
        }
      }
      return Dual(x);
    }
    return Dual(x, (arr == tarr && idx == tidx) ? 1.0 : 0.0);
  }
};

// Reverse of one unit by the 64 lanes of a wavefront (all lanes call it for
// the same unit, converged): F(acc, out) evaluates the unit's forward
// arithmetic and writes NOUT outputs; ybar are their adjoints.  One
// enumeration pass lists the inputs, then each lane evaluates with the
// derivative seeded on its own entries (lane l: inputs l, l + 64, ...).
template <class R, int NOUT, class F>
__device__ void reverse_unit(const View<R>& v, const double* ybar, F&& f, int* overflow_flag) {
  bool any = false;
  for (int j = 0; j < NOUT; ++j) any = any || ybar[j] != 0.0;
  if (!any) return;
  Acc<R> acc;
  acc.v = &v;
  acc.mode = 0;
  acc.n = 0;
  acc.lane = (int)(threadIdx.x & 63u);
  acc.overflow = false;
  acc.tarr = -1;
  acc.tidx = -1;
  for (int k = 0; k < KSLOT; ++k) acc.sarr[k] = acc.sidx[k] = -1;
  Dual out[NOUT];
  f(acc, out);
  if (acc.overflow && acc.lane == 0) atomicOr(overflow_flag, 1);
  const int nin = acc.n;
  acc.mode = 1;
  for (int k = 0; k * 64 < nin; ++k) {
    const bool mine = acc.lane + 64 * k < nin;
    const int a = k == 0 ? acc.sarr[0] : (k == 1 ? acc.sarr[1] : acc.sarr[KSLOT - 1]);
    const int i = k == 0 ? acc.sidx[0] : (k == 1 ? acc.sidx[1] : acc.sidx[KSLOT - 1]);
    acc.tarr = mine ? a : -1;
    acc.tidx = mine ? i : -1;
    f(acc, out);
    double g = 0.0;
    for (int j = 0; j < NOUT; ++j) g += ybar[j] * out[j].d;
    if (mine && g != 0.0) {
      const long idx = (a == AR_PB || a == AR_SIG) ? 0 : i;
      atomicAdd(&v.bar[a][idx], g);
    }
  }
}

__device__ inline int coord_lb(int s, int n, int periodic) {
  if (s >= 0 && s < n) return s;
  if (!periodic) return -1;
  return s < 0 ? s + n : s - n;
}
__device__ inline int coord_ls(int s, int n, int periodic) {
  if (s >= 0 && s < n) return s;
  if (periodic) return s < 0 ? s + n * ((-s + n - 1) / n) : s % n;
  return s < 0 ? -1 - s : 2 * n - 1 - s;
}

// ---------------------------------------------------------------------------
// Forward arithmetic per unit (dual numbers), D2Q9 restated from the
// forward kernels.
// ---------------------------------------------------------------------------
using L9 = Lat<LSB_D2Q9>;
constexpr int Q9 = 9;

// interface bounce-back of link i at cell c (phase k) from the other-phase
// cell sc (eq:bb with eq:bb_cc and the stress jump eq:Sdecomp)
template <class R>
__device__ Dual iface_pull(Acc<R>& A, int c, int x, int y, int sc, int i, int k) {
  const View<R>& v = *A.v;
  const long N = v.N;
  const int cc[3] = {L9::cx(i), L9::cy(i), 0};
  const int j = opp<LSB_D2Q9>(i);
  const double w = wgt<LSB_D2Q9>(i);
  const Dual px = A.get(AR_PHI0, c), py = A.get(AR_PHI0, sc);
  const Dual q = px / (px - py);
  Dual uG[3], nG[3];
  for (int m = 0; m < 3; ++m) uG[m] = (Dual(1.0) - q) * A.get(AR_MIN, (1 + m) * N + c) + q * A.get(AR_MIN, (1 + m) * N + sc);
  Dual nn(0.0);
  for (int m = 0; m < 3; ++m) {
    nG[m] = (Dual(1.0) - q) * A.get(AR_GIN, m * N + c) + q * A.get(AR_GIN, m * N + sc);
    nn += nG[m] * nG[m];
  }
  const Dual nl = dsqrt(nn);
  if (nl.v > 1e-30) for (int m = 0; m < 3; ++m) nG[m] = nG[m] / nl;
  const Dual kG = (Dual(1.0) - q) * A.get(AR_GIN, 3 * N + c) + q * A.get(AR_GIN, 3 * N + sc);
  const int o = 1 - k;
  const Dual pb = A.get(AR_PB, 0);
  Dual p_own = Dual(v.rho_phys[k] / 3.0) * A.get(AR_MIN, c) + (k == 1 ? pb : Dual(0.0));
  Dual p_oth = Dual(v.rho_phys[o] / 3.0) * A.get(AR_MIN, sc) + (o == 1 ? pb : Dual(0.0));
  for (int m = 0; m < 3; ++m) {
    p_own = p_own + Dual(v.rho_phys[k] * v.acc[k][m] * (double)(-cc[m])) * q;
    p_oth = p_oth + Dual(v.rho_phys[o] * v.acc[o][m] * (double)cc[m]) * (Dual(1.0) - q);
  }
  const Dual p_l = k == 0 ? p_own : p_oth;
  const Dual p_g = k == 0 ? p_oth : p_own;
  const double eta_bar = 0.5 * (v.eta[0] + v.eta[1]);
  const double jeta = v.eta[1] - v.eta[0];
  const double rmax = v.rho_phys[0] > v.rho_phys[1] ? v.rho_phys[0] : v.rho_phys[1];
  const double eta_p = eta_bar >= rmax / 24.0 ? eta_bar : rmax / 12.0;
  const Dual sig = A.get(AR_SIG, 0);
  const Dual E = ((p_g - p_l) + sig * kG) / Dual(2.0 * eta_p);
  Dual Sb[6];
  for (int m = 0; m < 6; ++m) Sb[m] = Dual(0.5) * (A.get(AR_MIN, (4 + m) * N + c) + A.get(AR_MIN, (4 + m) * N + sc));
  const double acoef = -jeta / eta_bar;
  const Dual Sm[3][3] = {{Sb[0], Sb[3], Sb[4]}, {Sb[3], Sb[1], Sb[5]}, {Sb[4], Sb[5], Sb[2]}};
  const Dual cn = Dual((double)cc[0]) * nG[0] + Dual((double)cc[1]) * nG[1] + Dual((double)cc[2]) * nG[2];
  Dual nAn(0.0), nAc(0.0);
  for (int p = 0; p < 3; ++p)
    for (int r = 0; r < 3; ++r) {
      nAn = nAn + Dual(acoef) * nG[p] * Sm[p][r] * nG[r];
      nAc = nAc + Dual(acoef) * nG[p] * Sm[p][r] * Dual((double)cc[r]);
    }
  const Dual cSc = cn * cn * E + Dual(2.0) * cn * nAc - cn * cn * nAn;
  const double s_own = k == 0 ? 1.0 : -1.0;
  const Dual cu = Dual((double)cc[0]) * uG[0] + Dual((double)cc[1]) * uG[1] + Dual((double)cc[2]) * uG[2];
  const Dual W = Dual(6.0 * w) * (cu + q * (Dual(1.0) - q) * Dual(s_own) * cSc);
  const Dual dj = A.get(AR_AIN, j * N + c);
  if (q.v < 0.5) {
    const int fx = coord_lb(x + cc[0], v.nx, v.per[0]);
    const int fy = coord_lb(y + cc[1], v.ny, v.per[1]);
    if ((fx | fy) >= 0) {
      const int fc = fy * v.nx + fx;
      if ((v.tag0[fc] & T_GAS) == k) {
        const Dual djf = A.get(AR_AIN, j * N + fc);
        return Dual(2.0) * q * dj + (Dual(1.0) - Dual(2.0) * q) * djf + W;
      }
    }
    return dj + W;
  }
  const Dual di = A.get(AR_AIN, i * N + c);
  return dj / (Dual(2.0) * q) + (Dual(2.0) * q - Dual(1.0)) / (Dual(2.0) * q) * di + W / (Dual(2.0) * q);
}

// Source of the pull of direction i at cell c when no interface is
// crossed: streaming from the upstream cell, halfway bounce-back at a
// no-slip face (own cell, opposite direction, plus the moving-wall term cst)
// or specular reflection at a free-slip face (reflected direction at the
// mirrored cell).  sc is the cell whose phase decides whether the pull
// crosses the interface (-1 for no-slip faces), refl marks reflections.
struct Src {
  long idx;
  double cst;
  int sc;
  bool refl;
};

template <class V>
__device__ Src plain_source(const V& v, int c, int x, int y, int i) {
  const long N = v.N;
  const int cx = L9::cx(i), cy = L9::cy(i);
  const int sx = coord_lb(x - cx, v.nx, v.per[0]);
  const int sy = coord_lb(y - cy, v.ny, v.per[1]);
  if ((sx | sy) >= 0) {
    const int sc = sy * v.nx + sx;
    return Src{(long)i * N + sc, 0.0, sc, false};
  }
  const int pos[2] = {x, y};
  const int cc[2] = {cx, cy};
  const int sv[2] = {sx, sy};
  int src[2], rc[2];
  for (int ax = 0; ax < 2; ++ax) {
    src[ax] = sv[ax] < 0 ? pos[ax] : sv[ax];
    rc[ax] = sv[ax] < 0 ? -cc[ax] : cc[ax];
  }
  for (int ax = 0; ax < 2; ++ax) {
    if (sv[ax] >= 0) continue;
    const int face = 2 * ax + (pos[ax] - cc[ax] < 0 ? 0 : 1);
    if (v.bcf[face] == LSB_NOSLIP) {
      const double cu = cc[0] * v.wall_u[face][0] + cc[1] * v.wall_u[face][1];
      return Src{(long)opp<LSB_D2Q9>(i) * N + c, 6.0 * wgt<LSB_D2Q9>(i) * cu, -1, false};
    }
  }
  const int sc = src[1] * v.nx + src[0];
  int ir = 0;
  for (int m = 0; m < Q9; ++m)
    if (L9::cx(m) == rc[0] && L9::cy(m) == rc[1]) ir = m;
  return Src{(long)ir * N + sc, 0.0, sc, true};
}

// incoming deviation of direction i at cell c (phase k) of step n; at
// interface-adjacent cells a pull whose source lies in the other phase is
// the interface bounce-back (a reflected source: bounce-back at the cell)
template <class R>
__device__ Dual pull(Acc<R>& A, int c, int x, int y, int i, int k, bool spec) {
  const View<R>& v = *A.v;
  const Src s = plain_source(v, c, x, y, i);
  if (spec && s.sc >= 0 && (v.tag0[s.sc] & T_GAS) != k) {
    if (s.refl) return A.get(AR_AIN, (long)opp<LSB_D2Q9>(i) * v.N + c);
    return iface_pull(A, c, x, y, s.sc, i, k);
  }
  const Dual d = A.get(AR_AIN, s.idx);
  return s.cst != 0.0 ? d + Dual(s.cst) : d;
}

// BGK collision with body force of the incoming deviations f of a cell of
// phase k: out[0..8] populations of step n + 1, out[9..18] the moments
// (rho - 1, u, S) written on LS-active cells
template <class View_>
__device__ void collision(const View_& v, int k, const Dual* f, Dual* out) {
  Dual rp(0.0), m0(0.0), m1(0.0);
  for (int i = 0; i < Q9; ++i) {
    rp += f[i];
    m0 += Dual((double)L9::cx(i)) * f[i];
    m1 += Dual((double)L9::cy(i)) * f[i];
  }
  const Dual rho = Dual(1.0) + rp;
  const Dual inv = Dual(1.0) / rho;
  const Dual ux = m0 * inv, uy = m1 * inv;
  const Dual uu = ux * ux + uy * uy;
  const double om = v.omega[k];
  const double fx = 3.0 * v.acc[k][0], fy = 3.0 * v.acc[k][1];
  Dual P0(0.0), P1(0.0), P3(0.0);
  for (int i = 0; i < Q9; ++i) {
    const double w = wgt<LSB_D2Q9>(i);
    const double cx = L9::cx(i), cy = L9::cy(i);
    const Dual cu = Dual(cx) * ux + Dual(cy) * uy;
    const Dual deq = Dual(w) * (rp + rho * (Dual(3.0) * cu + Dual(4.5) * cu * cu - Dual(1.5) * uu));
    const Dual fn = f[i] - deq;
    P0 += Dual(cx * cx) * fn;
    P1 += Dual(cy * cy) * fn;
    P3 += Dual(cx * cy) * fn;
    out[i] = f[i] - Dual(om) * fn + Dual(w * (cx * fx + cy * fy)) * rho;
  }
  const Dual fac = Dual(-1.5 * om) * inv;
  out[9] = rp;
  out[10] = ux;
  out[11] = uy;
  out[12] = Dual(0.0);
  out[13] = fac * P0;
  out[14] = fac * P1;
  out[15] = Dual(0.0);
  out[16] = fac * P3;
  out[17] = Dual(0.0);
  out[18] = Dual(0.0);
}

// extension seed at an interface-adjacent cell: mean over the cut links of
// the velocity interpolated to the interface (out[0..2])
template <class R>
__device__ void seed_iface(Acc<R>& A, int c, Dual* out) {
  const View<R>& v = *A.v;
  const long N = v.N;
  const int x = c % v.nx, y = c / v.nx;
  const int k = v.tag0[c] & T_GAS;
  const Dual pc = A.get(AR_PHI0, c);
  Dual acc[3] = {Dual(0.0), Dual(0.0), Dual(0.0)};
  int cnt = 0;
  for (int i = 0; i < Q9; ++i) {
    if (c2<LSB_D2Q9>(i) == 0) continue;
    const int sx = coord_lb(x - L9::cx(i), v.nx, v.per[0]);
    const int sy = coord_lb(y - L9::cy(i), v.ny, v.per[1]);
    if ((sx | sy) < 0) continue;
    const int sc = sy * v.nx + sx;
    if ((v.tag0[sc] & T_GAS) == k) continue;
    const Dual q = pc / (pc - A.get(AR_PHI0, sc));
    for (int m = 0; m < 3; ++m)
      acc[m] += (Dual(1.0) - q) * A.get(AR_MNEW, (1 + m) * N + c) + q * A.get(AR_MNEW, (1 + m) * N + sc);
    ++cnt;
  }
  for (int m = 0; m < 3; ++m) out[m] = acc[m] / Dual((double)cnt);
}

// one upwind extension sweep at an LS-active, not interface-adjacent cell:
// reads the velocity of the previous sweep (AR_UT), writes out[0..2]
template <class R>
__device__ void ext_sweep(Acc<R>& A, int c, Dual* out) {
  const View<R>& v = *A.v;
  const long N = v.N;
  const int x = c % v.nx, y = c / v.nx;
  Dual u[3];
  for (int m = 0; m < 3; ++m) u[m] = A.get(AR_UT, m * N + c);
  const Dual ph = A.get(AR_PHI0, c);
  const Dual sg = ph / dsqrt(ph * ph + Dual(1.0));
  const int pos[2] = {x, y};
  const int n[2] = {v.nx, v.ny};
  Dual o[3] = {u[0], u[1], u[2]};
  for (int ax = 0; ax < 2; ++ax) {
    const Dual vv = sg * A.get(AR_GIN, ax * N + c);
    if (vv.v == 0.0) continue;
    const int dir = vv.v > 0.0 ? -1 : 1;
    const int s = coord_lb(pos[ax] + dir, n[ax], v.per[ax]);
    // beyond a free-slip face: the cell's mirror image (normal component
    // reversed); beyond a no-slip face: skipped
    if (s < 0 && v.bcf[2 * ax + (dir > 0 ? 1 : 0)] != LSB_FREESLIP) continue;
    int p2[2] = {x, y};
    p2[ax] = s < 0 ? pos[ax] : s;
    const int nc = p2[1] * v.nx + p2[0];
    if (!(v.tag0[nc] & T_ACT)) continue;
    for (int m = 0; m < 3; ++m) {
      const Dual w = A.get(AR_UT, m * N + nc);
      const Dual un = (s < 0 && m == ax) ? Dual(0.0) - w : w;
      const Dual diff = vv.v > 0.0 ? (u[m] - un) : (un - u[m]);
      o[m] = o[m] - Dual(v.ext_dtau) * vv * diff;
    }
  }
  for (int m = 0; m < 3; ++m) out[m] = o[m];
}

// fifth-order upwind derivative along one axis (positive: upwind from -)
__device__ inline Dual upwind5(Dual fm3, Dual fm2, Dual fm1, Dual f0, Dual fp1, Dual fp2, Dual fp3, bool positive) {
  if (positive)
    return (Dual(-2.0) * fm3 + Dual(15.0) * fm2 - Dual(60.0) * fm1 + Dual(20.0) * f0 + Dual(30.0) * fp1 -
            Dual(3.0) * fp2) / Dual(60.0);
  return (Dual(3.0) * fm2 - Dual(30.0) * fm1 - Dual(20.0) * f0 + Dual(60.0) * fp1 - Dual(15.0) * fp2 +
          Dual(2.0) * fp3) / Dual(60.0);
}

// TVD-RK3 stage at an LS-active cell of step n (out[0]); the extension
// velocity is the last sweep's (AR_UTOUT)
template <class R>
__device__ void rk_stage(Acc<R>& A, int c, int stage, Dual* out) {
  const View<R>& v = *A.v;
  const long N = v.N;
  const int x = c % v.nx, y = c / v.nx;
  const int in = stage == 1 ? AR_PHI0 : (stage == 2 ? AR_S1 : AR_S2);
  Dual r(0.0);
  for (int ax = 0; ax < 2; ++ax) {
    const Dual u = A.get(AR_UTOUT, ax * N + c);
    Dual f[7];
    for (int o = -3; o <= 3; ++o) {
      int p[2] = {x, y};
      const int n[2] = {v.nx, v.ny};
      p[ax] = coord_ls(p[ax] + o, n[ax], v.per[ax]);
      f[o + 3] = A.get(in, p[1] * v.nx + p[0]);
    }
    const Dual dd = upwind5(f[0], f[1], f[2], f[3], f[4], f[5], f[6], u.v >= 0.0);
    r = r - u * dd;
  }
  const Dual vv = A.get(in, c) + r;
  Dual o;
  if (stage == 1) o = vv;
  else if (stage == 2) o = Dual(0.75) * A.get(AR_PHI0, c) + Dual(0.25) * vv;
  else {
    o = Dual(1.0 / 3.0) * A.get(AR_PHI0, c) + Dual(2.0 / 3.0) * vv;
    if (o.v > v.band_snap) o = Dual(v.band);
    if (o.v < -v.band_snap) o = Dual(-v.band);
  }
  out[0] = o;
}

// WENO5 of five successive differences (the forward kernel's weights)
__device__ inline Dual weno5d(Dual v1, Dual v2, Dual v3, Dual v4, Dual v5) {
  const double eps = 1e-6;
  const Dual p0 = v1 * Dual(1.0 / 3.0) - v2 * Dual(7.0 / 6.0) + v3 * Dual(11.0 / 6.0);
  const Dual p1 = -v2 * Dual(1.0 / 6.0) + v3 * Dual(5.0 / 6.0) + v4 * Dual(1.0 / 3.0);
  const Dual p2 = v3 * Dual(1.0 / 3.0) + v4 * Dual(5.0 / 6.0) - v5 * Dual(1.0 / 6.0);
  const Dual a0 = v1 - Dual(2.0) * v2 + v3, b0 = v1 - Dual(4.0) * v2 + Dual(3.0) * v3;
  const Dual a1 = v2 - Dual(2.0) * v3 + v4, b1 = v2 - v4;
  const Dual a2 = v3 - Dual(2.0) * v4 + v5, b2 = Dual(3.0) * v3 - Dual(4.0) * v4 + v5;
  const Dual s0 = Dual(13.0 / 12.0) * a0 * a0 + Dual(0.25) * b0 * b0;
  const Dual s1 = Dual(13.0 / 12.0) * a1 * a1 + Dual(0.25) * b1 * b1;
  const Dual s2 = Dual(13.0 / 12.0) * a2 * a2 + Dual(0.25) * b2 * b2;
  const Dual e0 = Dual(eps) + s0, e1 = Dual(eps) + s1, e2 = Dual(eps) + s2;
  const Dual w0 = Dual(0.1) / (e0 * e0), w1 = Dual(0.6) / (e1 * e1), w2 = Dual(0.3) / (e2 * e2);
  return (w0 * p0 + w1 * p1 + w2 * p2) / (w0 + w1 + w2);
}

// One pseudo-time RK3 stage of the reinitialisation at an LS-active cell:
// stage 1 reads the pseudo step's level set (AR_RPHI), stage 2 its first
// stage value (AR_RS1), stage 3 its second (AR_RS2); stages 2 and 3 blend
// with AR_RPHI.  The smoothed sign and the subcell fix next to the zero set
// use the level set before the reinitialisation (AR_P0); the Godunov
// branches, the fix set and the clamp at +-B (last stage of the last pseudo
// step) follow the primal values.
template <class R>
__device__ void reinit_stage(Acc<R>& A, int c, int stage, bool last, Dual* out) {
  const View<R>& v = *A.v;
  const int x = c % v.nx, y = c / v.nx;
  const int in = stage == 1 ? AR_RPHI : (stage == 2 ? AR_RS1 : AR_RS2);
  auto at = [&](int ax, int o) {
    int p[2] = {x, y};
    const int n[2] = {v.nx, v.ny};
    p[ax] = coord_ls(p[ax] + o, n[ax], v.per[ax]);
    return p[1] * v.nx + p[0];
  };
  const Dual ph0 = A.get(AR_P0, c);
  const Dual S0 = ph0 / dsqrt(ph0 * ph0 + Dual(1.0));
  const Dual c0 = A.get(in, c);
  Dual h2(0.0);
  for (int ax = 0; ax < 2; ++ax) {
    const Dual m3 = A.get(in, at(ax, -3)), m2 = A.get(in, at(ax, -2)), m1 = A.get(in, at(ax, -1));
    const Dual q1 = A.get(in, at(ax, 1)), q2 = A.get(in, at(ax, 2)), q3 = A.get(in, at(ax, 3));
    const Dual dm = weno5d(m2 - m3, m1 - m2, c0 - m1, q1 - c0, q2 - q1);
    const Dual dp = weno5d(q3 - q2, q2 - q1, q1 - c0, c0 - m1, m1 - m2);
    Dual aa(0.0), bb(0.0);
    if (S0.v > 0.0) {
      if (dm.v > 0.0) aa = dm;
      if (dp.v < 0.0) bb = dp;
    } else {
      if (dm.v < 0.0) aa = dm;
      if (dp.v > 0.0) bb = dp;
    }
    const Dual a2 = aa * aa, b2 = bb * bb;
    h2 += a2.v > b2.v ? a2 : b2;
  }
  Dual rt = -S0 * (dsqrt(h2) - Dual(1.0));
  // subcell fix: the cell has an axis neighbour across the zero set of phi0
  const bool g0 = ph0.v >= 0.0;
  bool fix = false;
  for (int ax = 0; ax < 2; ++ax)
    for (int sg = -1; sg <= 1; sg += 2) fix = fix || ((A.load(AR_P0, at(ax, sg)) >= 0.0) != g0);
  if (fix) {
    Dual acc(0.0);
    int cnt = 0;
    for (int ax = 0; ax < 2; ++ax)
      for (int sg = -1; sg <= 1; sg += 2) {
        const int j = at(ax, sg);
        const Dual pj = A.get(AR_P0, j);
        if ((pj.v >= 0.0) == g0) continue;
        acc += ph0 * (c0 - A.get(in, j)) / (ph0 - pj);
        ++cnt;
      }
    rt += Dual(0.5) * (acc / Dual((double)cnt) - c0);
  }
  const Dual vv = c0 + Dual(v.reinit_dtau) * rt;
  Dual o;
  if (stage == 1) {
    o = vv;
  } else if (stage == 2) {
    o = Dual(0.75) * A.get(AR_RPHI, c) + Dual(0.25) * vv;
  } else {
    o = Dual(1.0 / 3.0) * A.get(AR_RPHI, c) + Dual(2.0 / 3.0) * vv;
    if (last) {
      if (o.v > v.band_snap) o = Dual(v.band);
      if (o.v < -v.band_snap) o = Dual(-v.band);
    }
  }
  out[0] = o;
}

// geometry (normal, curvature) at cell c from the level set `arr`
template <class R>
__device__ void geometry(Acc<R>& A, int c, int arr, Dual* out) {
  const View<R>& v = *A.v;
  const int x = c % v.nx, y = c / v.nx;
  auto at = [&](int dx, int dy) {
    const int sx = coord_ls(x + dx, v.nx, v.per[0]);
    const int sy = coord_ls(y + dy, v.ny, v.per[1]);
    return A.get(arr, sy * v.nx + sx);
  };
  const Dual p = A.get(arr, c);
  const Dual gx = Dual(0.5) * (at(1, 0) - at(-1, 0));
  const Dual gy = Dual(0.5) * (at(0, 1) - at(0, -1));
  const Dual xx = at(1, 0) - Dual(2.0) * p + at(-1, 0);
  const Dual yy = at(0, 1) - Dual(2.0) * p + at(0, -1);
  const Dual xy = Dual(0.25) * (at(1, 1) - at(1, -1) - at(-1, 1) + at(-1, -1));
  const Dual g2 = gx * gx + gy * gy;
  const Dual g = dsqrt(g2);
  if (g.v < 1e-12) {
    for (int m = 0; m < 4; ++m) out[m] = Dual(0.0);
    return;
  }
  out[0] = gx / g;
  out[1] = gy / g;
  out[2] = Dual(0.0);
  const Dual num = xx * (gy * gy) + yy * (gx * gx) - Dual(2.0) * gx * gy * xy;
  out[3] = num / (g2 * g);
}

// refill of a cell whose phase changed in step n: out[0..8] populations,
// out[9..18] moments
template <class R>
__device__ void refill(Acc<R>& A, int c, Dual* out) {
  const View<R>& v = *A.v;
  const long N = v.N;
  const int x = c % v.nx, y = c / v.nx;
  const uint8_t t = v.tag1[c];
  const int knew = t & T_GAS;
  const int kold = (t & T_OLDGAS) ? 1 : 0;
  const double sgn = knew == 1 ? 1.0 : -1.0;
  // candidate directions by alignment with the normal into the new phase
  // (a decision: taken on the primal values)
  const double g0 = A.load(AR_GNEW, c), g1 = A.load(AR_GNEW, N + c);
  const double m0 = sgn * g0, m1 = sgn * g1;
  int order[Q9];
  double score[Q9];
  int nc = 0;
  for (int i = 0; i < Q9; ++i) {
    const int cx = L9::cx(i), cy = L9::cy(i);
    const int l2 = cx * cx + cy * cy;
    if (l2 == 0) continue;
    const double sc = (cx * m0 + cy * m1) / sqrt((double)l2);
    if (!(sc > 0.0)) continue;
    int p = nc++;
    order[p] = i;
    score[p] = sc;
    while (p > 0 && score[p - 1] < sc) {
      order[p] = order[p - 1]; score[p] = score[p - 1];
      order[p - 1] = i; score[p - 1] = sc;
      --p;
    }
  }
  const Dual rhoO = A.get(AR_MNEW, c);
  const Dual uG[3] = {A.get(AR_MNEW, N + c), A.get(AR_MNEW, 2 * N + c), A.get(AR_MNEW, 3 * N + c)};
  const Dual pb = A.get(AR_PB, 0);
  const Dual pold = Dual(v.rho_phys[kold] / 3.0) * rhoO + (kold == 1 ? pb : Dual(0.0));
  const Dual kap = A.get(AR_GNEW, 3 * N + c);
  const Dual sig = A.get(AR_SIG, 0);
  const Dual pnew = knew == 0 ? pold + sig * kap : pold - sig * kap;
  const Dual rhoG = (pnew - (knew == 1 ? pb : Dual(0.0))) / Dual(v.rho_phys[knew] / 3.0);
  auto established = [&](int sc) {
    const uint8_t ts = v.tag1[sc];
    return (ts & T_GAS) == knew && ((ts & T_OLDGAS) ? 1 : 0) == knew;
  };
  for (int tt = 0; tt < nc; ++tt) {
    const int i = order[tt];
    const int ex = L9::cx(i), ey = L9::cy(i);
    const int x1 = coord_lb(x + ex, v.nx, v.per[0]), y1 = coord_lb(y + ey, v.ny, v.per[1]);
    if ((x1 | y1) < 0) continue;
    const int c1 = y1 * v.nx + x1;
    if (!established(c1)) continue;
    const int x2 = coord_lb(x + 2 * ex, v.nx, v.per[0]), y2 = coord_lb(y + 2 * ey, v.ny, v.per[1]);
    int c2c = -1;
    if ((x2 | y2) >= 0) {
      const int cc2 = y2 * v.nx + x2;
      if (established(cc2)) c2c = cc2;
    }
    const bool two = c2c >= 0;
    Dual q;
    const int xm = coord_lb(x - ex, v.nx, v.per[0]), ym = coord_lb(y - ey, v.ny, v.per[1]);
    const Dual phc = A.get(AR_PHI1, c);
    bool crossed = false;
    if ((xm | ym) >= 0) {
      const Dual phm = A.get(AR_PHI1, ym * v.nx + xm);
      if ((phm.v >= 0.0) != (phc.v >= 0.0)) {
        crossed = true;
        q = phc / (phc - phm);
      }
    }
    if (!crossed) {
      const double len = sqrt((double)(ex * ex + ey * ey));
      const Dual en = (Dual((double)ex) * A.get(AR_GNEW, c) + Dual((double)ey) * A.get(AR_GNEW, N + c)) / Dual(len);
      const Dual aen = dfabs(en);
      if (aen.v < 1e-12) q = Dual(1.0);
      else {
        q = dfabs(phc) / (aen * Dual(len));
        if (q.v > 1.0) q = Dual(1.0);
      }
    }
    Dual w0, w1, w2(0.0);
    if (two) {
      w0 = Dual(2.0) / ((q + Dual(1.0)) * (q + Dual(2.0)));
      w1 = Dual(2.0) * q / (q + Dual(1.0));
      w2 = -q / (q + Dual(2.0));
    } else {
      w0 = Dual(1.0) / (Dual(1.0) + q);
      w1 = q / (Dual(1.0) + q);
    }
    const Dual rhoB = v.rho_phys[knew] >= v.rho_phys[kold] ? rhoG : A.get(AR_MNEW, c1);
    const Dual rr = w0 * rhoB + w1 * A.get(AR_MNEW, c1) + (two ? w2 * A.get(AR_MNEW, c2c) : Dual(0.0));
    Dual ur[3];
    for (int m = 0; m < 3; ++m)
      ur[m] = w0 * uG[m] + w1 * A.get(AR_MNEW, (1 + m) * N + c1) + (two ? w2 * A.get(AR_MNEW, (1 + m) * N + c2c) : Dual(0.0));
    const Dual r1 = A.get(AR_MNEW, c1);
    const Dual u1[3] = {A.get(AR_MNEW, N + c1), A.get(AR_MNEW, 2 * N + c1), A.get(AR_MNEW, 3 * N + c1)};
    const Dual uur = ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2];
    const Dual uu1 = u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2];
    for (int k = 0; k < Q9; ++k) {
      const double w = wgt<LSB_D2Q9>(k);
      const Dual cur = Dual((double)L9::cx(k)) * ur[0] + Dual((double)L9::cy(k)) * ur[1];
      const Dual cu1 = Dual((double)L9::cx(k)) * u1[0] + Dual((double)L9::cy(k)) * u1[1];
      const Dual de = Dual(w) * (rr + (Dual(1.0) + rr) * (Dual(3.0) * cur + Dual(4.5) * cur * cur - Dual(1.5) * uur));
      const Dual de1 = Dual(w) * (r1 + (Dual(1.0) + r1) * (Dual(3.0) * cu1 + Dual(4.5) * cu1 * cu1 - Dual(1.5) * uu1));
      const Dual d1 = A.get(AR_ANEW, k * N + c1);
      out[k] = de + (d1 - de1);
    }
    out[9] = rr;
    for (int m = 0; m < 3; ++m) out[10 + m] = ur[m];
    for (int m = 0; m < 6; ++m) out[13 + m] = A.get(AR_MNEW, (4 + m) * N + c1);
    return;
  }
  const Dual uu = uG[0] * uG[0] + uG[1] * uG[1] + uG[2] * uG[2];
  for (int k = 0; k < Q9; ++k) {
    const double w = wgt<LSB_D2Q9>(k);
    const Dual cu = Dual((double)L9::cx(k)) * uG[0] + Dual((double)L9::cy(k)) * uG[1];
    out[k] = Dual(w) * (rhoG + (Dual(1.0) + rhoG) * (Dual(3.0) * cu + Dual(4.5) * cu * cu - Dual(1.5) * uu));
  }
  out[9] = rhoG;
  for (int m = 0; m < 3; ++m) out[10 + m] = uG[m];
  for (int m = 0; m < 6; ++m) out[13 + m] = Dual(0.0);
}

__device__ inline double heaviside_prime(double phi, double eps) {
  if (phi < -eps || phi > eps) return 0.0;
  const double pi = 3.14159265358979323846;
  return 0.5 * (1.0 / eps + cos(pi * phi / eps) / eps);
}

// ---------------------------------------------------------------------------
// Reverse kernels.  All take every cell of the grid (the two-dimensional
// workloads are small) and skip those outside the sub-step's cell set.
// ---------------------------------------------------------------------------
#define ADJ_FOR_CELLS(v) for (int c = blockIdx.x * 256 + threadIdx.x; c < (v).N; c += gridDim.x * 256)

// Cells whose reverse is spread over a wavefront.  Wave w tests the 64 cells
// w, w + nchunks, w + 2 nchunks, ... (interleaved, so the band's cells spread
// evenly over the waves): `want(c)` runs once per cell on its own lane (it
// may also do a cell's cheap pass-through work), then `body(c)` runs with all
// 64 lanes for every wanted cell.  Launch with a grid of unit_blocks(N).
template <class P, class B>
__device__ void for_units(long N, P&& want, B&& body) {
  const long nchunks = (N + 63) >> 6;
  const long lane = threadIdx.x & 63u;
  const long nw = (long)gridDim.x * 4;
  for (long w = ((long)blockIdx.x * 256 + threadIdx.x) >> 6; w < nchunks; w += nw) {
    const long c = w + lane * nchunks;
    const bool on = c < N && want((int)c);
    unsigned long long m = __ballot(on);
    while (m) {
      const int b = __builtin_ctzll(m);
      m &= m - 1;
      body((int)(w + (long)b * nchunks));
    }
  }
}
__host__ __device__ inline int unit_blocks(long N) {
  const long g = (((N + 63) >> 6) + 3) >> 2;
  return (int)(g < 65536 ? g : 65536);
}

// d(centroid_axis)/d phi, times a weight: bar[c] += s * H'(phi_c) (x_c - xc) / V
template <class R>
__global__ __launch_bounds__(256) void k_centroid_adj(const R* phi, double* bar, int nx, int N, double eps,
                                                      const double* xc, const double* V, const double* wgt3) {
  for (int c = blockIdx.x * 256 + threadIdx.x; c < N; c += gridDim.x * 256) {
    const double hp = heaviside_prime((double)phi[c], eps);
    if (hp == 0.0) continue;
    const double pos[2] = {c % nx + 0.5, c / nx + 0.5};
    double g = 0.0;
    for (int a = 0; a < 2; ++a) g += wgt3[a] * hp * (pos[a] - xc[a]) / V[0];
    bar[c] += g;
  }
}

// refill, part 1: take the adjoints of the refilled values of every
// flipped cell (the forward overwrote the collide-stream outputs there)
template <class R>
__global__ __launch_bounds__(256) void k_refill_take(View<R> v, double* ytmp) {
  const long N = v.N;
  ADJ_FOR_CELLS(v) {
    const uint8_t t1 = v.tag1[c];
    if (((t1 & T_GAS) != 0) == ((t1 & T_OLDGAS) != 0)) continue;
    for (int k = 0; k < Q9; ++k) {
      ytmp[k * N + c] = v.bar[AR_ANEW][k * N + c];
      v.bar[AR_ANEW][k * N + c] = 0.0;
    }
    for (int m = 0; m < 10; ++m) {
      ytmp[(9 + m) * N + c] = v.bar[AR_MNEW][m * N + c];
      v.bar[AR_MNEW][m * N + c] = 0.0;
    }
  }
}

// refill, part 2: transposed Jacobian of the refill into its inputs
template <class R>
__global__ __launch_bounds__(256) void k_refill_adj(View<R> v, const double* ytmp, int* overflow) {
  const long N = v.N;
  for_units(
      N,
      [&](int c) {
        const uint8_t t1 = v.tag1[c];
        return ((t1 & T_GAS) != 0) != ((t1 & T_OLDGAS) != 0);
      },
      [&](int c) {
        double yb[19];
        for (int m = 0; m < 19; ++m) yb[m] = ytmp[m * N + c];
        reverse_unit<R, 19>(v, yb, [&](Acc<R>& A, Dual* out) { refill(A, c, out); }, overflow);
      });
}

// geometry of the LS-active cells of `tags` from the level set `arr`
template <class R>
__global__ __launch_bounds__(256) void k_geometry_adj(View<R> v, int use_tag1, int arr, const double* gbar, int* overflow) {
  const long N = v.N;
  for_units(
      N, [&](int c) { return ((use_tag1 ? v.tag1[c] : v.tag0[c]) & T_ACT) != 0; },
      [&](int c) {
        double yb[4];
        for (int m = 0; m < 4; ++m) yb[m] = gbar[m * N + c];
        reverse_unit<R, 4>(v, yb, [&](Acc<R>& A, Dual* out) { geometry(A, c, arr, out); }, overflow);
      });
}

// TVD-RK3 stage (3, 2 or 1): output adjoint obar; cells outside the band
// of step n pass phi through (stage 3 only; atomic, since band cells whose
// stencils reach such a cell add into the same entry)
template <class R>
__global__ __launch_bounds__(256) void k_rk_adj(View<R> v, int stage, const double* obar, int* overflow) {
  for_units(
      v.N,
      [&](int c) {
        const bool act = (v.tag0[c] & T_ACT) != 0;
        if (!act && stage == 3) atomicAdd(&v.bar[AR_PHI0][c], obar[c]);
        return act;
      },
      [&](int c) {
        double yb[1] = {obar[c]};
        reverse_unit<R, 1>(v, yb, [&](Acc<R>& A, Dual* out) { rk_stage(A, c, stage, out); }, overflow);
      });
}

// reinitialisation stage (3, 2 or 1) of one pseudo step: output adjoint
// obar on the LS-active cells (the only ones the forward stage updates)
template <class R>
__global__ __launch_bounds__(256) void k_reinit_adj(View<R> v, int stage, int last, const double* obar, int* overflow) {
  for_units(
      v.N, [&](int c) { return (v.tag0[c] & T_ACT) != 0; },
      [&](int c) {
        double yb[1] = {obar[c]};
        reverse_unit<R, 1>(v, yb, [&](Acc<R>& A, Dual* out) { reinit_stage(A, c, stage, last != 0, out); },
                           overflow);
      });
}

// adjoint of the level set before the reinitialisation on the LS-active
// cells: the first pseudo step's input plus the smoothed-sign / fix
// reference (the same values); elsewhere the level set passed through
__global__ __launch_bounds__(256) void k_reinit_finish(const uint8_t* tag0, const double* rphibar, const double* p0bar,
                                                       double* phibar, int N) {
  for (int c = blockIdx.x * 256 + threadIdx.x; c < N; c += gridDim.x * 256)
    if (tag0[c] & T_ACT) phibar[c] = rphibar[c] + p0bar[c];
}

// extension sweep: adjoint of the sweep's output (AR_UTOUT) into the
// previous sweep's velocity (AR_UT), phi_n and G_n; seeded cells hold
// their velocity.  The output's adjoint is consumed: every cell's is read
// once (by its own lane, or by the wavefront running its unit) and then
// cleared, so the buffer is zero for its next use as an accumulator (the
// sweep reads no AR_UTOUT value through its inputs).
template <class R>
__global__ __launch_bounds__(256) void k_sweep_adj(View<R> v, int* overflow) {
  const long N = v.N;
  for_units(
      N,
      [&](int c) {
        const uint8_t t = v.tag0[c];
        const bool unit = (t & T_ACT) && !(t & T_SPEC);
        if ((t & T_ACT) && (t & T_SPEC))
          for (int m = 0; m < 3; ++m) atomicAdd(&v.bar[AR_UT][m * N + c], v.bar[AR_UTOUT][m * N + c]);
        if (!unit)
          for (int m = 0; m < 3; ++m) v.bar[AR_UTOUT][m * N + c] = 0.0;
        return unit;
      },
      [&](int c) {
        double yb[3];
        for (int m = 0; m < 3; ++m) yb[m] = v.bar[AR_UTOUT][m * N + c];
        reverse_unit<R, 3>(v, yb, [&](Acc<R>& A, Dual* out) { ext_sweep(A, c, out); }, overflow);
        if ((threadIdx.x & 63u) == 0u)
          for (int m = 0; m < 3; ++m) v.bar[AR_UTOUT][m * N + c] = 0.0;
      });
}

// extension seed: adjoint of the seeded velocity (AR_UTOUT) into the
// collide-stream moments and phi_n; away from the interface the seed is the
// cell's own velocity moment
// (the output's adjoint is consumed and cleared as in k_sweep_adj)
template <class R>
__global__ __launch_bounds__(256) void k_seed_adj(View<R> v, int* overflow) {
  const long N = v.N;
  for_units(
      N,
      [&](int c) {
        const uint8_t t = v.tag0[c];
        const bool unit = (t & T_ACT) && (t & T_SPEC);
        if ((t & T_ACT) && !(t & T_SPEC))
          for (int m = 0; m < 3; ++m) atomicAdd(&v.bar[AR_MNEW][(1 + m) * N + c], v.bar[AR_UTOUT][m * N + c]);
        if (!unit)
          for (int m = 0; m < 3; ++m) v.bar[AR_UTOUT][m * N + c] = 0.0;
        return unit;
      },
      [&](int c) {
        double yb[3];
        for (int m = 0; m < 3; ++m) yb[m] = v.bar[AR_UTOUT][m * N + c];
        reverse_unit<R, 3>(v, yb, [&](Acc<R>& A, Dual* out) { seed_iface(A, c, out); }, overflow);
        if ((threadIdx.x & 63u) == 0u)
          for (int m = 0; m < 3; ++m) v.bar[AR_UTOUT][m * N + c] = 0.0;
      });
}

// Collide-stream: adjoint of the populations of step n + 1 and (on LS-active
// cells) of the moments into the inputs of step n.  Cells that are not
// interface-adjacent (one thread per cell): each incoming population is a
// single input plus a constant, so the adjoint is the collision's transposed
// Jacobian, column by column.
template <class R>
__global__ __launch_bounds__(256) void k_collide_adj_plain(View<R> v) {
  const long N = v.N;
  ADJ_FOR_CELLS(v) {
    const uint8_t t = v.tag0[c];
    if (t & T_SPEC) continue;
    double yb[19];
    for (int i = 0; i < Q9; ++i) yb[i] = v.bar[AR_ANEW][i * N + c];
    const bool active = (t & T_ACT) != 0;
    for (int m = 0; m < 10; ++m) yb[9 + m] = active ? v.bar[AR_MNEW][m * N + c] : 0.0;
    bool any = false;
    for (int j = 0; j < 19; ++j) any = any || yb[j] != 0.0;
    if (!any) continue;
    const int x = c % v.nx, y = c / v.nx, k = t & T_GAS;
    long src[Q9];
    double f0[Q9];
    for (int i = 0; i < Q9; ++i) {
      const Src sr = plain_source(v, c, x, y, i);
      src[i] = sr.idx;
      const double d = (double)v.val[AR_AIN][sr.idx];
      f0[i] = sr.cst != 0.0 ? d + sr.cst : d;
    }
    for (int e = 0; e < Q9; ++e) {
      Dual f[Q9], out[19];
      for (int i = 0; i < Q9; ++i) f[i] = Dual(f0[i], i == e ? 1.0 : 0.0);
      collision(v, k, f, out);
      double g = 0.0;
      for (int j = 0; j < 19; ++j) g += yb[j] * out[j].d;
      if (g != 0.0) atomicAdd(&v.bar[AR_AIN][src[e]], g);
    }
  }
}

// Interface-adjacent cells (one cell per wavefront): lane i < 9 takes the
// collision's derivative with respect to incoming population i, then each
// pull is reversed as a unit of its own with that adjoint.
template <class R>
__global__ __launch_bounds__(256) void k_collide_adj(View<R> v, int* overflow) {
  const long N = v.N;
  for_units(
      N, [&](int c) { return (v.tag0[c] & T_SPEC) != 0; },
      [&](int c) {
        const uint8_t t = v.tag0[c];
        const bool active = (t & T_ACT) != 0;
        const int x = c % v.nx, y = c / v.nx, k = t & T_GAS;
        double yb[19];
        for (int i = 0; i < Q9; ++i) yb[i] = v.bar[AR_ANEW][i * N + c];
        for (int m = 0; m < 10; ++m) yb[9 + m] = active ? v.bar[AR_MNEW][m * N + c] : 0.0;
        bool any = false;
        for (int j = 0; j < 19; ++j) any = any || yb[j] != 0.0;
        if (!any) return;
        const int lane = (int)(threadIdx.x & 63u);
        double fb = 0.0;
        if (lane < Q9) {
          Acc<R> A;  // values only: no seed
          A.v = &v;
          A.mode = 1;
          A.tarr = -1;
          A.tidx = -1;
          Dual f[Q9], out[19];
          for (int i = 0; i < Q9; ++i) f[i] = Dual(pull(A, c, x, y, i, k, true).v, i == lane ? 1.0 : 0.0);
          collision(v, k, f, out);
          for (int j = 0; j < 19; ++j) fb += yb[j] * out[j].d;
        }
        for (int i = 0; i < Q9; ++i) {
          const double fbi = __shfl(fb, i);
          reverse_unit<R, 1>(v, &fbi, [&](Acc<R>& A, Dual* out) { out[0] = pull(A, c, x, y, i, k, true); }, overflow);
        }
      });
}

// initial populations and moments (hydrostatic density about the initial
// centroid xc0): adjoint into xc0 (block partial sums, fixed order)
template <class R>
__global__ __launch_bounds__(256) void k_init_pop_adj(View<R> v, const double* u0, double* partial) {
  const long N = v.N;
  double acc[2] = {0.0, 0.0};
  ADJ_FOR_CELLS(v) {
    const int k = v.tag0[c] & T_GAS;
    double u[2] = {0.0, 0.0};
    if (u0) { u[0] = u0[3 * (size_t)c]; u[1] = u0[3 * (size_t)c + 1]; }
    const double uu = u[0] * u[0] + u[1] * u[1];
    // d(populations, rho - 1)/d rho
    double g = 0.0;
    for (int i = 0; i < Q9; ++i) {
      const double w = wgt<LSB_D2Q9>(i);
      const double cu = L9::cx(i) * u[0] + L9::cy(i) * u[1];
      g += v.bar[AR_AIN][i * N + c] * w * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
    g += v.bar[AR_MIN][c];
    // d rho / d xc0_a = -acc_k,a / cs^2
    for (int a = 0; a < 2; ++a) acc[a] += g * (-3.0 * v.acc[k][a]);
  }
  __shared__ double red[2][256];
  red[0][threadIdx.x] = acc[0];
  red[1][threadIdx.x] = acc[1];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = red[0][0];
    partial[2 * blockIdx.x + 1] = red[1][0];
  }
}

// weights of the gas-pressure baseline's centroid dependence:
// Pb = pb0 + rho_l sum_a g_a (xc_a - xc0_a); w_a = Pbbar rho_l g_a, and the
// adjoint of xc0 receives -w_a; the consumed Pbbar is cleared
__global__ void k_pb_weights(double* pbbar, double rho_l, double g0, double g1, double* w, double* xc0bar) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double b = pbbar[0];
  w[0] = b * rho_l * g0;
  w[1] = b * rho_l * g1;
  xc0bar[0] -= w[0];
  xc0bar[1] -= w[1];
  pbbar[0] = 0.0;
}

// centroid (x, y) and Heaviside volume of a level set, one block, fixed
// summation order
template <class R>
__global__ __launch_bounds__(256) void k_centroid1(const R* phi, int nx, int N, double eps, double* xc, double* V) {
  double s[3] = {0.0, 0.0, 0.0};
  for (int c = threadIdx.x; c < N; c += 256) {
    const double p = (double)phi[c];
    double h;
    if (p < -eps) h = 0.0;
    else if (p > eps) h = 1.0;
    else h = 0.5 * (1.0 + p / eps + sin(3.14159265358979323846 * p / eps) / 3.14159265358979323846);
    s[0] += h;
    s[1] += h * (c % nx + 0.5);
    s[2] += h * (c / nx + 0.5);
  }
  __shared__ double red[3][256];
  for (int m = 0; m < 3; ++m) red[m][threadIdx.x] = s[m];
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k)
      for (int m = 0; m < 3; ++m) red[m][threadIdx.x] += red[m][threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    V[0] = red[0][0];
    xc[0] = red[1][0] / red[0][0];
    xc[1] = red[2][0] / red[0][0];
  }
}

__global__ void k_set_sigma(double* dst, double sigma) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = sigma;
}

__global__ void k_set_unit(double* w, int axis) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    w[0] = axis == 0 ? 1.0 : 0.0;
    w[1] = axis == 1 ? 1.0 : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_zero(double* p, long n) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) p[i] = 0.0;
}

// several device-to-device copies in one launch: 16-byte words where both
// ends are 16-byte aligned, then the remaining bytes
struct CopySet {
  static constexpr int kMax = 8;
  const char* src[kMax];
  char* dst[kMax];
  long bytes[kMax];
  int count;
};
__global__ __launch_bounds__(256) void k_copy_set(const CopySet z) {
  const long t0 = blockIdx.x * 256L + threadIdx.x, step = (long)gridDim.x * 256;
  for (int j = 0; j < z.count; ++j) {
    const char* const s = z.src[j];
    char* const d = z.dst[j];
    const long n = z.bytes[j];
    const bool aligned = ((reinterpret_cast<uintptr_t>(s) | reinterpret_cast<uintptr_t>(d)) & 15u) == 0u;
    const long n16 = aligned ? n / 16 : 0;
    for (long i = t0; i < n16; i += step)
      reinterpret_cast<uint4*>(d)[i] = reinterpret_cast<const uint4*>(s)[i];
    for (long i = n16 * 16 + t0; i < n; i += step) d[i] = s[i];
  }
}

// several arrays cleared by one launch
struct ZeroSet {
  static constexpr int kMax = 8;
  double* p[kMax];
  long n[kMax];
  int count;
};
__global__ __launch_bounds__(256) void k_zero_set(const ZeroSet z) {
  for (int j = 0; j < z.count; ++j) {
    double* const p = z.p[j];
    const long n = z.n[j];
    for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) p[i] = 0.0;
  }
}

// sum of the block partials of k_init_pop_adj into the xc0 adjoint
__global__ void k_sum_partials(const double* partial, int nblocks, double* xc0bar) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s0 = 0.0, s1 = 0.0;
  for (int b = 0; b < nblocks; ++b) { s0 += partial[2 * b]; s1 += partial[2 * b + 1]; }
  xc0bar[0] += s0;
  xc0bar[1] += s1;
}

// gradient with respect to the unclamped initial level set
__global__ __launch_bounds__(256) void k_phi0_grad(const double* phibar, const double* phi0, double band, int N,
                                                   double* out) {
  for (int c = blockIdx.x * 256 + threadIdx.x; c < N; c += gridDim.x * 256) {
    const double p = phi0[c];
    out[c] = (p >= -(band - kBandSnap) && p <= band - kBandSnap) ? phibar[c] : 0.0;
  }
}

}  // namespace adj
}  // namespace lsb
