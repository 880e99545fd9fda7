// CPU oracle: two-level static grid refinement of the lattice Boltzmann
// solver (D2Q9, BGK, FP64), ratio 2.  Test infrastructure only: the tests,
// the smoke check and the benchmark's CPU-baseline leg call it; the product
// path never does.
//
// The paper couples its grid levels after Dupuis and Chopard: populations
// missing at a refinement jump are interpolated in space and time from the
// known neighbouring populations of the other level, and the collision
// frequency of eq. (omega) is taken with each level's time step so that the
// viscosity is the same on both (Sec. 2, lattice Boltzmann method).  With
// dt = dx on each level and a ratio of 2 that gives tau_f = 2 tau_c - 1/2 in
// each level's lattice units.  The paper gives no further detail; the steps
// below are the reading this build takes (node layout, interpolation order,
// rescaling of the non-equilibrium part, order of the sub-steps):
//
//   nodes      coarse (I, J), periodic on both axes; the fine patch covers
//              the coarse nodes [ia, ib] x [ja, jb] at half spacing, fine
//              node (i, j) at (ia + i/2, ja + j/2), i in [0, 2(ib-ia)],
//              j in [0, 2(jb-ja)]; coarse nodes strictly inside the box are
//              covered, those on its boundary are perimeter nodes.
//   coarse     every uncovered coarse node pulls, keeps its pre-collision
//   step       populations G(t+1) if it is a perimeter node, and collides
//              with tau_c.
//   fine       two sub-steps (t + 1/2, t + 1); a fine perimeter node takes
//   sub-steps  each population whose source lies outside the patch from G:
//              in time (G(t) + G(t+1))/2, then G(t+1); along an edge the
//              mean of the two coarse perimeter nodes beside an odd fine
//              node; the non-equilibrium part about the equilibrium of the
//              interpolated moments scaled by the ratio of tau dt between
//              the levels, tau_f / (2 tau_c).  Collision with tau_f.
//   restrict   in the second sub-step, a fine node on a covered coarse node
//              gives that node its coarse post-collision populations: the
//              fine pre-collision non-equilibrium part scaled back by
//              2 tau_c / tau_f, then collided with tau_c, which is
//              f_eq + 2 (tau_c - 1) / tau_f (f - f_eq).
#include <cmath>
#include <vector>

namespace ref {

constexpr int Q = 9;
// D2Q9 in the paper's ordering, rest direction last
constexpr int CX[Q] = {-1, 1, 0, 0, -1, -1, 1, 1, 0};
constexpr int CY[Q] = {0, 0, -1, 1, -1, 1, 1, -1, 0};
constexpr double W[Q] = {1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 4.0 / 9};

// eq. (feq) with c_s^2 = 1/3
void feq(double rho, double ux, double uy, double* out) {
  const double uu = ux * ux + uy * uy;
  for (int q = 0; q < Q; ++q) {
    const double cu = CX[q] * ux + CY[q] * uy;
    out[q] = W[q] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

void moments(const double* f, double& rho, double& ux, double& uy) {
  rho = 0.0;
  double mx = 0.0, my = 0.0;
  for (int q = 0; q < Q; ++q) {
    rho += f[q];
    mx += CX[q] * f[q];
    my += CY[q] * f[q];
  }
  ux = mx / rho;
  uy = my / rho;
}

struct Ref {
  int nx, ny, ia, ib, ja, jb, mx, my;
  double tc, tf;
  std::vector<double> fc, ff;  // post-collision populations [q][node]
  std::vector<double> g0, g1;  // coarse pre-collision populations over the patch box, times t and t+1

  long nc() const { return (long)nx * ny; }
  long nf() const { return (long)(mx + 1) * (my + 1); }
  long nb() const { return (long)(ib - ia + 1) * (jb - ja + 1); }
  long box(int I, int J) const { return (long)(J - ja) * (ib - ia + 1) + (I - ia); }
  bool covered(int I, int J) const { return I > ia && I < ib && J > ja && J < jb; }
  bool perimeter(int I, int J) const {
    return I >= ia && I <= ib && J >= ja && J <= jb && (I == ia || I == ib || J == ja || J == jb);
  }

  void init(const double* rc, const double* uc, const double* rf, const double* uf) {
    fc.assign(Q * nc(), 0.0);
    ff.assign(Q * nf(), 0.0);
    g0.assign(Q * nb(), 0.0);
    g1.assign(Q * nb(), 0.0);
    double e[Q];
    for (int J = 0; J < ny; ++J)
      for (int I = 0; I < nx; ++I) {
        const long n = (long)J * nx + I;
        feq(rc[n], uc[2 * n], uc[2 * n + 1], e);
        for (int q = 0; q < Q; ++q) fc[q * nc() + n] = e[q];
        if (perimeter(I, J))
          for (int q = 0; q < Q; ++q) g0[q * nb() + box(I, J)] = e[q];
      }
    for (long n = 0; n < nf(); ++n) {
      feq(rf[n], uf[2 * n], uf[2 * n + 1], e);
      for (int q = 0; q < Q; ++q) ff[q * nf() + n] = e[q];
    }
  }

  // interpolated coarse pre-collision set at fine perimeter node (i, j):
  // weights a (time t) and b (time t + 1)
  void coarse_set(int i, int j, double a, double b, double* H) const {
    auto node = [&](int I, int J, double s) {
      for (int q = 0; q < Q; ++q) H[q] += s * (a * g0[q * nb() + box(I, J)] + b * g1[q * nb() + box(I, J)]);
    };
    for (int q = 0; q < Q; ++q) H[q] = 0.0;
    if (i % 2 == 0 && j % 2 == 0) {
      node(ia + i / 2, ja + j / 2, 1.0);
    } else if (i % 2 != 0) {  // on a horizontal edge
      node(ia + (i - 1) / 2, ja + j / 2, 0.5);
      node(ia + (i + 1) / 2, ja + j / 2, 0.5);
    } else {  // on a vertical edge
      node(ia + i / 2, ja + (j - 1) / 2, 0.5);
      node(ia + i / 2, ja + (j + 1) / 2, 0.5);
    }
  }

  void step() {
    // coarse step t -> t+1 on the uncovered nodes
    std::vector<double> nfc = fc;
    double f[Q], e[Q];
    for (int J = 0; J < ny; ++J)
      for (int I = 0; I < nx; ++I) {
        if (covered(I, J)) continue;
        const long n = (long)J * nx + I;
        for (int q = 0; q < Q; ++q) {
          const int sI = ((I - CX[q]) % nx + nx) % nx, sJ = ((J - CY[q]) % ny + ny) % ny;
          f[q] = fc[q * nc() + (long)sJ * nx + sI];
        }
        if (perimeter(I, J))
          for (int q = 0; q < Q; ++q) g1[q * nb() + box(I, J)] = f[q];
        double rho, ux, uy;
        moments(f, rho, ux, uy);
        feq(rho, ux, uy, e);
        for (int q = 0; q < Q; ++q) nfc[q * nc() + n] = f[q] - (f[q] - e[q]) / tc;
      }
    // two fine sub-steps
    for (int s = 1; s <= 2; ++s) {
      const double a = s == 1 ? 0.5 : 0.0, b = s == 1 ? 0.5 : 1.0;
      std::vector<double> nff(ff.size());
      for (int j = 0; j <= my; ++j)
        for (int i = 0; i <= mx; ++i) {
          const long n = (long)j * (mx + 1) + i;
          bool missing = false;
          for (int q = 0; q < Q; ++q) {
            const int si = i - CX[q], sj = j - CY[q];
            if (si < 0 || si > mx || sj < 0 || sj > my) {
              missing = true;
              continue;
            }
            f[q] = ff[q * nf() + (long)sj * (mx + 1) + si];
          }
          if (missing) {
            double H[Q], eh[Q], rh, uxh, uyh;
            coarse_set(i, j, a, b, H);
            moments(H, rh, uxh, uyh);
            feq(rh, uxh, uyh, eh);
            for (int q = 0; q < Q; ++q) {
              const int si = i - CX[q], sj = j - CY[q];
              if (si < 0 || si > mx || sj < 0 || sj > my) f[q] = eh[q] + tf / (2.0 * tc) * (H[q] - eh[q]);
            }
          }
          double rho, ux, uy;
          moments(f, rho, ux, uy);
          feq(rho, ux, uy, e);
          for (int q = 0; q < Q; ++q) nff[q * nf() + n] = f[q] - (f[q] - e[q]) / tf;
          if (s == 2 && i % 2 == 0 && j % 2 == 0 && covered(ia + i / 2, ja + j / 2)) {
            const long m = (long)(ja + j / 2) * nx + ia + i / 2;
            for (int q = 0; q < Q; ++q) nfc[q * nc() + m] = e[q] + 2.0 * (tc - 1.0) / tf * (f[q] - e[q]);
          }
        }
      ff.swap(nff);
    }
    fc.swap(nfc);
    g0.swap(g1);
  }
};

}  // namespace ref

extern "C" {

// tau_f <= 0 selects the constant-viscosity value 2 tau_c - 1/2; the tests
// pass another value only to check that a pin catches a wrong one.
void* orc_ref_create(int nx, int ny, const int* patch, double tau_c, double tau_f) {
  if (nx < 4 || ny < 4 || !patch) return nullptr;
  const int ia = patch[0], ib = patch[1], ja = patch[2], jb = patch[3];
  if (ia < 1 || ib > nx - 2 || ib - ia < 2 || ja < 1 || jb > ny - 2 || jb - ja < 2 || !(tau_c > 0.5)) return nullptr;
  ref::Ref* r = new ref::Ref();
  r->nx = nx;
  r->ny = ny;
  r->ia = ia;
  r->ib = ib;
  r->ja = ja;
  r->jb = jb;
  r->mx = 2 * (ib - ia);
  r->my = 2 * (jb - ja);
  r->tc = tau_c;
  r->tf = tau_f > 0.0 ? tau_f : 2.0 * tau_c - 0.5;
  return r;
}

void orc_ref_destroy(void* h) { delete static_cast<ref::Ref*>(h); }

int orc_ref_init(void* h, const double* rho_c, const double* u_c, const double* rho_f, const double* u_f) {
  static_cast<ref::Ref*>(h)->init(rho_c, u_c, rho_f, u_f);
  return 0;
}

int orc_ref_step(void* h, int n) {
  ref::Ref* r = static_cast<ref::Ref*>(h);
  for (int s = 0; s < n; ++s) r->step();
  return 0;
}

// populations [Q][nodes] of both levels (post-collision; the covered coarse
// nodes hold the restricted values)
int orc_ref_get(void* h, double* fc, double* ff) {
  const ref::Ref* r = static_cast<const ref::Ref*>(h);
  for (size_t k = 0; k < r->fc.size(); ++k) fc[k] = r->fc[k];
  for (size_t k = 0; k < r->ff.size(); ++k) ff[k] = r->ff[k];
  return 0;
}
}
