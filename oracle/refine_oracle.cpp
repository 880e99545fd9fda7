// CPU oracle: two-level static grid refinement of the lattice Boltzmann
// solver (D2Q9, D3Q19, D3Q27; BGK, FP64), ratio 2.  Test infrastructure only: the tests,
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
//   nodes      coarse (I, J, K), periodic on every axis; the fine patch
//              covers the coarse nodes [ia, ib] x [ja, jb] (x [ka, kb]) at
//              half spacing, fine node (i, j, k) at (ia + i/2, ja + j/2,
//              ka + k/2); coarse nodes strictly inside the box are covered,
//              those on its boundary are perimeter nodes.
//   coarse     every uncovered coarse node pulls, keeps its pre-collision
//   step       populations G(t+1) if it is a perimeter node, and collides
//              with tau_c.
//   fine       two sub-steps (t + 1/2, t + 1); a fine perimeter node takes
//   sub-steps  each population whose source lies outside the patch from G:
//              in time (G(t) + G(t+1))/2, then G(t+1); in space, along
//              each odd fine coordinate the mean of the two coarse nodes
//              beside it (2 or, at a face centre, 4 coarse nodes); the
//              non-equilibrium part about the equilibrium of the
//              interpolated moments scaled by the ratio of tau dt between
//              the levels, tau_f / (2 tau_c).  Collision with tau_f.
//   restrict   in the second sub-step, a fine node on a covered coarse node
//              gives that node its coarse post-collision populations: the
//              fine pre-collision non-equilibrium part scaled back by
//              2 tau_c / tau_f, then collided with tau_c, which is
//              f_eq + 2 (tau_c - 1) / tau_f (f - f_eq).
#include <cmath>
#include <vector>

// the oracle's velocity sets in the paper's ordering (lsb_oracle.cpp)
extern "C" int orc_lattice(int lattice, int* D, int* Q, int* c, double* w, int* opp);

namespace ref {

constexpr int QMAX = 27;

struct Ref {
  int D = 2, Q = 9;
  int cx[QMAX], cy[QMAX], cz[QMAX];
  double w[QMAX];
  int nx, ny, nz, ia, ib, ja, jb, ka, kb, mx, my, mz;
  double tc, tf;
  std::vector<double> fc, ff;  // post-collision populations [q][node], x fastest
  std::vector<double> g0, g1;  // coarse pre-collision populations over the patch box, times t and t+1

  long nc() const { return (long)nx * ny * nz; }
  long nf() const { return (long)(mx + 1) * (my + 1) * (mz + 1); }
  long nb() const { return (long)(ib - ia + 1) * (jb - ja + 1) * (kb - ka + 1); }
  long cidx(int I, int J, int K) const { return ((long)K * ny + J) * nx + I; }
  long fidx(int i, int j, int k) const { return ((long)k * (my + 1) + j) * (mx + 1) + i; }
  long box(int I, int J, int K) const { return ((long)(K - ka) * (jb - ja + 1) + (J - ja)) * (ib - ia + 1) + (I - ia); }
  bool in_box(int I, int J, int K) const {
    return I >= ia && I <= ib && J >= ja && J <= jb && (D == 2 || (K >= ka && K <= kb));
  }
  bool covered(int I, int J, int K) const {
    return I > ia && I < ib && J > ja && J < jb && (D == 2 || (K > ka && K < kb));
  }
  bool perimeter(int I, int J, int K) const { return in_box(I, J, K) && !covered(I, J, K); }

  // eq. (feq) with c_s^2 = 1/3
  void feq(double rho, double ux, double uy, double uz, double* out) const {
    const double uu = ux * ux + uy * uy + uz * uz;
    for (int q = 0; q < Q; ++q) {
      const double cu = cx[q] * ux + cy[q] * uy + cz[q] * uz;
      out[q] = w[q] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
  }
  void moments(const double* f, double& rho, double& ux, double& uy, double& uz) const {
    rho = 0.0;
    double mxs = 0.0, mys = 0.0, mzs = 0.0;
    for (int q = 0; q < Q; ++q) {
      rho += f[q];
      mxs += cx[q] * f[q];
      mys += cy[q] * f[q];
      mzs += cz[q] * f[q];
    }
    ux = mxs / rho;
    uy = mys / rho;
    uz = mzs / rho;
  }

  // u holds D components per node
  void init(const double* rc, const double* uc, const double* rf, const double* uf) {
    fc.assign(Q * nc(), 0.0);
    ff.assign(Q * nf(), 0.0);
    g0.assign(Q * nb(), 0.0);
    g1.assign(Q * nb(), 0.0);
    double e[QMAX];
    for (int K = 0; K < nz; ++K)
      for (int J = 0; J < ny; ++J)
        for (int I = 0; I < nx; ++I) {
          const long n = cidx(I, J, K);
          feq(rc[n], uc[D * n], uc[D * n + 1], D == 3 ? uc[D * n + 2] : 0.0, e);
          for (int q = 0; q < Q; ++q) fc[q * nc() + n] = e[q];
          if (perimeter(I, J, K))
            for (int q = 0; q < Q; ++q) g0[q * nb() + box(I, J, K)] = e[q];
        }
    for (long n = 0; n < nf(); ++n) {
      feq(rf[n], uf[D * n], uf[D * n + 1], D == 3 ? uf[D * n + 2] : 0.0, e);
      for (int q = 0; q < Q; ++q) ff[q * nf() + n] = e[q];
    }
  }

  // interpolated coarse pre-collision set at fine perimeter node (i, j, k):
  // time weights a (t) and b (t + 1); along each odd coordinate the mean of
  // the two coarse nodes beside it (z outermost, x innermost)
  void coarse_set(int i, int j, int k, double a, double b, double* H) const {
    for (int q = 0; q < Q; ++q) H[q] = 0.0;
    const int ox = i & 1, oy = j & 1, oz = k & 1;
    const double s = (ox ? 0.5 : 1.0) * (oy ? 0.5 : 1.0) * (oz ? 0.5 : 1.0);
    for (int dz = 0; dz <= oz; ++dz)
      for (int dy = 0; dy <= oy; ++dy)
        for (int dx = 0; dx <= ox; ++dx) {
          const int I = ia + (i - ox) / 2 + dx, J = ja + (j - oy) / 2 + dy, K = ka + (k - oz) / 2 + dz;
          const long bx = box(I, J, K);
          for (int q = 0; q < Q; ++q) H[q] += s * (a * g0[q * nb() + bx] + b * g1[q * nb() + bx]);
        }
  }

  bool outside(int si, int sj, int sk) const { return si < 0 || si > mx || sj < 0 || sj > my || sk < 0 || sk > mz; }

  void step() {
    // coarse step t -> t+1 on the uncovered nodes
    std::vector<double> nfc = fc;
    double f[QMAX], e[QMAX];
    for (int K = 0; K < nz; ++K)
      for (int J = 0; J < ny; ++J)
        for (int I = 0; I < nx; ++I) {
          if (covered(I, J, K)) continue;
          const long n = cidx(I, J, K);
          for (int q = 0; q < Q; ++q) {
            const int sI = ((I - cx[q]) % nx + nx) % nx, sJ = ((J - cy[q]) % ny + ny) % ny;
            const int sK = ((K - cz[q]) % nz + nz) % nz;
            f[q] = fc[q * nc() + cidx(sI, sJ, sK)];
          }
          if (perimeter(I, J, K))
            for (int q = 0; q < Q; ++q) g1[q * nb() + box(I, J, K)] = f[q];
          double rho, ux, uy, uz;
          moments(f, rho, ux, uy, uz);
          feq(rho, ux, uy, uz, e);
          for (int q = 0; q < Q; ++q) nfc[q * nc() + n] = f[q] - (f[q] - e[q]) / tc;
        }
    // two fine sub-steps
    for (int s = 1; s <= 2; ++s) {
      const double a = s == 1 ? 0.5 : 0.0, b = s == 1 ? 0.5 : 1.0;
      std::vector<double> nff(ff.size());
      for (int k = 0; k <= mz; ++k)
        for (int j = 0; j <= my; ++j)
          for (int i = 0; i <= mx; ++i) {
            const long n = fidx(i, j, k);
            bool missing = false;
            for (int q = 0; q < Q; ++q) {
              const int si = i - cx[q], sj = j - cy[q], sk = k - cz[q];
              if (outside(si, sj, sk)) {
                missing = true;
                continue;
              }
              f[q] = ff[q * nf() + fidx(si, sj, sk)];
            }
            if (missing) {
              double H[QMAX], eh[QMAX], rh, uxh, uyh, uzh;
              coarse_set(i, j, k, a, b, H);
              moments(H, rh, uxh, uyh, uzh);
              feq(rh, uxh, uyh, uzh, eh);
              for (int q = 0; q < Q; ++q)
                if (outside(i - cx[q], j - cy[q], k - cz[q])) f[q] = eh[q] + tf / (2.0 * tc) * (H[q] - eh[q]);
            }
            double rho, ux, uy, uz;
            moments(f, rho, ux, uy, uz);
            feq(rho, ux, uy, uz, e);
            for (int q = 0; q < Q; ++q) nff[q * nf() + n] = f[q] - (f[q] - e[q]) / tf;
            if (s == 2 && i % 2 == 0 && j % 2 == 0 && k % 2 == 0 &&
                covered(ia + i / 2, ja + j / 2, ka + k / 2)) {
              const long m = cidx(ia + i / 2, ja + j / 2, ka + k / 2);
              for (int q = 0; q < Q; ++q) nfc[q * nc() + m] = e[q] + 2.0 * (tc - 1.0) / tf * (f[q] - e[q]);
            }
          }
      ff.swap(nff);
    }
    fc.swap(nfc);
    g0.swap(g1);
  }

  // Level-set refinement sensor (Sec. 3, adaptive mesh refinement): a coarse
  // node is tagged for refinement where it lies in the gas or within d_ref
  // of it.  This build's level set is negative in the liquid and >= 0 in the
  // gas, the opposite of the sign the sensor is written with, so the test is
  // phi >= -d_ref.  The patch is the tagged nodes' bounding box grown by
  // margin nodes, clamped to keep one node to spare at each grid face and
  // widened to at least two cells per axis; out = (ia, ib, ja, jb, ka, kb).
  // Returns false (out untouched) when no node is tagged.
  bool sensor_box(const double* phi, double d_ref, int margin, int* out) const {
    int lo[3] = {nx, ny, nz}, hi[3] = {-1, -1, -1};
    for (int K = 0; K < nz; ++K)
      for (int J = 0; J < ny; ++J)
        for (int I = 0; I < nx; ++I) {
          if (!(phi[cidx(I, J, K)] >= -d_ref)) continue;
          const int p[3] = {I, J, K};
          for (int d = 0; d < 3; ++d) {
            if (p[d] < lo[d]) lo[d] = p[d];
            if (p[d] > hi[d]) hi[d] = p[d];
          }
        }
    if (hi[0] < 0) return false;
    const int n[3] = {nx, ny, nz};
    for (int d = 0; d < D; ++d) {
      int a = lo[d] - margin, b = hi[d] + margin;
      if (a < 1) a = 1;
      if (b > n[d] - 2) b = n[d] - 2;
      while (b - a < 2) {
        if (b < n[d] - 2) ++b;
        else --a;
      }
      out[2 * d] = a;
      out[2 * d + 1] = b;
    }
    if (D == 2) out[4] = out[5] = 0;
    return true;
  }

  // Re-meshing onto a new patch box at the end of a coarse step (state at
  // time t: post-collision populations of both levels, the covered coarse
  // nodes holding restricted values).  New fine nodes inside the old patch
  // keep the old fine populations; the others take the coarse populations
  // interpolated like the perimeter's (the mean of the 2, 4 or 8 coarse
  // nodes around an off-grid fine node), their non-equilibrium part scaled
  // by the post-collision ratio (tau_f - 1) / (2 (tau_c - 1)) about the
  // equilibrium of the interpolated moments (the equilibrium alone when
  // tau_c = 1, where the coarse post-collision state holds no
  // non-equilibrium part).  The new perimeter's pre-collision sets G(t) come
  // from the coarse post-collision populations by inverting the BGK step,
  // f_eq + tau_c / (tau_c - 1) (f - f_eq) (f_eq at tau_c = 1).  Covered
  // coarse nodes are restricted again at the end of the next step; coarse
  // nodes the patch no longer covers keep their restricted values.
  void remesh(const int* np) {
    const int oia = ia, oib = ib, oja = ja, ojb = jb, oka = ka, okb = kb, omx = mx, omy = my, omz = mz;
    const std::vector<double> off = ff;
    const long onf = nf();
    ia = np[0];
    ib = np[1];
    ja = np[2];
    jb = np[3];
    ka = D == 3 ? np[4] : 0;
    kb = D == 3 ? np[5] : 0;
    mx = 2 * (ib - ia);
    my = 2 * (jb - ja);
    mz = 2 * (kb - ka);
    ff.assign(Q * nf(), 0.0);
    g0.assign(Q * nb(), 0.0);
    g1.assign(Q * nb(), 0.0);
    double H[QMAX], e[QMAX];
    const bool flat = tc == 1.0;
    const double up = flat ? 0.0 : (tf - 1.0) / (2.0 * (tc - 1.0));
    for (int k = 0; k <= mz; ++k)
      for (int j = 0; j <= my; ++j)
        for (int i = 0; i <= mx; ++i) {
          // coarse-unit position times two
          const int X2 = 2 * ia + i, Y2 = 2 * ja + j, Z2 = 2 * ka + k;
          const int oi = X2 - 2 * oia, oj = Y2 - 2 * oja, ok = Z2 - 2 * oka;
          const long n = fidx(i, j, k);
          if (oi >= 0 && oi <= omx && oj >= 0 && oj <= omy && ok >= 0 && ok <= omz) {
            const long on = ((long)ok * (omy + 1) + oj) * (omx + 1) + oi;
            for (int q = 0; q < Q; ++q) ff[q * nf() + n] = off[q * onf + on];
            continue;
          }
          const int ox = X2 & 1, oy = Y2 & 1, oz = Z2 & 1;
          const double s = (ox ? 0.5 : 1.0) * (oy ? 0.5 : 1.0) * (oz ? 0.5 : 1.0);
          for (int q = 0; q < Q; ++q) H[q] = 0.0;
          for (int dz = 0; dz <= oz; ++dz)
            for (int dy = 0; dy <= oy; ++dy)
              for (int dx = 0; dx <= ox; ++dx) {
                const long m = cidx((X2 - ox) / 2 + dx, (Y2 - oy) / 2 + dy, (Z2 - oz) / 2 + dz);
                for (int q = 0; q < Q; ++q) H[q] += s * fc[q * nc() + m];
              }
          double rho, ux, uy, uz;
          moments(H, rho, ux, uy, uz);
          feq(rho, ux, uy, uz, e);
          for (int q = 0; q < Q; ++q) ff[q * nf() + n] = e[q] + up * (H[q] - e[q]);
        }
    const double down = flat ? 0.0 : tc / (tc - 1.0);
    for (int K = ka; K <= (D == 3 ? kb : 0); ++K)
      for (int J = ja; J <= jb; ++J)
        for (int I = ia; I <= ib; ++I) {
          if (!perimeter(I, J, K)) continue;
          const long m = cidx(I, J, K);
          double f[QMAX];
          for (int q = 0; q < Q; ++q) f[q] = fc[q * nc() + m];
          double rho, ux, uy, uz;
          moments(f, rho, ux, uy, uz);
          feq(rho, ux, uy, uz, e);
          for (int q = 0; q < Q; ++q) g0[q * nb() + box(I, J, K)] = e[q] + down * (f[q] - e[q]);
        }
    (void)oib;
    (void)ojb;
    (void)okb;
  }
};

}  // namespace ref

extern "C" {

// lattice: 0 D2Q9, 1 D3Q19, 2 D3Q27 (the oracle's numbering); n = (nx, ny,
// nz) with nz = 1 in 2D; patch = (ia, ib, ja, jb, ka, kb), ka = kb = 0 in 2D.
// tau_f <= 0 selects the constant-viscosity value 2 tau_c - 1/2; the tests
// pass another value only to check that a pin catches a wrong one.
void* orc_ref_create(int lattice, const int* n, const int* patch, double tau_c, double tau_f) {
  if (!n || !patch) return nullptr;
  ref::Ref* r = new ref::Ref();
  int c[3 * ref::QMAX], opp[ref::QMAX];
  if (orc_lattice(lattice, &r->D, &r->Q, c, r->w, opp) != 0) {
    delete r;
    return nullptr;
  }
  for (int q = 0; q < r->Q; ++q) {
    r->cx[q] = c[3 * q];
    r->cy[q] = c[3 * q + 1];
    r->cz[q] = c[3 * q + 2];
  }
  r->nx = n[0];
  r->ny = n[1];
  r->nz = r->D == 3 ? n[2] : 1;
  r->ia = patch[0];
  r->ib = patch[1];
  r->ja = patch[2];
  r->jb = patch[3];
  r->ka = r->D == 3 ? patch[4] : 0;
  r->kb = r->D == 3 ? patch[5] : 0;
  const bool ok = r->nx >= 4 && r->ny >= 4 && (r->D == 2 || r->nz >= 4) && r->ia >= 1 && r->ib <= r->nx - 2 &&
                  r->ib - r->ia >= 2 && r->ja >= 1 && r->jb <= r->ny - 2 && r->jb - r->ja >= 2 &&
                  (r->D == 2 || (r->ka >= 1 && r->kb <= r->nz - 2 && r->kb - r->ka >= 2)) && tau_c > 0.5;
  if (!ok) {
    delete r;
    return nullptr;
  }
  r->mx = 2 * (r->ib - r->ia);
  r->my = 2 * (r->jb - r->ja);
  r->mz = 2 * (r->kb - r->ka);
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

// sensor box from a coarse level set (out: ia, ib, ja, jb, ka, kb); returns 1
// when a node is tagged, 0 otherwise
int orc_ref_sensor(void* h, const double* phi, double d_ref, int margin, int* out) {
  return static_cast<ref::Ref*>(h)->sensor_box(phi, d_ref, margin, out) ? 1 : 0;
}

// re-mesh onto the patch (ia, ib, ja, jb, ka, kb); -1 if it does not fit the grid
int orc_ref_remesh(void* h, const int* patch) {
  ref::Ref* r = static_cast<ref::Ref*>(h);
  const int n[3] = {r->nx, r->ny, r->nz};
  for (int d = 0; d < r->D; ++d)
    if (patch[2 * d] < 1 || patch[2 * d + 1] > n[d] - 2 || patch[2 * d + 1] - patch[2 * d] < 2) return -1;
  r->remesh(patch);
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
