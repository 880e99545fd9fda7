// CPU oracle: static grid refinement of the lattice Boltzmann solver (D2Q9,
// D3Q19, D3Q27; BGK, FP64), ratio 2, nested levels or a tree of boxes, with
// the level-set sensor and re-meshing.  Test infrastructure only: the tests,
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
// below are the reading taken here (node layout, interpolation order,
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
//   nesting    a grid may hold finer boxes of its own (one, or several at
//              least one of its nodes apart: a tree), each a box of its
//              nodes with one node to spare at each side; every pair of
//              adjacent grids is coupled as above (tau doubles minus 1/2
//              from level to level), and a grid's sub-step is followed by
//              each of its boxes' two sub-steps, the second of which
//              restricts into the grid's new populations.  A level restricts into
//              its parent from its own pre-collision populations, which at
//              nodes covered by its child come from the child's restriction
//              (the levels hand their data down one jump at a time).
#include <algorithm>
#include <cmath>
#include <vector>

// the oracle's velocity sets in the paper's ordering (lsb_oracle.cpp)
extern "C" int orc_lattice(int lattice, int* D, int* Q, int* c, double* w, int* opp);

namespace ref {

constexpr int QMAX = 27;
constexpr int LMAX = 4;   // levels of a chain
constexpr int BMAX = 16;  // grids of a tree: the coarse grid and up to 15 boxes

// one grid level: nodes (i, j, k), i in [0, mx], and for a refined level its
// box [ia, ib] x [ja, jb] (x [ka, kb]) in the parent's node coordinates, node
// (i, j, k) sitting at the parent's (ia + i/2, ja + j/2, ka + k/2)
struct Level {
  int D = 2;
  int mx = 0, my = 0, mz = 0;
  int ia = 0, ib = 0, ja = 0, jb = 0, ka = 0, kb = 0;
  double tau = 1.0;
  int parent = -1;             // index of the parent grid (-1: the coarse grid itself)
  std::vector<int> kids;       // boxes refining this grid (disjoint, one node apart at least)
  std::vector<double> f;       // post-collision populations [q][node], x fastest
  std::vector<double> g0, g1;  // the parent's pre-collision sets over the box, times t and t + 1

  long n() const { return (long)(mx + 1) * (my + 1) * (mz + 1); }
  long idx(int i, int j, int k) const { return ((long)k * (my + 1) + j) * (mx + 1) + i; }
  long nb() const { return (long)(ib - ia + 1) * (jb - ja + 1) * (kb - ka + 1); }
  long box(int I, int J, int K) const { return ((long)(K - ka) * (jb - ja + 1) + (J - ja)) * (ib - ia + 1) + (I - ia); }
  // parent-node tests
  bool in_box(int I, int J, int K) const {
    return I >= ia && I <= ib && J >= ja && J <= jb && (D == 2 || (K >= ka && K <= kb));
  }
  bool covered(int I, int J, int K) const {
    return I > ia && I < ib && J > ja && J < jb && (D == 2 || (K > ka && K < kb));
  }
  bool perimeter(int I, int J, int K) const { return in_box(I, J, K) && !covered(I, J, K); }
  bool outside(int si, int sj, int sk) const { return si < 0 || si > mx || sj < 0 || sj > my || sk < 0 || sk > mz; }
  void set_box(const int* p) {
    ia = p[0];
    ib = p[1];
    ja = p[2];
    jb = p[3];
    ka = D == 3 ? p[4] : 0;
    kb = D == 3 ? p[5] : 0;
    mx = 2 * (ib - ia);
    my = 2 * (jb - ja);
    mz = 2 * (kb - ka);
  }
};

struct Ref {
  int D = 2, Q = 9;
  int cx[QMAX], cy[QMAX], cz[QMAX];
  double w[QMAX];
  int L = 2;        // grids: the coarse grid and the boxes
  Level lv[BMAX];   // lv[0]: the periodic coarse grid; a box's parent has a smaller index

  // every box refines the one before it (a chain of nested levels)
  bool chain() const {
    for (int l = 1; l < L; ++l)
      if (lv[l].parent != l - 1) return false;
    return true;
  }

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

  // equilibrium state from rho[l] and u[l] (D components per node) on every
  // level; each refined level's G(t) is its parent's initial populations on
  // the box perimeter
  void init(const double* const* rho, const double* const* u) {
    double e[QMAX];
    for (int l = 0; l < L; ++l) {
      Level& v = lv[l];
      v.f.assign(Q * v.n(), 0.0);
      for (long n = 0; n < v.n(); ++n) {
        feq(rho[l][n], u[l][D * n], u[l][D * n + 1], D == 3 ? u[l][D * n + 2] : 0.0, e);
        for (int q = 0; q < Q; ++q) v.f[q * v.n() + n] = e[q];
      }
    }
    for (int l = 1; l < L; ++l) {
      Level& c = lv[l];
      const Level& p = lv[c.parent];
      c.g0.assign(Q * c.nb(), 0.0);
      c.g1.assign(Q * c.nb(), 0.0);
      for (int K = c.ka; K <= c.kb; ++K)
        for (int J = c.ja; J <= c.jb; ++J)
          for (int I = c.ia; I <= c.ib; ++I)
            if (c.perimeter(I, J, K))
              for (int q = 0; q < Q; ++q) c.g0[q * c.nb() + c.box(I, J, K)] = p.f[q * p.n() + p.idx(I, J, K)];
    }
  }

  // interpolated parent pre-collision set at perimeter node (i, j, k) of
  // level c: time weights a (t) and b (t + 1); along each odd coordinate the
  // mean of the two parent nodes beside it (z outermost, x innermost)
  void coarse_set(const Level& c, int i, int j, int k, double a, double b, double* H) const {
    for (int q = 0; q < Q; ++q) H[q] = 0.0;
    const int ox = i & 1, oy = j & 1, oz = k & 1;
    const double s = (ox ? 0.5 : 1.0) * (oy ? 0.5 : 1.0) * (oz ? 0.5 : 1.0);
    for (int dz = 0; dz <= oz; ++dz)
      for (int dy = 0; dy <= oy; ++dy)
        for (int dx = 0; dx <= ox; ++dx) {
          const long bx = c.box(c.ia + (i - ox) / 2 + dx, c.ja + (j - oy) / 2 + dy, c.ka + (k - oz) / 2 + dz);
          for (int q = 0; q < Q; ++q) H[q] += s * (a * c.g0[q * c.nb() + bx] + b * c.g1[q * c.nb() + bx]);
        }
  }

  // One time step of grid l, returning its new post-collision populations.
  // The coarse grid pulls periodically and skips the nodes its boxes cover;
  // a box takes the populations whose source lies outside it from the
  // parent's G (time weights a, b), and with restrict_ writes the parent's
  // covered nodes into parent_new.  Nodes on a child box's perimeter store
  // their pre-collision sets as that child's G(t + 1).
  std::vector<double> step_level(int l, double a, double b, bool restrict_, std::vector<double>* parent_new) {
    Level& v = lv[l];
    const Level* p = l > 0 ? &lv[v.parent] : nullptr;
    std::vector<double> out = v.f;
    double f[QMAX], e[QMAX];
    for (int k = 0; k <= v.mz; ++k)
      for (int j = 0; j <= v.my; ++j)
        for (int i = 0; i <= v.mx; ++i) {
          bool skip = false;
          for (int kd : v.kids) skip = skip || (l == 0 && lv[kd].covered(i, j, k));
          if (skip) continue;
          bool missing = false;
          for (int q = 0; q < Q; ++q) {
            int si = i - cx[q], sj = j - cy[q], sk = k - cz[q];
            if (l == 0) {
              si = (si + v.mx + 1) % (v.mx + 1);
              sj = (sj + v.my + 1) % (v.my + 1);
              sk = (sk + v.mz + 1) % (v.mz + 1);
            } else if (v.outside(si, sj, sk)) {
              missing = true;
              continue;
            }
            f[q] = v.f[q * v.n() + v.idx(si, sj, sk)];
          }
          if (missing) {
            double H[QMAX], eh[QMAX], rh, uxh, uyh, uzh;
            coarse_set(v, i, j, k, a, b, H);
            moments(H, rh, uxh, uyh, uzh);
            feq(rh, uxh, uyh, uzh, eh);
            for (int q = 0; q < Q; ++q)
              if (v.outside(i - cx[q], j - cy[q], k - cz[q])) f[q] = eh[q] + v.tau / (2.0 * p->tau) * (H[q] - eh[q]);
          }
          for (int kd : v.kids) {
            Level& c = lv[kd];
            if (c.perimeter(i, j, k))
              for (int q = 0; q < Q; ++q) c.g1[q * c.nb() + c.box(i, j, k)] = f[q];
          }
          double rho, ux, uy, uz;
          moments(f, rho, ux, uy, uz);
          feq(rho, ux, uy, uz, e);
          const long n = v.idx(i, j, k);
          for (int q = 0; q < Q; ++q) out[q * v.n() + n] = f[q] - (f[q] - e[q]) / v.tau;
          if (restrict_ && i % 2 == 0 && j % 2 == 0 && k % 2 == 0 && v.covered(v.ia + i / 2, v.ja + j / 2, v.ka + k / 2)) {
            const long m = p->idx(v.ia + i / 2, v.ja + j / 2, v.ka + k / 2);
            for (int q = 0; q < Q; ++q)
              (*parent_new)[q * p->n() + m] = e[q] + 2.0 * (p->tau - 1.0) / v.tau * (f[q] - e[q]);
          }
        }
    return out;
  }

  // the two sub-steps of box l within one step of its parent, each
  // followed by its child boxes' two sub-steps (one child after the other)
  void advance(int l, std::vector<double>& parent_new) {
    for (int s = 1; s <= 2; ++s) {
      std::vector<double> nf = step_level(l, s == 1 ? 0.5 : 0.0, s == 1 ? 0.5 : 1.0, s == 2, &parent_new);
      for (int kd : lv[l].kids) {
        advance(kd, nf);
        lv[kd].g0.swap(lv[kd].g1);
      }
      lv[l].f.swap(nf);
    }
  }

  void step() {
    std::vector<double> nf = step_level(0, 0.0, 0.0, false, nullptr);
    for (int kd : lv[0].kids) {
      advance(kd, nf);
      lv[kd].g0.swap(lv[kd].g1);
    }
    lv[0].f.swap(nf);
  }

  // Level-set refinement sensor (Sec. 3, adaptive mesh refinement): a coarse
  // node is tagged for refinement where it lies in the gas or within d_ref
  // of it.  The level set here is negative in the liquid and >= 0 in the
  // gas, the opposite of the sign the sensor is written with, so the test is
  // phi >= -d_ref.  The patch is the tagged nodes' bounding box grown by
  // margin nodes, clamped to keep one node to spare at each grid face and
  // widened to at least two cells per axis; out = (ia, ib, ja, jb, ka, kb).
  // Returns false (out untouched) when no node is tagged.
  bool sensor_box(const double* phi, double d_ref, int margin, int* out) const {
    const Level& g = lv[0];
    const int n[3] = {g.mx + 1, g.my + 1, g.mz + 1};
    int lo[3] = {n[0], n[1], n[2]}, hi[3] = {-1, -1, -1};
    for (int K = 0; K < n[2]; ++K)
      for (int J = 0; J < n[1]; ++J)
        for (int I = 0; I < n[0]; ++I) {
          if (!(phi[g.idx(I, J, K)] >= -d_ref)) continue;
          const int pt[3] = {I, J, K};
          for (int d = 0; d < 3; ++d) {
            if (pt[d] < lo[d]) lo[d] = pt[d];
            if (pt[d] > hi[d]) hi[d] = pt[d];
          }
        }
    if (hi[0] < 0) return false;
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

  // Sensor for a tree of root boxes: every tagged coarse node (phi >=
  // -d_ref, as sensor_box) belongs to its nearest seed (seeds are coarse
  // nodes; squared distances compared exactly, ties to the lower index);
  // each seed with tagged nodes gives their bounding box grown by margin,
  // clamped one node inside the grid and widened to two cells per axis;
  // boxes closer than one node apart are merged into their union box until
  // every pair is apart (a merged box takes the earlier one's place).
  // out: 6 ints per box; returns the number of boxes.
  int sensor_seeded(const double* phi, double d_ref, int margin, int ns, const int* seeds, int* out) const {
    const Level& g = lv[0];
    const int n[3] = {g.mx + 1, g.my + 1, g.mz + 1};
    std::vector<int> lo(3 * ns), hi(3 * ns, -1);
    for (int k = 0; k < ns; ++k)
      for (int d = 0; d < 3; ++d) lo[3 * k + d] = n[d];
    for (int K = 0; K < n[2]; ++K)
      for (int J = 0; J < n[1]; ++J)
        for (int I = 0; I < n[0]; ++I) {
          if (!(phi[g.idx(I, J, K)] >= -d_ref)) continue;
          int best = 0;
          long bd = -1;
          for (int k = 0; k < ns; ++k) {
            const long dx = I - seeds[3 * k], dy = J - seeds[3 * k + 1], dz = K - seeds[3 * k + 2];
            const long dd = dx * dx + dy * dy + dz * dz;
            if (bd < 0 || dd < bd) {
              bd = dd;
              best = k;
            }
          }
          const int pt[3] = {I, J, K};
          for (int d = 0; d < 3; ++d) {
            if (pt[d] < lo[3 * best + d]) lo[3 * best + d] = pt[d];
            if (pt[d] > hi[3 * best + d]) hi[3 * best + d] = pt[d];
          }
        }
    std::vector<std::vector<int>> boxes;
    for (int k = 0; k < ns; ++k) {
      if (hi[3 * k] < 0) continue;
      std::vector<int> b(6, 0);
      for (int d = 0; d < D; ++d) {
        int a = lo[3 * k + d] - margin, c = hi[3 * k + d] + margin;
        if (a < 1) a = 1;
        if (c > n[d] - 2) c = n[d] - 2;
        while (c - a < 2) {
          if (c < n[d] - 2) ++c;
          else --a;
        }
        b[2 * d] = a;
        b[2 * d + 1] = c;
      }
      boxes.push_back(b);
    }
    for (bool merged = true; merged;) {
      merged = false;
      for (size_t a = 0; a < boxes.size() && !merged; ++a)
        for (size_t b = a + 1; b < boxes.size() && !merged; ++b) {
          bool apart = false;
          for (int d = 0; d < D; ++d)
            apart = apart || boxes[a][2 * d + 1] + 2 <= boxes[b][2 * d] || boxes[b][2 * d + 1] + 2 <= boxes[a][2 * d];
          if (apart) continue;
          for (int d = 0; d < D; ++d) {
            boxes[a][2 * d] = std::min(boxes[a][2 * d], boxes[b][2 * d]);
            boxes[a][2 * d + 1] = std::max(boxes[a][2 * d + 1], boxes[b][2 * d + 1]);
          }
          boxes.erase(boxes.begin() + (long)b);
          merged = true;
        }
    }
    for (size_t k = 0; k < boxes.size(); ++k)
      for (int d = 0; d < 6; ++d) out[6 * k + d] = boxes[k][d];
    return (int)boxes.size();
  }

  // origin of each level's nodes in that level's spacing, counted from
  // coarse node 0: o[0] = 0, o[l] = 2 (o[l-1] + box corner of level l)
  void origins(long o[BMAX][3]) const {
    for (int d = 0; d < 3; ++d) o[0][d] = 0;
    for (int l = 1; l < L; ++l) {
      const int p = lv[l].parent;
      o[l][0] = 2 * (o[p][0] + lv[l].ia);
      o[l][1] = 2 * (o[p][1] + lv[l].ja);
      o[l][2] = 2 * (o[p][2] + lv[l].ka);
    }
  }

  // Level-set sensor for every refined level: the tagged coarse nodes'
  // bounding box (as sensor_box) grown by margins[l - 1] coarse nodes for
  // level l, written in the parent's node coordinates (a coarse position X
  // is parent node 2^(l-1) X - o[l-1]) and clamped to keep one parent node
  // to spare at each side, at least two cells per axis; out holds 6 ints per
  // level.  Levels are taken in order, each inside the one just computed.
  bool sensor_boxes(const double* phi, double d_ref, const int* margins, int* out) const {
    int box[6];
    if (!sensor_box(phi, d_ref, margins[0], box)) return false;
    for (int d = 0; d < 6; ++d) out[d] = box[d];
    // the tagged box itself (margin 0, unclamped)
    const Level& g = lv[0];
    const int n[3] = {g.mx + 1, g.my + 1, g.mz + 1};
    int lo[3] = {n[0], n[1], n[2]}, hi[3] = {-1, -1, -1};
    for (int K = 0; K < n[2]; ++K)
      for (int J = 0; J < n[1]; ++J)
        for (int I = 0; I < n[0]; ++I) {
          if (!(phi[g.idx(I, J, K)] >= -d_ref)) continue;
          const int pt[3] = {I, J, K};
          for (int d = 0; d < 3; ++d) {
            if (pt[d] < lo[d]) lo[d] = pt[d];
            if (pt[d] > hi[d]) hi[d] = pt[d];
          }
        }
    long org[3] = {0, 0, 0};  // origin of the parent level (level 0 first)
    int pm[3] = {0, 0, 0};    // parent's last node index per axis
    long scale = 1;           // 2^(l-1)
    for (int l = 2; l < L; ++l) {
      const int* pb = out + 6 * (l - 2);  // the parent's box, in its own parent's coordinates
      for (int d = 0; d < D; ++d) {
        org[d] = 2 * (org[d] + pb[2 * d]);
        pm[d] = 2 * (pb[2 * d + 1] - pb[2 * d]);
      }
      scale *= 2;
      int* ob = out + 6 * (l - 1);
      for (int d = 0; d < D; ++d) {
        long a = scale * (lo[d] - margins[l - 1]) - org[d], b = scale * (hi[d] + margins[l - 1]) - org[d];
        if (a < 1) a = 1;
        if (b > pm[d] - 1) b = pm[d] - 1;
        while (b - a < 2) {
          if (b < pm[d] - 1) ++b;
          else --a;
        }
        ob[2 * d] = (int)a;
        ob[2 * d + 1] = (int)b;
      }
      if (D == 2) ob[4] = ob[5] = 0;
    }
    return true;
  }

  // Re-meshing onto new boxes at the end of a coarse step (state at time t:
  // post-collision populations of every level, covered nodes holding
  // restricted values), box 1 first, each box inside its re-meshed parent
  // (a chain of levels or a tree, whose shape stays); boxes holds 6 ints per
  // box in the parent's node coordinates.  A new node of level l at a position the old level l
  // covered keeps the old populations; the others take the parent's
  // populations interpolated like the perimeter's (the mean of the 2, 4 or 8
  // parent nodes around an off-grid node), their non-equilibrium part scaled
  // by the post-collision ratio (tau_l - 1) / (2 (tau_{l-1} - 1)) about the
  // equilibrium of the interpolated moments (the equilibrium alone when
  // tau_{l-1} = 1, where the parent's post-collision state holds no
  // non-equilibrium part).  Each level's new perimeter sets G(t) come from
  // the parent's post-collision populations by inverting the BGK step,
  // f_eq + tau / (tau - 1) (f - f_eq) with the parent's tau (f_eq at
  // tau = 1).  Covered nodes are restricted again at the end of the next
  // step; nodes a level no longer covers keep their restricted values.
  void remesh_levels(const int* boxes) {
    long oo[BMAX][3], on[BMAX][3];
    origins(oo);
    const std::vector<Level> old(lv, lv + L);
    for (int d = 0; d < 3; ++d) on[0][d] = 0;
    for (int l = 1; l < L; ++l) {
      Level& v = lv[l];
      const Level& p = lv[v.parent];
      const Level& o = old[l];
      v.set_box(boxes + 6 * (l - 1));
      on[l][0] = 2 * (on[v.parent][0] + v.ia);
      on[l][1] = 2 * (on[v.parent][1] + v.ja);
      on[l][2] = 2 * (on[v.parent][2] + v.ka);
      v.f.assign(Q * v.n(), 0.0);
      v.g0.assign(Q * v.nb(), 0.0);
      v.g1.assign(Q * v.nb(), 0.0);
      double H[QMAX], e[QMAX];
      const double tc = p.tau, tf = v.tau;
      const bool flat = tc == 1.0;
      const double up = flat ? 0.0 : (tf - 1.0) / (2.0 * (tc - 1.0));
      for (int k = 0; k <= v.mz; ++k)
        for (int j = 0; j <= v.my; ++j)
          for (int i = 0; i <= v.mx; ++i) {
            const long n = v.idx(i, j, k);
            const long oi = on[l][0] + i - oo[l][0], oj = on[l][1] + j - oo[l][1], ok = on[l][2] + k - oo[l][2];
            if (!o.outside((int)oi, (int)oj, (int)ok)) {
              for (int q = 0; q < Q; ++q) v.f[q * v.n() + n] = o.f[q * o.n() + o.idx((int)oi, (int)oj, (int)ok)];
              continue;
            }
            // position in the parent's node units, times two
            const int X2 = 2 * v.ia + i, Y2 = 2 * v.ja + j, Z2 = 2 * v.ka + k;
            const int ox = X2 & 1, oy = Y2 & 1, oz = Z2 & 1;
            const double s = (ox ? 0.5 : 1.0) * (oy ? 0.5 : 1.0) * (oz ? 0.5 : 1.0);
            for (int q = 0; q < Q; ++q) H[q] = 0.0;
            for (int dz = 0; dz <= oz; ++dz)
              for (int dy = 0; dy <= oy; ++dy)
                for (int dx = 0; dx <= ox; ++dx) {
                  const long m = p.idx((X2 - ox) / 2 + dx, (Y2 - oy) / 2 + dy, (Z2 - oz) / 2 + dz);
                  for (int q = 0; q < Q; ++q) H[q] += s * p.f[q * p.n() + m];
                }
            double rho, ux, uy, uz;
            moments(H, rho, ux, uy, uz);
            feq(rho, ux, uy, uz, e);
            for (int q = 0; q < Q; ++q) v.f[q * v.n() + n] = e[q] + up * (H[q] - e[q]);
          }
      const double down = flat ? 0.0 : tc / (tc - 1.0);
      for (int K = v.ka; K <= v.kb; ++K)
        for (int J = v.ja; J <= v.jb; ++J)
          for (int I = v.ia; I <= v.ib; ++I) {
            if (!v.perimeter(I, J, K)) continue;
            const long m = p.idx(I, J, K);
            double f[QMAX];
            for (int q = 0; q < Q; ++q) f[q] = p.f[q * p.n() + m];
            double rho, ux, uy, uz;
            moments(f, rho, ux, uy, uz);
            feq(rho, ux, uy, uz, e);
            for (int q = 0; q < Q; ++q) v.g0[q * v.nb() + v.box(I, J, K)] = e[q] + down * (f[q] - e[q]);
          }
    }
  }
};

}  // namespace ref

extern "C" {

// A tree of boxes: box b (1 .. nbox) refines grid parents[b - 1] (0: the
// coarse grid, else an earlier box) over boxes[6 (b - 1) ...] = (ia, ib, ja,
// jb, ka, kb) of the parent's nodes (ka = kb = 0 in 2D), with one node to
// spare at every side of the parent, at least two cells per axis, and
// siblings at least one parent node apart.  tau[b] <= 0 (or tau == NULL)
// selects the constant-viscosity value 2 tau[parent] - 1/2.
void* orc_tree_create(int lattice, const int* n, int nbox, const int* parents, const int* boxes, double tau_c,
                      const double* tau) {
  if (!n || (nbox > 0 && (!parents || !boxes)) || nbox < 1 || nbox + 1 > ref::BMAX || !(tau_c > 0.5)) return nullptr;
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
  r->L = nbox + 1;
  for (int l = 0; l < r->L; ++l) r->lv[l].D = r->D;
  ref::Level& g = r->lv[0];
  g.mx = n[0] - 1;
  g.my = n[1] - 1;
  g.mz = r->D == 3 ? n[2] - 1 : 0;
  g.tau = tau_c;
  bool ok = g.mx >= 3 && g.my >= 3 && (r->D == 2 || g.mz >= 3);
  for (int l = 1; l < r->L && ok; ++l) {
    ref::Level& v = r->lv[l];
    v.parent = parents[l - 1];
    ok = v.parent >= 0 && v.parent < l;
    if (!ok) break;
    const ref::Level& p = r->lv[v.parent];
    v.set_box(boxes + 6 * (l - 1));
    v.tau = tau && tau[l] > 0.0 ? tau[l] : 2.0 * p.tau - 0.5;
    ok = v.ia >= 1 && v.ib <= p.mx - 1 && v.ib - v.ia >= 2 && v.ja >= 1 && v.jb <= p.my - 1 && v.jb - v.ja >= 2 &&
         (r->D == 2 || (v.ka >= 1 && v.kb <= p.mz - 1 && v.kb - v.ka >= 2));
    // siblings at least one parent node apart on some axis
    for (int o : r->lv[v.parent].kids) {
      const ref::Level& w = r->lv[o];
      const bool apart = v.ib + 2 <= w.ia || w.ib + 2 <= v.ia || v.jb + 2 <= w.ja || w.jb + 2 <= v.ja ||
                         (r->D == 3 && (v.kb + 2 <= w.ka || w.kb + 2 <= v.ka));
      ok = ok && apart;
    }
    r->lv[v.parent].kids.push_back(l);
  }
  if (!ok) {
    delete r;
    return nullptr;
  }
  return r;
}

// lattice: 0 D2Q9, 1 D3Q19, 2 D3Q27 (the oracle's numbering); n = (nx, ny,
// nz) with nz = 1 in 2D; levels in [2, 4]; patches[6 (l - 1) ...] = (ia, ib,
// ja, jb, ka, kb) of level l in level l - 1's node coordinates (ka = kb = 0
// in 2D), each with one node to spare at every side of its parent (level 0:
// 1 <= ia, ib <= nx - 2) and at least two cells per axis.  tau[l] <= 0 (or
// tau == NULL) selects the constant-viscosity value 2 tau[l-1] - 1/2; the
// tests pass another value only to check that a pin catches a wrong one.
void* orc_mref_create(int lattice, const int* n, int levels, const int* patches, double tau_c, const double* tau) {
  if (levels < 2 || levels > ref::LMAX) return nullptr;
  int parents[ref::LMAX];
  for (int l = 1; l < levels; ++l) parents[l - 1] = l - 1;
  return orc_tree_create(lattice, n, levels - 1, parents, patches, tau_c, tau);
}

// two levels: patch of level 1, tau_f <= 0 for 2 tau_c - 1/2
void* orc_ref_create(int lattice, const int* n, const int* patch, double tau_c, double tau_f) {
  const double tau[2] = {tau_c, tau_f};
  return orc_mref_create(lattice, n, 2, patch, tau_c, tau);
}

void orc_ref_destroy(void* h) { delete static_cast<ref::Ref*>(h); }

// rho[l] [nodes of level l], u[l] [nodes][D] for every level
int orc_mref_init(void* h, const double* const* rho, const double* const* u) {
  static_cast<ref::Ref*>(h)->init(rho, u);
  return 0;
}

int orc_ref_init(void* h, const double* rho_c, const double* u_c, const double* rho_f, const double* u_f) {
  const double* rho[2] = {rho_c, rho_f};
  const double* u[2] = {u_c, u_f};
  if (static_cast<ref::Ref*>(h)->L != 2) return -1;
  return orc_mref_init(h, rho, u);
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

// re-mesh a two-level hierarchy onto the patch (ia, ib, ja, jb, ka, kb); -1
// if it does not fit the grid or the hierarchy has more levels
int orc_ref_remesh(void* h, const int* patch) {
  ref::Ref* r = static_cast<ref::Ref*>(h);
  if (r->L != 2 || !r->chain() || r->lv[0].f.empty()) return -1;
  const ref::Level& g = r->lv[0];
  const int n[3] = {g.mx + 1, g.my + 1, g.mz + 1};
  for (int d = 0; d < r->D; ++d)
    if (patch[2 * d] < 1 || patch[2 * d + 1] > n[d] - 2 || patch[2 * d + 1] - patch[2 * d] < 2) return -1;
  r->remesh_levels(patch);
  return 0;
}

// seeded sensor (boxes for a tree of root boxes): seeds are ns coarse nodes
// (3 ints each); out receives 6 ints per box; returns the number of boxes
int orc_ref_sensor_seeded(void* h, const double* phi, double d_ref, int margin, int ns, const int* seeds, int* out) {
  return static_cast<ref::Ref*>(h)->sensor_seeded(phi, d_ref, margin, ns, seeds, out);
}

// nested sensor: margins[l - 1] (coarse nodes) for level l; out receives 6
// ints per refined level; returns 1 when a node is tagged, 0 otherwise
int orc_ref_sensor_levels(void* h, const double* phi, double d_ref, const int* margins, int* out) {
  if (!static_cast<ref::Ref*>(h)->chain()) return -1;
  return static_cast<ref::Ref*>(h)->sensor_boxes(phi, d_ref, margins, out) ? 1 : 0;
}

// nested re-mesh onto boxes (nboxes boxes of 6 ints, one per refined grid,
// each in its new parent's node coordinates); -1 if the count differs from
// the refined grids or a box does not fit its parent
int orc_ref_remesh_levels(void* h, const int* boxes, int nboxes) {
  ref::Ref* r = static_cast<ref::Ref*>(h);
  if (nboxes != r->L - 1) return -1;
  if (r->lv[0].f.empty()) return -1;  // not initialised
  int last[ref::BMAX][3];  // each grid's last node index per axis, after the re-mesh
  last[0][0] = r->lv[0].mx;
  last[0][1] = r->lv[0].my;
  last[0][2] = r->lv[0].mz;
  for (int l = 1; l < r->L; ++l) {
    const int* b = boxes + 6 * (l - 1);
    const int p = r->lv[l].parent;
    for (int d = 0; d < r->D; ++d)
      if (b[2 * d] < 1 || b[2 * d + 1] > last[p][d] - 1 || b[2 * d + 1] - b[2 * d] < 2) return -1;
    for (int o = 1; o < l; ++o) {  // siblings stay one parent node apart
      if (r->lv[o].parent != p) continue;
      const int* w = boxes + 6 * (o - 1);
      bool apart = false;
      for (int d = 0; d < r->D; ++d) apart = apart || b[2 * d + 1] + 2 <= w[2 * d] || w[2 * d + 1] + 2 <= b[2 * d];
      if (!apart) return -1;
    }
    for (int d = 0; d < 3; ++d) last[l][d] = d < r->D ? 2 * (b[2 * d + 1] - b[2 * d]) : 0;
  }
  r->remesh_levels(boxes);
  return 0;
}

// post-collision populations [Q][nodes] of one level (the covered nodes hold
// the restricted values)
int orc_mref_get(void* h, int level, double* out) {
  const ref::Ref* r = static_cast<const ref::Ref*>(h);
  if (level < 0 || level >= r->L) return -1;
  const std::vector<double>& f = r->lv[level].f;
  for (size_t k = 0; k < f.size(); ++k) out[k] = f[k];
  return 0;
}

int orc_ref_get(void* h, double* fc, double* ff) {
  orc_mref_get(h, 0, fc);
  return orc_mref_get(h, 1, ff);
}
}
