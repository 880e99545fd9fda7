// refine2.hip -- the two-phase step on a two-level grid (lsb_refine2.h).
//
// The paper keeps the interface on the finest level, with the same level on
// both of its sides (Sec. 3.2), and couples its refinement levels after
// Dupuis and Chopard with the relaxation time rescaled per level
// (Sec. 2.1).  Here a periodic coarse grid runs each phase's plain BGK step
// (no interface can reach it) and one refined box runs the whole two-phase
// step of lsb.h in its own lattice units, as an lsb_plan whose faces read
// the coarse grid's populations (kFaceInject faces, ghost array [Q][N]).
//
// Per coarse step, on the caller's stream:
//   k_r2_coarse    pull + BGK with force on the uncovered coarse nodes; the
//                  box perimeter keeps its pre-collision sets G(t+1);
//   k_r2_inject    the ghost populations of the fine surface nodes from G,
//                  for the first and then the second fine sub-step;
//   fine step      the two-phase step of the fine plan (twice);
//   k_r2_restrict  every covered coarse node from the fine state (the ring
//                  next to the perimeter is what the coarse step reads);
//   k_r2_band      the fine level's LS-active cells keep 3 cells from the
//                  box faces (a sticky flag, read at the end of the call).
// Re-meshing (the box keeps its extents and follows the interface):
//   k_r2_sensor         bounding box of the fine cells with phi >= -d_ref;
//   k_r2_remesh_fine    the fine state moved, new nodes from the coarse level;
//   k_r2_perimeter_sets the new perimeter's pre-collision sets, inverted
//                       from the coarse state.
// The coarse populations are FP64 whatever the fine storage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "driver.h"
#include "../../include/lsb_refine2.h"

namespace {

using lsb::Lat;
using lsb::wgt;

int fail(int code, const std::string& msg) {
  lsb::set_error(msg);
  return code;
}

#define R2_HIP(x)                                                                                     \
  do {                                                                                                \
    hipError_t e_ = (x);                                                                              \
    if (e_ != hipSuccess) return fail(LSB_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));  \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Geometry: coarse nodes (I, J, K), box [b0, b1] x [b2, b3] (x [b4, b5]) of
// coarse nodes, fine node (i, j, k) at coarse coordinates (b0 + i/2, ...).
struct Geo {
  int D;
  int nx, ny, nz;   // coarse nodes per axis
  int b[6];         // box, inclusive; b4 = b5 = 0 in 2D
  int bw, bh;       // box nodes along x and y
  long nc, nb;      // coarse nodes, box nodes
  int fx, fy, fz;   // fine nodes per axis
  long nf;
  long ns;          // fine surface nodes
};

// Per phase k: coarse omega_k = 1 / tau_c,k, the relaxation times of both
// levels, the coarse and fine body accelerations (a_f = a_c / 2) and the
// reference density of the fine storage's codec.
struct Phys {
  double om[2], tc[2], tf[2];
  double acc[2][3], accf[2][3];
  double rref[2];
  double inv_scale;
};

__device__ __forceinline__ bool covered(const Geo& g, int I, int J, int K) {
  return I > g.b[0] && I < g.b[1] && J > g.b[2] && J < g.b[3] && (g.D == 2 || (K > g.b[4] && K < g.b[5]));
}
__device__ __forceinline__ bool in_box(const Geo& g, int I, int J, int K) {
  return I >= g.b[0] && I <= g.b[1] && J >= g.b[2] && J <= g.b[3] && (g.D == 2 || (K >= g.b[4] && K <= g.b[5]));
}
__device__ __forceinline__ bool inner_ring(const Geo& g, int I, int J, int K) {
  if (!covered(g, I, J, K)) return false;
  bool r = I == g.b[0] + 1 || I == g.b[1] - 1 || J == g.b[2] + 1 || J == g.b[3] - 1;
  if (g.D == 3) r = r || K == g.b[4] + 1 || K == g.b[5] - 1;
  return r;
}
__device__ __forceinline__ long bidx(const Geo& g, int I, int J, int K) {
  return ((long)(K - g.b[4]) * g.bh + (J - g.b[2])) * g.bw + (I - g.b[0]);
}

// second-order equilibrium (eq:feq) and the first-order body force
// w_i rho (c_i . a) / cs^2 of Sec. 2.1
template <int LAT>
__device__ __forceinline__ void moments(const double* f, double& rho, double u[3]) {
  using L = Lat<LAT>;
  double r = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    r += f[q];
    m0 += (double)L::cx(q) * f[q];
    m1 += (double)L::cy(q) * f[q];
    m2 += (double)L::cz(q) * f[q];
  }
  rho = r;
  u[0] = m0 / r;
  u[1] = m1 / r;
  u[2] = m2 / r;
}
template <int LAT>
__device__ __forceinline__ double feq(int q, double rho, const double u[3]) {
  using L = Lat<LAT>;
  const double cu = (double)L::cx(q) * u[0] + (double)L::cy(q) * u[1] + (double)L::cz(q) * u[2];
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  return wgt<LAT>(q) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}
template <int LAT>
__device__ __forceinline__ double force(int q, double rho, const double a[3]) {
  using L = Lat<LAT>;
  return 3.0 * wgt<LAT>(q) * rho * ((double)L::cx(q) * a[0] + (double)L::cy(q) * a[1] + (double)L::cz(q) * a[2]);
}

__device__ __forceinline__ void coarse_coords(const Geo& g, long c, int& I, int& J, int& K) {
  I = (int)(c % g.nx);
  J = (int)((c / g.nx) % g.ny);
  K = (int)(c / ((long)g.nx * g.ny));
}
// Surface node s of the fine level (0 <= s < ns): the two z faces (3D),
// then the two y faces less their z edges, then the two x faces less their
// y and z edges; each face row by row, x (or y) fastest.
__device__ __forceinline__ void surface_coords(const Geo& g, long s, int& i, int& j, int& k) {
  const int ez = g.D == 3 ? g.fz - 2 : 1;  // interior z extent (z = 1 .. fz - 2, or the one plane in 2D)
  const int z0 = g.D == 3 ? 1 : 0;
  const long nzf = g.D == 3 ? (long)g.fx * g.fy : 0;  // nodes of one z face
  if (s < 2 * nzf) {
    const long t = s < nzf ? s : s - nzf;
    k = s < nzf ? 0 : g.fz - 1;
    j = (int)(t / g.fx);
    i = (int)(t - (long)j * g.fx);
    return;
  }
  s -= 2 * nzf;
  const long nyf = (long)g.fx * ez;  // nodes of one y face
  if (s < 2 * nyf) {
    const long t = s < nyf ? s : s - nyf;
    j = s < nyf ? 0 : g.fy - 1;
    k = z0 + (int)(t / g.fx);
    i = (int)(t - (long)(k - z0) * g.fx);
    return;
  }
  s -= 2 * nyf;
  const long nxf = (long)(g.fy - 2) * ez;  // nodes of one x face
  const long t = s < nxf ? s : s - nxf;
  i = s < nxf ? 0 : g.fx - 1;
  k = z0 + (int)(t / (g.fy - 2));
  j = 1 + (int)(t - (long)(k - z0) * (g.fy - 2));
}

__device__ __forceinline__ void fine_coords(const Geo& g, long c, int& i, int& j, int& k) {
  i = (int)(c % g.fx);
  j = (int)((c / g.fx) % g.fy);
  k = (int)(c / ((long)g.fx * g.fy));
}

// Initial coarse state: equilibria of (rho, u) (u: 3 values per node), the
// phase from phi (gas where phi >= 0) and the perimeter's pre-collision sets
// one step before the start (the initial state less one step of force).
template <int LAT>
__global__ __launch_bounds__(256) void k_r2_init(Geo g, Phys ph, const double* __restrict__ phi,
                                                 const double* __restrict__ rho, const double* __restrict__ u,
                                                 double* __restrict__ f0, uint8_t* __restrict__ kc,
                                                 double* __restrict__ g0) {
  constexpr int Q = Lat<LAT>::Q;
  for (long c = blockIdx.x * 256L + threadIdx.x; c < g.nc; c += (long)gridDim.x * 256) {
    int I, J, K;
    coarse_coords(g, c, I, J, K);
    const int k = phi[c] >= 0.0 ? 1 : 0;
    kc[c] = (uint8_t)k;
    const double uc[3] = {u[3 * c], u[3 * c + 1], u[3 * c + 2]};
    double e[Q], r = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      e[q] = feq<LAT>(q, rho[c], uc);
      f0[(size_t)q * g.nc + c] = e[q];
      r += e[q];
    }
    if (in_box(g, I, J, K) && !covered(g, I, J, K)) {
      const long bi = bidx(g, I, J, K);
#pragma unroll
      for (int q = 0; q < Q; ++q) g0[(size_t)q * g.nb + bi] = e[q] - force<LAT>(q, r, ph.acc[k]);
    }
  }
}

// Coarse step on the uncovered nodes (periodic pull, BGK of the node's
// phase with its body force); perimeter nodes also keep their pre-collision
// populations in g1.
template <int LAT>
__global__ __launch_bounds__(256) void k_r2_coarse(Geo g, Phys ph, const double* __restrict__ fin,
                                                   double* __restrict__ fout, const uint8_t* __restrict__ kc,
                                                   double* __restrict__ g1) {
  using L = Lat<LAT>;
  constexpr int Q = L::Q;
  for (long c = blockIdx.x * 256L + threadIdx.x; c < g.nc; c += (long)gridDim.x * 256) {
    int I, J, K;
    coarse_coords(g, c, I, J, K);
    if (covered(g, I, J, K)) continue;
    double f[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      int si = I - L::cx(q), sj = J - L::cy(q), sk = K - L::cz(q);
      si = si < 0 ? si + g.nx : (si >= g.nx ? si - g.nx : si);
      sj = sj < 0 ? sj + g.ny : (sj >= g.ny ? sj - g.ny : sj);
      sk = sk < 0 ? sk + g.nz : (sk >= g.nz ? sk - g.nz : sk);
      f[q] = fin[(size_t)q * g.nc + ((long)sk * g.ny + sj) * g.nx + si];
    }
    if (in_box(g, I, J, K)) {
      const long bi = bidx(g, I, J, K);
#pragma unroll
      for (int q = 0; q < Q; ++q) g1[(size_t)q * g.nb + bi] = f[q];
    }
    const int k = kc[c];
    double rho, u[3];
    moments<LAT>(f, rho, u);
    const double om = k ? ph.om[1] : ph.om[0];
    const double* a = ph.acc[k];
#pragma unroll
    for (int q = 0; q < Q; ++q) fout[(size_t)q * g.nc + c] = f[q] - om * (f[q] - feq<LAT>(q, rho, u)) + force<LAT>(q, rho, a);
  }
}

// Ghost populations of the fine surface nodes for one sub-step: the coarse
// perimeter sets interpolated in time (weights wa on G(t), wb on G(t+1)) and
// space (the mean of the 2 or 4 coarse nodes beside an odd fine coordinate),
// their non-equilibrium part scaled by tau_f,k / (2 tau_c,k) of the fine
// node's phase k, plus one fine step of body force (a pre-collision set lags
// the physical time by one step of its own level), stored as deviations of
// the phase's reference density; only directions whose source lies outside.
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_r2_inject(Geo g, Phys ph, const double* __restrict__ g0,
                                                   const double* __restrict__ g1, double wa, double wb,
                                                   const uint8_t* __restrict__ ftag,
                                                   typename lsb::Step<LAT, ST>::R* __restrict__ ghost) {
  using L = Lat<LAT>;
  using R = typename lsb::Step<LAT, ST>::R;
  constexpr int Q = L::Q;
  for (long sidx = blockIdx.x * 256L + threadIdx.x; sidx < g.ns; sidx += (long)gridDim.x * 256) {
    int i, j, k;
    surface_coords(g, sidx, i, j, k);
    const long c = ((long)k * g.fy + j) * g.fx + i;
    const int o0 = i & 1, o1 = j & 1, o2 = g.D == 3 ? (k & 1) : 0;
    const double w = (o0 ? 0.5 : 1.0) * (o1 ? 0.5 : 1.0) * (o2 ? 0.5 : 1.0);
    double H[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) H[q] = 0.0;
    for (int dz = 0; dz <= o2; ++dz)
      for (int dy = 0; dy <= o1; ++dy)
        for (int dx = 0; dx <= o0; ++dx) {
          const long bx = bidx(g, g.b[0] + (i - o0) / 2 + dx, g.b[2] + (j - o1) / 2 + dy,
                               g.D == 3 ? g.b[4] + (k - o2) / 2 + dz : 0);
#pragma unroll
          for (int q = 0; q < Q; ++q) H[q] += w * (wa * g0[(size_t)q * g.nb + bx] + wb * g1[(size_t)q * g.nb + bx]);
        }
    double rho, u[3];
    moments<LAT>(H, rho, u);
    const int p = ftag[c] & lsb::T_GAS;
    const double r = ph.tf[p] / (2.0 * ph.tc[p]);
    const double rr = ph.rref[p];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int si = i - L::cx(q), sj = j - L::cy(q), sk = k - L::cz(q);
      const bool out = si < 0 || si >= g.fx || sj < 0 || sj >= g.fy || (g.D == 3 && (sk < 0 || sk >= g.fz));
      if (!out) continue;
      const double e = feq<LAT>(q, rho, u);
      ghost[(size_t)q * g.nf + c] = (R)(e + r * (H[q] - e) + force<LAT>(q, rho, ph.accf[p]) - wgt<LAT>(q) * rr);
    }
  }
}

// Restriction onto every covered coarse node (the coarse step reads only
// the ring next to the perimeter; the others keep the coarse state complete
// for the queries and re-meshing): the coincident fine node's
// pre-collision populations of the second sub-step, pulled again from the
// fine state before it (prev), less one fine step of force, f;
// e = f_eq(moments of f); coarse post-collision e + 2 (tau_c,k - 1) /
// tau_f,k (f - e) + the coarse body force.
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_r2_restrict(Geo g, Phys ph, const typename lsb::Step<LAT, ST>::T* __restrict__ prev,
                                                     const uint8_t* __restrict__ ftag, double* __restrict__ fout,
                                                     uint8_t* __restrict__ kc) {
  using L = Lat<LAT>;
  using S = lsb::Step<LAT, ST>;
  using R = typename S::R;
  using C = typename S::C;
  constexpr int Q = L::Q;
  for (long bi = blockIdx.x * 256L + threadIdx.x; bi < g.nb; bi += (long)gridDim.x * 256) {
    const int I = g.b[0] + (int)(bi % g.bw), J = g.b[2] + (int)((bi / g.bw) % g.bh);
    const int K = g.b[4] + (int)(bi / ((long)g.bw * g.bh));
    if (!covered(g, I, J, K)) continue;
    const int fi = 2 * (I - g.b[0]), fj = 2 * (J - g.b[2]), fk = g.D == 3 ? 2 * (K - g.b[4]) : 0;
    const long fcell = ((long)fk * g.fy + fj) * g.fx + fi;
    const int p = ftag[fcell] & lsb::T_GAS;
    const double rr = ph.rref[p];
    double f[Q], rf = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int src = (int)(((long)(fk - L::cz(q)) * g.fy + (fj - L::cy(q))) * g.fx + (fi - L::cx(q)));
      f[q] = (double)C::dec(prev[lsb::pidx<LAT>(q, src, (size_t)g.nf)], (R)wgt<LAT>(q), (R)ph.inv_scale) +
             wgt<LAT>(q) * rr;
      rf += f[q];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) f[q] -= force<LAT>(q, rf, ph.accf[p]);
    double rho, u[3];
    moments<LAT>(f, rho, u);
    const double a = 2.0 * (ph.tc[p] - 1.0) / ph.tf[p];
    const long c = ((long)K * g.ny + J) * g.nx + I;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const double e = feq<LAT>(q, rho, u);
      fout[(size_t)q * g.nc + c] = e + a * (f[q] - e) + force<LAT>(q, rho, ph.acc[p]);
    }
    kc[c] = (uint8_t)p;
  }
}

// The fine level's LS-active cells keep 3 cells from the box faces.
__global__ __launch_bounds__(256) void k_r2_band(Geo g, const uint8_t* __restrict__ ftag, int* __restrict__ flag) {
  for (long c = blockIdx.x * 256L + threadIdx.x; c < g.nf; c += (long)gridDim.x * 256) {
    int i, j, k;
    fine_coords(g, c, i, j, k);
    const bool shell = i < 3 || i > g.fx - 4 || j < 3 || j > g.fy - 4 || (g.D == 3 && (k < 3 || k > g.fz - 4));
    if (shell && (ftag[c] & lsb::T_ACT)) atomicOr(flag, 1);
  }
}

// The perimeter's pre-collision sets at the current time, inverted from the
// coarse post-collision populations f: with u = m/rho - a_c the
// pre-collision velocity and e = f_eq(rho, u), G = e + tau_c / (tau_c - 1)
// (f - F_c - e) (e at tau_c = 1).
template <int LAT>
__global__ __launch_bounds__(256) void k_r2_perimeter_sets(Geo g, Phys ph, const double* __restrict__ fc,
                                                           const uint8_t* __restrict__ kc, double* __restrict__ g0) {
  constexpr int Q = Lat<LAT>::Q;
  for (long bi = blockIdx.x * 256L + threadIdx.x; bi < g.nb; bi += (long)gridDim.x * 256) {
    const int I = g.b[0] + (int)(bi % g.bw), J = g.b[2] + (int)((bi / g.bw) % g.bh);
    const int K = g.b[4] + (int)(bi / ((long)g.bw * g.bh));
    if (covered(g, I, J, K)) continue;
    const long c = ((long)K * g.ny + J) * g.nx + I;
    const int k = kc[c];
    double f[Q], rho, u[3];
#pragma unroll
    for (int q = 0; q < Q; ++q) f[q] = fc[(size_t)q * g.nc + c];
    moments<LAT>(f, rho, u);
    for (int a = 0; a < 3; ++a) u[a] -= ph.acc[k][a];
    const double r = ph.tc[k] == 1.0 ? 0.0 : ph.tc[k] / (ph.tc[k] - 1.0);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const double e = feq<LAT>(q, rho, u);
      g0[(size_t)q * g.nb + bi] = e + r * (f[q] - force<LAT>(q, rho, ph.acc[k]) - e);
    }
  }
}

// Re-meshing, fine level: the state of the box moved by d coarse nodes
// (2 d fine cells) into the plan's other population and moment buffers and
// into s1 (the level set).  A node inside the old box copies its stored
// populations (same phase, same codec frame), level set and moments; a new
// node takes the coarse post-collision populations H interpolated as at the
// perimeter: with u = m/rho, e_c = f_eq(rho, u - a_c), e_f = f_eq(rho, u -
// a_f), the fine post-collision populations e_f + (tau_f - 1) / (2 (tau_c -
// 1)) (H - F_c - e_c) + F_f (none of H's non-equilibrium part at tau_c = 1),
// the level set at +-band by the coarse phase, moments (rho, u, 0).  g
// describes the new box.
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_r2_remesh_fine(Geo g, Phys ph, int d0, int d1, int d2,
                                                        const double* __restrict__ fc,
                                                        const uint8_t* __restrict__ kc,
                                                        typename lsb::Step<LAT, ST>::Args a) {
  using L = Lat<LAT>;
  using S = lsb::Step<LAT, ST>;
  using R = typename S::R;
  using C = typename S::C;
  constexpr int Q = L::Q;
  const size_t N = (size_t)g.nf;
  for (long c = blockIdx.x * 256L + threadIdx.x; c < g.nf; c += (long)gridDim.x * 256) {
    int i, j, k;
    fine_coords(g, c, i, j, k);
    const int oi = i + 2 * d0, oj = j + 2 * d1, ok = k + 2 * d2;
    if (oi >= 0 && oi < g.fx && oj >= 0 && oj < g.fy && ok >= 0 && ok < g.fz) {
      const int o = (int)(((long)ok * g.fy + oj) * g.fx + oi);
#pragma unroll
      for (int q = 0; q < Q; ++q) a.An[lsb::pidx<LAT>(q, (int)c, N)] = a.A[lsb::pidx<LAT>(q, o, N)];
      a.s1[c] = a.phi[o];
      for (int m = 0; m < 10; ++m) a.Mn[(size_t)m * N + c] = a.M[(size_t)m * N + o];
      continue;
    }
    const int o0 = i & 1, o1 = j & 1, o2 = g.D == 3 ? (k & 1) : 0;
    const double w = (o0 ? 0.5 : 1.0) * (o1 ? 0.5 : 1.0) * (o2 ? 0.5 : 1.0);
    double H[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) H[q] = 0.0;
    int kk = 0;
    for (int dz = 0; dz <= o2; ++dz)
      for (int dy = 0; dy <= o1; ++dy)
        for (int dx = 0; dx <= o0; ++dx) {
          const long cc = ((long)(g.D == 3 ? g.b[4] + (k - o2) / 2 + dz : 0) * g.ny + (g.b[2] + (j - o1) / 2 + dy)) * g.nx +
                          (g.b[0] + (i - o0) / 2 + dx);
          kk = kc[cc];
#pragma unroll
          for (int q = 0; q < Q; ++q) H[q] += w * fc[(size_t)q * g.nc + cc];
        }
    double rho, u[3], uc[3], uf[3];
    moments<LAT>(H, rho, u);
    for (int m = 0; m < 3; ++m) {
      uc[m] = u[m] - ph.acc[kk][m];
      uf[m] = u[m] - ph.accf[kk][m];
    }
    const double ratio = ph.tc[kk] == 1.0 ? 0.0 : (ph.tf[kk] - 1.0) / (2.0 * (ph.tc[kk] - 1.0));
    const R s = a.scale;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const double ec = feq<LAT>(q, rho, uc), ef = feq<LAT>(q, rho, uf);
      const double f = ef + ratio * (H[q] - force<LAT>(q, rho, ph.acc[kk]) - ec) + force<LAT>(q, rho, ph.accf[kk]);
      const R dev = (R)(f - wgt<LAT>(q) * ph.rref[kk]);
      a.An[lsb::pidx<LAT>(q, (int)c, N)] = C::enc(dev, (R)(1.0 / wgt<LAT>(q)), s);
    }
    a.s1[c] = kk ? a.band : -a.band;
    a.Mn[c] = (R)(rho - 1.0);
    for (int m = 0; m < 3; ++m) a.Mn[(size_t)(1 + m) * N + c] = (R)u[m];
    for (int m = 4; m < 10; ++m) a.Mn[(size_t)m * N + c] = (R)0;
  }
}

// Re-meshing: the initial gas centroid moves with the fine coordinates.
__global__ void k_r2_shift_xc0(double* __restrict__ scal, int slot, double dx, double dy, double dz) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    scal[slot] -= dx;
    scal[slot + 1] -= dy;
    scal[slot + 2] -= dz;
  }
}

// Sensor: bounding box of the fine cells with phi >= -d_ref (lo[3], hi[3]
// in out[0..5], started at (INT_MAX, -1)).
template <class R>
__global__ __launch_bounds__(256) void k_r2_sensor(Geo g, const R* __restrict__ phi, double d_ref, int* __restrict__ out) {
  for (long c = blockIdx.x * 256L + threadIdx.x; c < g.nf; c += (long)gridDim.x * 256) {
    if (!((double)phi[c] >= -d_ref)) continue;
    int i, j, k;
    fine_coords(g, c, i, j, k);
    atomicMin(&out[0], i);
    atomicMin(&out[1], j);
    atomicMin(&out[2], k);
    atomicMax(&out[3], i);
    atomicMax(&out[4], j);
    atomicMax(&out[5], k);
  }
}
__global__ void k_r2_sensor_init(int* __restrict__ out) {
  if (threadIdx.x < 6) out[threadIdx.x] = threadIdx.x < 3 ? 0x7fffffff : -1;
}

int grid_of(long n) { return (int)std::max<long>(1, std::min<long>((n + 255) / 256, 8192)); }

}  // namespace

struct lsb_ref2 {
  lsb_params Pc{}, Pf{};
  int lattice = 0, storage = 0, D = 2, Q = 9;
  Geo g{};
  Phys ph{};
  lsb_plan* fine = nullptr;
  char* ws = nullptr;
  size_t off_f[2] = {0, 0}, off_kc = 0, off_g[2] = {0, 0}, off_flag = 0, off_fine = 0, total = 0;
  int cur = 0, gcur = 0;
  bool bound = false, inited = false;
  long nstep = 0;
};

namespace {

template <int LAT, int ST>
void r2_step(lsb_ref2* r, hipStream_t st) {
  using R = typename lsb::Step<LAT, ST>::R;
  using T = typename lsb::Step<LAT, ST>::T;
  const Geo& g = r->g;
  double* fin = reinterpret_cast<double*>(r->ws + r->off_f[r->cur]);
  double* fout = reinterpret_cast<double*>(r->ws + r->off_f[r->cur ^ 1]);
  uint8_t* kc = reinterpret_cast<uint8_t*>(r->ws + r->off_kc);
  double* g0 = reinterpret_cast<double*>(r->ws + r->off_g[r->gcur]);
  double* g1 = reinterpret_cast<double*>(r->ws + r->off_g[r->gcur ^ 1]);
  lsb_plan* f = r->fine;
  R* ghost = reinterpret_cast<R*>(f->ws + f->off_ghost);
  const uint8_t* ftag = reinterpret_cast<const uint8_t*>(f->ws + f->off_tag);
  k_r2_coarse<LAT><<<grid_of(g.nc), 256, 0, st>>>(g, r->ph, fin, fout, kc, g1);
  for (int sub = 0; sub < 2; ++sub) {
    k_r2_inject<LAT, ST><<<grid_of(g.ns), 256, 0, st>>>(g, r->ph, g0, g1, sub ? 0.0 : 0.5, sub ? 1.0 : 0.5, ftag, ghost);
    f->ops->step(f, st);
    if (f->schedule == LSB_SCHED_OVERLAP) (void)hipStreamWaitEvent(st, f->ev_bulk_done, 0);
  }
  // after the swap the fine plan's other buffer holds the state before the
  // second sub-step
  const T* prev = reinterpret_cast<const T*>(f->ws + f->off_A[f->cur ^ 1]);
  k_r2_restrict<LAT, ST><<<grid_of(g.nb), 256, 0, st>>>(g, r->ph, prev, ftag, fout, kc);
  k_r2_band<<<grid_of(g.nf), 256, 0, st>>>(g, ftag, reinterpret_cast<int*>(r->ws + r->off_flag));
  r->cur ^= 1;
  r->gcur ^= 1;
  ++r->nstep;
}

template <int LAT>
void r2_init_coarse(lsb_ref2* r, const double* phi, const double* rho, const double* u, hipStream_t st) {
  k_r2_init<LAT><<<grid_of(r->g.nc), 256, 0, st>>>(r->g, r->ph, phi, rho, u,
                                                   reinterpret_cast<double*>(r->ws + r->off_f[0]),
                                                   reinterpret_cast<uint8_t*>(r->ws + r->off_kc),
                                                   reinterpret_cast<double*>(r->ws + r->off_g[0]));
}

// Re-meshing of the fine level onto the box now in r->g, moved by d coarse
// nodes: the shifted or new state into the plan's other buffers, which then
// become the current ones (both moment buffers equal), the level set into
// phi and both RK3 buffers, the initial centroid moved; then the plan's
// tags, band, geometry, lists and interface records are built again.
template <int LAT, int ST>
void r2_remesh_fine(lsb_ref2* r, const int* d, hipStream_t st) {
  using Dr = lsb::Driver<LAT, ST>;
  using R = typename lsb::Step<LAT, ST>::R;
  lsb_plan* f = r->fine;
  const typename lsb::Step<LAT, ST>::Args a = Dr::args(f, f->cur);
  k_r2_remesh_fine<LAT, ST><<<grid_of(r->g.nf), 256, 0, st>>>(
      r->g, r->ph, d[0], d[1], d[2], reinterpret_cast<const double*>(r->ws + r->off_f[r->cur]),
      reinterpret_cast<const uint8_t*>(r->ws + r->off_kc), a);
  f->cur ^= 1;
  const size_t N = (size_t)f->N, rb = sizeof(R);
  (void)hipMemcpyAsync(f->ws + f->off_M[f->cur ^ 1], f->ws + f->off_M[f->cur], 10 * N * rb, hipMemcpyDeviceToDevice, st);
  (void)hipMemcpyAsync(f->ws + f->off_phi, f->ws + f->off_s1, N * rb, hipMemcpyDeviceToDevice, st);
  (void)hipMemcpyAsync(f->ws + f->off_s2, f->ws + f->off_s1, N * rb, hipMemcpyDeviceToDevice, st);
  k_r2_shift_xc0<<<1, 64, 0, st>>>(reinterpret_cast<double*>(f->ws + f->off_scal), lsb::SC_XC0, 2.0 * d[0],
                                   2.0 * d[1], 2.0 * d[2]);
  f->ops->rebuild(f, st);
  f->ops->pack(f, st);
  k_r2_perimeter_sets<LAT><<<grid_of(r->g.nb), 256, 0, st>>>(
      r->g, r->ph, reinterpret_cast<const double*>(r->ws + r->off_f[r->cur]),
      reinterpret_cast<const uint8_t*>(r->ws + r->off_kc), reinterpret_cast<double*>(r->ws + r->off_g[r->gcur]));
  k_r2_band<<<grid_of(r->g.nf), 256, 0, st>>>(r->g, reinterpret_cast<const uint8_t*>(f->ws + f->off_tag),
                                               reinterpret_cast<int*>(r->ws + r->off_flag));
}

using RemeshFn = void (*)(lsb_ref2*, const int*, hipStream_t);
template <int LAT>
RemeshFn remesh_fn(int storage) {
  switch (storage) {
    case LSB_F64: return r2_remesh_fine<LAT, LSB_F64>;
    case LSB_F32: return r2_remesh_fine<LAT, LSB_F32>;
    case LSB_F16DEV: return r2_remesh_fine<LAT, LSB_F16DEV>;
    default: return r2_remesh_fine<LAT, LSB_BF16DEV>;
  }
}
RemeshFn remesh_fn(int lattice, int storage) {
  return lattice == LSB_D2Q9 ? remesh_fn<LSB_D2Q9>(storage)
                             : (lattice == LSB_D3Q19 ? remesh_fn<LSB_D3Q19>(storage) : remesh_fn<LSB_D3Q27>(storage));
}

using StepFn = void (*)(lsb_ref2*, hipStream_t);
template <int LAT>
StepFn step_fn(int storage) {
  switch (storage) {
    case LSB_F64: return r2_step<LAT, LSB_F64>;
    case LSB_F32: return r2_step<LAT, LSB_F32>;
    case LSB_F16DEV: return r2_step<LAT, LSB_F16DEV>;
    default: return r2_step<LAT, LSB_BF16DEV>;
  }
}
StepFn step_fn(int lattice, int storage) {
  return lattice == LSB_D2Q9 ? step_fn<LSB_D2Q9>(storage)
                             : (lattice == LSB_D3Q19 ? step_fn<LSB_D3Q19>(storage) : step_fn<LSB_D3Q27>(storage));
}

}  // namespace

extern "C" {

int lsb_ref2_create(const lsb_params* P, const int* box, lsb_ref2** out) {
  if (!P || !box || !out) return fail(LSB_EINVAL, "null argument");
  *out = nullptr;
  if (P->lattice < LSB_D2Q9 || P->lattice > LSB_D3Q27) return fail(LSB_EINVAL, "unknown lattice");
  // coarse walls are not taken on this path (see lsb_refine2.h)
  for (int f = 0; f < 6; ++f)
    if (P->bc[f] != LSB_PERIODIC) return fail(LSB_EINVAL, "the coarse grid must be periodic on every face");
  for (int k = 0; k < 2; ++k)
    if (P->collision[k] != LSB_BGK) return fail(LSB_EINVAL, "two-level grids take the BGK collision only");
  const int D = P->lattice == LSB_D2Q9 ? 2 : 3;
  const int n[3] = {P->nx, P->ny, P->nz};
  for (int a = 0; a < D; ++a)
    if (box[2 * a] < 1 || box[2 * a + 1] > n[a] - 2 || box[2 * a + 1] - box[2 * a] < 4)
      return fail(LSB_EINVAL, "box must keep one coarse node to every grid face and span at least 4 cells per axis");
  if ((double)P->nx * P->ny * P->nz > 2147483647.0 / 2) return fail(LSB_EINVAL, "coarse grid too large");
  lsb_params Pf = *P;
  Pf.nx = 2 * (box[1] - box[0]) + 1;
  Pf.ny = 2 * (box[3] - box[2]) + 1;
  Pf.nz = D == 3 ? 2 * (box[5] - box[4]) + 1 : 1;
  for (int f = 0; f < 6; ++f) Pf.bc[f] = f < 2 * D ? lsb::kFaceInject : LSB_PERIODIC;
  for (int k = 0; k < 2; ++k) {
    Pf.tau[k] = 2.0 * P->tau[k] - 0.5;
    for (int m = 0; m < 3; ++m) Pf.accel[k][m] = 0.5 * P->accel[k][m];
  }
  Pf.sigma = 2.0 * P->sigma;
  Pf.init_hydrostatic = 0;
  lsb_plan* fine = nullptr;
  if (int rc = lsb::create_plan(&Pf, true, &fine)) return rc;
  lsb_ref2* r = new lsb_ref2();
  r->Pc = *P;
  r->Pf = Pf;
  r->lattice = P->lattice;
  r->storage = P->storage;
  r->D = D;
  r->Q = fine->Q;
  r->fine = fine;
  Geo& g = r->g;
  g.D = D;
  g.nx = P->nx; g.ny = P->ny; g.nz = P->nz;
  for (int a = 0; a < 6; ++a) g.b[a] = a < 2 * D ? box[a] : 0;
  g.bw = g.b[1] - g.b[0] + 1;
  g.bh = g.b[3] - g.b[2] + 1;
  g.nc = (long)P->nx * P->ny * P->nz;
  g.nb = (long)g.bw * g.bh * (D == 3 ? g.b[5] - g.b[4] + 1 : 1);
  g.fx = Pf.nx; g.fy = Pf.ny; g.fz = Pf.nz;
  g.nf = (long)Pf.nx * Pf.ny * Pf.nz;
  // surface nodes: all minus the interior block (in 2D the one z plane)
  g.ns = g.nf - (long)(Pf.nx - 2) * (Pf.ny - 2) * (D == 3 ? Pf.nz - 2 : 1);
  Phys& ph = r->ph;
  for (int k = 0; k < 2; ++k) {
    ph.tc[k] = P->tau[k];
    ph.om[k] = 1.0 / P->tau[k];
    ph.tf[k] = Pf.tau[k];
    for (int m = 0; m < 3; ++m) {
      ph.acc[k][m] = P->accel[k][m];
      ph.accf[k][m] = Pf.accel[k][m];
    }
    ph.rref[k] = 1.0;
  }
  ph.inv_scale = P->storage == LSB_F16DEV ? std::ldexp(1.0, -P->fp16_scale_log2) : 1.0;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  for (int b = 0; b < 2; ++b) r->off_f[b] = take((size_t)r->Q * g.nc * sizeof(double));
  r->off_kc = take((size_t)g.nc);
  for (int b = 0; b < 2; ++b) r->off_g[b] = take((size_t)r->Q * g.nb * sizeof(double));
  r->off_flag = take(sizeof(int) * 32);  // band flag [0], sensor bounds [16..21]
  r->off_fine = o;
  r->total = o + fine->total;
  *out = r;
  return LSB_OK;
}

void lsb_ref2_destroy(lsb_ref2* r) {
  if (!r) return;
  lsb_destroy(r->fine);
  delete r;
}

int lsb_ref2_workspace_bytes(const lsb_ref2* r, size_t* bytes) {
  if (!r || !bytes) return fail(LSB_EINVAL, "null argument");
  *bytes = r->total;
  return LSB_OK;
}

int lsb_ref2_bind(lsb_ref2* r, void* ws, size_t bytes) {
  if (!r || !ws) return fail(LSB_EINVAL, "null argument");
  if (bytes < r->total) return fail(LSB_ENOMEM, "workspace too small: need " + std::to_string(r->total) + " bytes");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(LSB_EINVAL, "workspace must be 256-byte aligned");
  if (int rc = lsb_bind(r->fine, static_cast<char*>(ws) + r->off_fine, r->fine->total)) return rc;
  r->ws = static_cast<char*>(ws);
  r->bound = true;
  r->inited = false;
  return LSB_OK;
}

int lsb_ref2_fine_shape(const lsb_ref2* r, int* shape) {
  if (!r || !shape) return fail(LSB_EINVAL, "null argument");
  shape[0] = r->g.fx;
  shape[1] = r->g.fy;
  shape[2] = r->g.fz;
  return LSB_OK;
}

int lsb_ref2_fine(lsb_ref2* r, lsb_plan** fine) {
  if (!r || !fine) return fail(LSB_EINVAL, "null argument");
  *fine = r->fine;
  return LSB_OK;
}

int lsb_ref2_init(lsb_ref2* r, const double* phi_c, const double* rho_c, const double* u_c, const double* phi_f,
                  const double* rho_f, const double* u_f, void* stream) {
  if (!r) return fail(LSB_EINVAL, "null handle");
  if (!r->bound) return fail(LSB_ESTATE, "lsb_ref2_init before lsb_ref2_bind");
  if (!phi_c || !rho_c || !u_c || !phi_f || !rho_f || !u_f) return fail(LSB_EINVAL, "null field");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (int rc = lsb_init(r->fine, phi_f, rho_f, u_f, 1, stream)) return rc;
  // the fine codec's reference densities are fixed by its initialisation
  const bool dev16 = r->storage == LSB_F16DEV || r->storage == LSB_BF16DEV;
  for (int k = 0; k < 2; ++k) r->ph.rref[k] = dev16 ? (double)(float)r->fine->rho_ref[k] : 1.0;
  R2_HIP(hipMemsetAsync(r->ws + r->off_g[0], 0, 2 * (r->off_g[1] - r->off_g[0]), st));
  R2_HIP(hipMemsetAsync(r->ws + r->off_flag, 0, sizeof(int), st));
  R2_HIP(hipMemsetAsync(r->fine->ws + r->fine->off_ghost, 0, (size_t)r->Q * r->g.nf * r->fine->bytes_real, st));
  switch (r->lattice) {
    case LSB_D2Q9: r2_init_coarse<LSB_D2Q9>(r, phi_c, rho_c, u_c, st); break;
    case LSB_D3Q19: r2_init_coarse<LSB_D3Q19>(r, phi_c, rho_c, u_c, st); break;
    default: r2_init_coarse<LSB_D3Q27>(r, phi_c, rho_c, u_c, st); break;
  }
  R2_HIP(hipGetLastError());
  r->cur = 0;
  r->gcur = 0;
  r->nstep = 0;
  r->inited = true;
  return LSB_OK;
}

int lsb_ref2_step(lsb_ref2* r, int nsteps, void* stream) {
  if (!r) return fail(LSB_EINVAL, "null handle");
  if (!r->inited) return fail(LSB_ESTATE, "lsb_ref2_step before lsb_ref2_init");
  if (nsteps < 0) return fail(LSB_EINVAL, "negative step count");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const StepFn fn = step_fn(r->lattice, r->storage);
  for (int s = 0; s < nsteps; ++s) {
    fn(r, st);
    R2_HIP(hipGetLastError());
  }
  int flag = 0;
  R2_HIP(hipMemcpyAsync(&flag, r->ws + r->off_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  R2_HIP(hipStreamSynchronize(st));
  if (flag) return fail(LSB_EBAND, "the level-set band came within 3 fine cells of the refined box's faces");
  return LSB_OK;
}

long lsb_ref2_step_count(const lsb_ref2* r) { return r ? r->nstep : -1; }

int lsb_ref2_get_box(const lsb_ref2* r, int* box) {
  if (!r || !box) return fail(LSB_EINVAL, "null argument");
  for (int a = 0; a < 6; ++a) box[a] = r->g.b[a];
  return LSB_OK;
}

int lsb_ref2_sensor(lsb_ref2* r, double d_ref, int* box, void* stream) {
  if (!r || !box) return fail(LSB_EINVAL, "null argument");
  if (!r->inited) return fail(LSB_ESTATE, "no state");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int* dev = reinterpret_cast<int*>(r->ws + r->off_flag) + 16;
  k_r2_sensor_init<<<1, 64, 0, st>>>(dev);
  const char* phi = r->fine->ws + r->fine->off_phi;
  if (r->storage == LSB_F64)
    k_r2_sensor<double><<<grid_of(r->g.nf), 256, 0, st>>>(r->g, reinterpret_cast<const double*>(phi), d_ref, dev);
  else
    k_r2_sensor<float><<<grid_of(r->g.nf), 256, 0, st>>>(r->g, reinterpret_cast<const float*>(phi), d_ref, dev);
  R2_HIP(hipGetLastError());
  int lohi[6];
  R2_HIP(hipMemcpyAsync(lohi, dev, sizeof(lohi), hipMemcpyDeviceToHost, st));
  R2_HIP(hipStreamSynchronize(st));
  const Geo& g = r->g;
  for (int a = 0; a < 6; ++a) box[a] = g.b[a];
  if (lohi[3] < 0) return LSB_OK;
  const int n[3] = {g.nx, g.ny, g.nz};
  for (int a = 0; a < r->D; ++a) {
    // the tagged cells' bounding box centred: origin round(b0 + (lo + hi) / 4
    // - E / 2), counted in quarter nodes, clamped one node inside the grid
    const int E = g.b[2 * a + 1] - g.b[2 * a];
    const long q4 = 4L * g.b[2 * a] + lohi[a] + lohi[3 + a] - 2L * E + 2;
    long b0 = q4 >= 0 ? q4 / 4 : -((-q4 + 3) / 4);
    b0 = std::max<long>(1, std::min<long>(b0, n[a] - 2 - E));
    box[2 * a] = (int)b0;
    box[2 * a + 1] = (int)b0 + E;
  }
  return LSB_OK;
}

int lsb_ref2_remesh(lsb_ref2* r, const int* box, void* stream) {
  if (!r || !box) return fail(LSB_EINVAL, "null argument");
  if (!r->inited) return fail(LSB_ESTATE, "lsb_ref2_remesh before lsb_ref2_init");
  Geo& g = r->g;
  const int n[3] = {g.nx, g.ny, g.nz};
  int d[3] = {0, 0, 0};
  for (int a = 0; a < r->D; ++a) {
    if (box[2 * a + 1] - box[2 * a] != g.b[2 * a + 1] - g.b[2 * a])
      return fail(LSB_EINVAL, "re-meshing keeps the box extents");
    if (box[2 * a] < 1 || box[2 * a + 1] > n[a] - 2)
      return fail(LSB_EINVAL, "box must keep one coarse node to every grid face");
    d[a] = box[2 * a] - g.b[2 * a];
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int a = 0; a < r->D; ++a) {
    g.b[2 * a] = box[2 * a];
    g.b[2 * a + 1] = box[2 * a + 1];
  }
  remesh_fn(r->lattice, r->storage)(r, d, st);
  R2_HIP(hipGetLastError());
  int flag = 0;
  R2_HIP(hipMemcpyAsync(&flag, r->ws + r->off_flag, sizeof(int), hipMemcpyDeviceToHost, st));
  R2_HIP(hipStreamSynchronize(st));
  if (flag) return fail(LSB_EBAND, "the level-set band is not inside the refined box with 3 fine cells to spare");
  return LSB_OK;
}

int lsb_ref2_get_coarse(lsb_ref2* r, double* pop, uint8_t* phase, void* stream) {
  if (!r) return fail(LSB_EINVAL, "null handle");
  if (!r->inited) return fail(LSB_ESTATE, "no state");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (pop)
    R2_HIP(hipMemcpyAsync(pop, r->ws + r->off_f[r->cur], (size_t)r->Q * r->g.nc * sizeof(double),
                          hipMemcpyDeviceToDevice, st));
  if (phase) R2_HIP(hipMemcpyAsync(phase, r->ws + r->off_kc, (size_t)r->g.nc, hipMemcpyDeviceToDevice, st));
  return LSB_OK;
}

}  // extern "C"
