// refine.hip -- static grid refinement of the lattice Boltzmann solver
// (D2Q9, D3Q19, D3Q27; BGK, FP64, ratio 2; two to four nested levels) behind
// the C ABI of lsb_refine.h.
//
// The coupling of the levels follows the approach the paper adopts for its
// refinement jumps (Sec. 2, lattice Boltzmann method): populations missing
// at the jump come from the other level by interpolation in space and time,
// and the collision frequency eq. (omega) is taken per level for a single
// viscosity (tau_f = 2 tau_c - 1/2).  lsb_refine.h states the steps.
//
// Per coarse step, bandwidth-bound FP64 streams (Q x 8 B read and written
// per node update) and one small perimeter launch:
//   k_ref_coarse  pull + BGK on the uncovered coarse nodes; the perimeter
//                 nodes also keep their pre-collision sets (G(t+1)), stored
//                 face by face;
//   k_ref_edge    per fine perimeter node, the populations whose source lies
//                 outside the patch, from G, stored where the pull reads
//                 them: a one-node ghost shell around the fine arrays; both
//                 fine sub-steps' shells in one launch;
//   k_ref_fine    pull + BGK on the fine nodes (no branch on the perimeter);
//                 the second sub-step restricts onto the covered coarse
//                 nodes.
// With nested levels a refined level is also the parent of the next: its
// k_ref_fine keeps the child perimeter's sets as k_ref_coarse does, and each
// of its sub-steps is followed by the child's edge and two fine launches.
// One x-row segment of 256 nodes per block (x along the lanes), so every
// population plane is read and written in contiguous 2 KB runs; blocks are
// ordered so that each XCD streams a contiguous band of rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "common.h"
#include "../../include/lsb_refine.h"

namespace lsb {
void set_error(const std::string& msg);
}

namespace {

using lsb::Lat;
using lsb::wgt;

// One pair of adjacent levels: the parent (coarse) and its patch (fine).
// Parent node (I, J, K) sits at po + (K ph + J) pw + I of a population plane
// of nc entries: for the periodic coarse grid pw = nx, ph = ny, po = 0; for
// a refined parent its padded pitches and the offset of its node (0, 0, 0).
struct RefArgs {
  int D;
  int nx, ny, nz, ia, ib, ja, jb, ka, kb, mx, my, mz;  // parent nodes per axis; fine nodes (mx + 1) x (my + 1) x (mz + 1)
  int pw, ph;                                          // parent pitches
  long po;                                             // parent node (0, 0, 0)
  int bw, bh, bd;                                      // patch box extents in x, y, z (bd = 1 in 2D)
  int fw, fh;                                          // fine pitches with the ghost shell: row_pitch(mx), my + 3
  long nc, nf, nb;                                     // nodes: coarse, fine (with the shell), box surface
  long fo[6];                                          // start of each face's nodes in the surface arrays
  double tc, tf;
  const double* fc_in;
  double* fc_out;
  const double* ff_in;
  double* ff_out;
  const double* g0;  // coarse pre-collision sets on the box surface, time t
  double* g1;        // time t + 1
};

// The boxes refining one grid, as its kernels see them: each box's extent in
// the grid's node coordinates, its perimeter-set faces and where the sets of
// the time level being written go (g).
constexpr int kMaxKids = LSB_REF_MAX_BOXES;

struct KidBox {
  int D, ia, ib, ja, jb, ka, kb, bw, bh;
  long fo[6], nb;
  double* g;
};

struct Kids {
  int n;
  KidBox k[kMaxKids];
};

// Blocks are dispatched round-robin over the 8 XCDs; logical block L of a
// row-major (row, segment) order goes to one XCD's contiguous share, so the
// rows a block pulls from sit in the same L2.  A bijection of [0, nb) for
// any nb.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned x = b & 7u, k = b >> 3, q = nb >> 3, r = nb & 7u;
  return x * q + (x < r ? x : r) + k;
}

template <int LAT>
__device__ __forceinline__ void moments(const double* f, double& rho, double& ux, double& uy, double& uz) {
  using L = Lat<LAT>;
  rho = 0.0;
  double mx = 0.0, my = 0.0, mz = 0.0;
#pragma unroll
  for (int q = 0; q < L::Q; ++q) {
    rho += f[q];
    mx += L::cx(q) * f[q];
    my += L::cy(q) * f[q];
    mz += L::cz(q) * f[q];
  }
  ux = mx / rho;
  uy = my / rho;
  uz = mz / rho;
}

// eq. (feq), c_s^2 = 1/3
template <int LAT>
__device__ __forceinline__ double equilibrium(int q, double rho, double ux, double uy, double uz) {
  using L = Lat<LAT>;
  const double uu = ux * ux + uy * uy + uz * uz;
  const double cu = L::cx(q) * ux + L::cy(q) * uy + L::cz(q) * uz;
  return wgt<LAT>(q) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

// The coarse perimeter's sets are stored face by face, each face a 2D array
// whose fastest index runs along the face (y on the x faces, x on the y and
// z faces), so the threads of a face read consecutive entries.  Faces: 0/1
// at I = ia / ib, 2/3 at J = ja / jb, 4/5 at K = ka / kb (3D).  A node on an
// edge or corner of the box is stored on each of its faces.
template <class B>
__device__ __forceinline__ long face_index(const B& a, int f, int I, int J, int K) {
  if (f < 2) return a.fo[f] + (long)(K - a.ka) * a.bh + (J - a.ja);
  if (f < 4) return a.fo[f] + (long)(K - a.ka) * a.bw + (I - a.ia);
  return a.fo[f] + (long)(J - a.ja) * a.bw + (I - a.ia);
}

// stores set v (Q values) of perimeter node (I, J, K) on each face it lies on
template <int Q, class B>
__device__ __forceinline__ void store_faces(const B& a, double* g, int I, int J, int K, const double* v) {
  const bool on[6] = {I == a.ia, I == a.ib, J == a.ja, J == a.jb, a.D == 3 && K == a.ka, a.D == 3 && K == a.kb};
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    if (!on[f]) continue;
    const long b = face_index(a, f, I, J, K);
#pragma unroll
    for (int q = 0; q < Q; ++q) g[q * a.nb + b] = v[q];
  }
}

template <class B>
__device__ __forceinline__ bool covered(const B& a, int I, int J, int K) {
  return I > a.ia && I < a.ib && J > a.ja && J < a.jb && (a.D == 2 || (K > a.ka && K < a.kb));
}

template <class B>
__device__ __forceinline__ bool in_box(const B& a, int I, int J, int K) {
  return I >= a.ia && I <= a.ib && J >= a.ja && J <= a.jb && (a.D == 2 || (K >= a.ka && K <= a.kb));
}

// A refined level's rows start their node 0 at column 16 of a pitch that is
// a multiple of 16 doubles, so a 256-node row segment is 128-byte aligned;
// columns 15 and mx + 17 hold the ghost shell.
constexpr int kRowOrigin = 16;

__host__ __device__ __forceinline__ int row_pitch(int mx) { return (mx + kRowOrigin + 2 + 15) & ~15; }

__device__ __forceinline__ long fine_index(const RefArgs& a, int i, int j, int k) {
  return ((long)(k + (a.D == 3 ? 1 : 0)) * a.fh + (j + 1)) * a.fw + i + kRowOrigin;
}

// One level's nodes in its population arrays: sx x sy x sz nodes, node
// (i, j, k) at po + (k ph + j) pw + i of planes of n entries.
struct Grid {
  int sx, sy, sz, pw, ph;
  long po, n;
};

// equilibrium initial state of one grid; its boxes' perimeter sets G(t) are
// those equilibria
template <int LAT>
__global__ __launch_bounds__(256) void k_ref_init_level(Grid g, const double* rho, const double* u, double* f,
                                                        Kids kids) {
  constexpr int Q = Lat<LAT>::Q, D = Lat<LAT>::D;
  const long nn = (long)g.sx * g.sy * g.sz;
  for (long n = (long)blockIdx.x * 256 + threadIdx.x; n < nn; n += (long)gridDim.x * 256) {
    const int i = (int)(n % g.sx), j = (int)((n / g.sx) % g.sy), k = (int)(n / ((long)g.sx * g.sy));
    const double ux = u[D * n], uy = u[D * n + 1], uz = D == 3 ? u[D * n + 2] : 0.0;
    const long p = g.po + ((long)k * g.ph + j) * g.pw + i;
    double e[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      e[q] = equilibrium<LAT>(q, rho[n], ux, uy, uz);
      f[q * g.n + p] = e[q];
    }
    for (int b = 0; b < kids.n; ++b)
      if (in_box(kids.k[b], i, j, k) && !covered(kids.k[b], i, j, k)) store_faces<Q>(kids.k[b], kids.k[b].g, i, j, k, e);
  }
}

// uncovered coarse nodes: pull (periodic), keep the pre-collision sets of
// the boxes' perimeter nodes, collide with tau_c
template <int LAT>
__global__ __launch_bounds__(256) void k_ref_coarse(RefArgs a, Kids kids, int segs) {
  using L = Lat<LAT>;
  constexpr int Q = L::Q;
  const int Lb = (int)xcd_block(blockIdx.x, gridDim.x);
  const int row = Lb / segs, x = (Lb - row * segs) * 256 + (int)threadIdx.x;
  if (x >= a.nx) return;
  const int y = row % a.ny, z = row / a.ny;
  int kid = -1;  // the box whose perimeter or interior holds the node (boxes are disjoint)
  for (int b = 0; b < kids.n; ++b)
    if (in_box(kids.k[b], x, y, z)) kid = b;
  if (kid >= 0 && covered(kids.k[kid], x, y, z)) return;  // restricted from the fine level
  const int xs[3] = {x + 1 == a.nx ? 0 : x + 1, x, x == 0 ? a.nx - 1 : x - 1};  // source for c = -1, 0, 1
  const int ys[3] = {y + 1 == a.ny ? 0 : y + 1, y, y == 0 ? a.ny - 1 : y - 1};
  const int zs[3] = {z + 1 == a.nz ? 0 : z + 1, z, z == 0 ? a.nz - 1 : z - 1};
  double f[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q)
    f[q] = a.fc_in[q * a.nc + ((long)zs[L::cz(q) + 1] * a.ny + ys[L::cy(q) + 1]) * a.nx + xs[L::cx(q) + 1]];
  if (kid >= 0) store_faces<Q>(kids.k[kid], kids.k[kid].g, x, y, z, f);
  double rho, ux, uy, uz;
  moments<LAT>(f, rho, ux, uy, uz);
  const long n = ((long)z * a.ny + y) * a.nx + x;
#pragma unroll
  for (int q = 0; q < Q; ++q) a.fc_out[q * a.nc + n] = f[q] - (f[q] - equilibrium<LAT>(q, rho, ux, uy, uz)) / a.tc;
}

// fine perimeter nodes: the populations whose source lies outside the patch
// (time weights wa on G(t), wb on G(t+1)), written into the ghost shell of
// the fine buffer that sub-step reads, where k_ref_fine pulls them from;
// both sub-steps in one launch (blockIdx.y), since the shells are disjoint
// from what the fine steps write and G(t), G(t+1) are known once the coarse
// step is done.  Each surface node has one owner: the x faces take all their
// nodes, the y faces those with 0 < i < mx, the z faces (3D) those with
// 0 < i < mx and 0 < j < my.
template <int LAT>
__global__ __launch_bounds__(256) void k_ref_edge(RefArgs a, double* ff1, double* ff2) {
  using L = Lat<LAT>;
  constexpr int Q = L::Q;
  const double wa = blockIdx.y == 0 ? 0.5 : 0.0, wb = blockIdx.y == 0 ? 0.5 : 1.0;
  double* ff = blockIdx.y == 0 ? ff1 : ff2;
  long t = (long)blockIdx.x * 256 + threadIdx.x;
  const long ax = (long)(a.my + 1) * (a.mz + 1), ay = (long)(a.mx - 1) * (a.mz + 1);
  const long az = a.D == 3 ? (long)(a.mx - 1) * (a.my - 1) : 0;
  int i, j, k, face;
  if (t < 2 * ax) {
    const long u = t % ax;
    face = t < ax ? 0 : 1;
    i = t < ax ? 0 : a.mx;
    j = (int)(u % (a.my + 1));
    k = (int)(u / (a.my + 1));
  } else if ((t -= 2 * ax) < 2 * ay) {
    const long u = t % ay;
    face = t < ay ? 2 : 3;
    j = t < ay ? 0 : a.my;
    i = 1 + (int)(u % (a.mx - 1));
    k = (int)(u / (a.mx - 1));
  } else if ((t -= 2 * ay) < 2 * az) {
    const long u = t % az;
    face = t < az ? 4 : 5;
    k = t < az ? 0 : a.mz;
    i = 1 + (int)(u % (a.mx - 1));
    j = 1 + (int)(u / (a.mx - 1));
  } else {
    return;
  }
  // the coarse set at this node: along each odd coordinate the mean of the
  // two coarse nodes beside it (z outermost, x innermost), all on the node's
  // face
  const int ox = i & 1, oy = j & 1, oz = k & 1;
  const double s = (ox ? 0.5 : 1.0) * (oy ? 0.5 : 1.0) * (oz ? 0.5 : 1.0);
  double H[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) H[q] = 0.0;
  for (int dz = 0; dz <= oz; ++dz)
    for (int dy = 0; dy <= oy; ++dy)
      for (int dx = 0; dx <= ox; ++dx) {
        const long b = face_index(a, face, a.ia + (i - ox) / 2 + dx, a.ja + (j - oy) / 2 + dy, a.ka + (k - oz) / 2 + dz);
#pragma unroll
        for (int q = 0; q < Q; ++q) H[q] += s * (wa * a.g0[q * a.nb + b] + wb * a.g1[q * a.nb + b]);
      }
  double rh, uxh, uyh, uzh;
  moments<LAT>(H, rh, uxh, uyh, uzh);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int si = i - L::cx(q), sj = j - L::cy(q), sk = k - L::cz(q);
    if (si < 0 || si > a.mx || sj < 0 || sj > a.my || sk < 0 || sk > a.mz) {
      const double eh = equilibrium<LAT>(q, rh, uxh, uyh, uzh);
      ff[q * a.nf + fine_index(a, si, sj, sk)] = eh + a.tf / (2.0 * a.tc) * (H[q] - eh);
    }
  }
}

// fine nodes: pull (the ghost shell holds the perimeter's inward populations),
// collide with tau_f; with restrict_ set, the fine nodes on covered coarse
// nodes write those nodes' post-collision populations.  With child boxes
// (this level as their parent), the nodes on a child's perimeter keep their
// pre-collision sets (the child's G(t+1)) and the nodes a child covers store
// nothing (the child's restriction writes them).
template <int LAT, bool CHILD>
__global__ __launch_bounds__(256) void k_ref_fine(RefArgs a, Kids kids, int segs, int restrict_) {
  using L = Lat<LAT>;
  constexpr int Q = L::Q;
  const int Lb = (int)xcd_block(blockIdx.x, gridDim.x);
  const int row = Lb / segs, i = (Lb - row * segs) * 256 + (int)threadIdx.x;
  if (i > a.mx) return;
  const int j = row % (a.my + 1), k = row / (a.my + 1);
  const long p = fine_index(a, i, j, k);
  const long plane = (long)a.fw * a.fh;
  double f[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) f[q] = a.ff_in[q * a.nf + p - L::cz(q) * plane - L::cy(q) * a.fw - L::cx(q)];
  bool keep = true;
  if (CHILD) {
    int kid = -1;
    for (int b = 0; b < kids.n; ++b)
      if (in_box(kids.k[b], i, j, k)) kid = b;
    if (kid >= 0) {
      if (covered(kids.k[kid], i, j, k)) keep = false;
      else store_faces<Q>(kids.k[kid], kids.k[kid].g, i, j, k, f);
    }
  }
  double rho, ux, uy, uz;
  moments<LAT>(f, rho, ux, uy, uz);
  const bool rs = restrict_ && !(i & 1) && !(j & 1) && !(k & 1) && covered(a, a.ia + i / 2, a.ja + j / 2, a.ka + k / 2);
  const long m = rs ? a.po + ((long)(a.ka + k / 2) * a.ph + a.ja + j / 2) * a.pw + a.ia + i / 2 : 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double e = equilibrium<LAT>(q, rho, ux, uy, uz);
    if (keep) a.ff_out[q * a.nf + p] = f[q] - (f[q] - e) / a.tf;
    if (rs) a.fc_out[q * a.nc + m] = e + 2.0 * (a.tc - 1.0) / a.tf * (f[q] - e);
  }
}

// the fine nodes without the ghost shell, [Q][nodes]
__global__ __launch_bounds__(256) void k_ref_unpad(RefArgs a, int Q, const double* ff, double* out) {
  const long n1 = (long)(a.mx + 1) * (a.my + 1) * (a.mz + 1);
  for (long t = (long)blockIdx.x * 256 + threadIdx.x; t < Q * n1; t += (long)gridDim.x * 256) {
    const long q = t / n1, n = t - q * n1;
    const int i = (int)(n % (a.mx + 1)), j = (int)((n / (a.mx + 1)) % (a.my + 1));
    const int k = (int)(n / ((long)(a.mx + 1) * (a.my + 1)));
    out[t] = ff[q * a.nf + fine_index(a, i, j, k)];
  }
}

// Level-set refinement sensor (Sec. 3, adaptive mesh refinement): coarse
// nodes in the gas or within d_ref of it are tagged.  The level set here is
// >= 0 in the gas, the opposite of the sign the sensor is written with, so
// the test is phi >= -d_ref.  Per block the bounding box of the tagged nodes
// (lo x, y, z then hi x, y, z; lo = n, hi = -1 when none).
constexpr int kSensorBlocks = 1024;

__device__ __forceinline__ int block_min(int v, int* sh) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  v = min(min(sh[0], sh[1]), min(sh[2], sh[3]));
  __syncthreads();
  return v;
}

__global__ __launch_bounds__(256) void k_ref_sensor(RefArgs a, const double* phi, double d_ref, int* part) {
  __shared__ int sh[4];
  // his are reduced as minima of -x (start +1: -1 when nothing is tagged)
  int v[6] = {a.nx, a.ny, a.nz, 1, 1, 1};
  for (long n = (long)blockIdx.x * 256 + threadIdx.x; n < a.nc; n += (long)gridDim.x * 256) {
    if (!(phi[n] >= -d_ref)) continue;
    const int x = (int)(n % a.nx), y = (int)((n / a.nx) % a.ny), z = (int)(n / ((long)a.nx * a.ny));
    v[0] = min(v[0], x);
    v[1] = min(v[1], y);
    v[2] = min(v[2], z);
    v[3] = min(v[3], -x);
    v[4] = min(v[4], -y);
    v[5] = min(v[5], -z);
  }
  for (int d = 0; d < 6; ++d) {
    const int m = block_min(v[d], sh);
    if (threadIdx.x == 0) part[blockIdx.x * 6 + d] = m;
  }
}

// Seeded sensor: every tagged node belongs to its nearest seed (a coarse
// node; squared distances in 64-bit integers, ties to the lower index); per
// block and seed the bounding box of its nodes, reduced as k_ref_sensor
// does.  part: [block][seed][6].
constexpr int kMaxSeeds = LSB_REF_MAX_BOXES;

struct Seeds {
  int n;
  int p[kMaxSeeds][3];
};

__global__ __launch_bounds__(256) void k_ref_sensor_seeded(RefArgs a, const double* phi, double d_ref, Seeds sd,
                                                           int* part) {
  __shared__ int sh[4];
  int v[kMaxSeeds][6];
#pragma unroll
  for (int k = 0; k < kMaxSeeds; ++k) {
    v[k][0] = a.nx;
    v[k][1] = a.ny;
    v[k][2] = a.nz;
    v[k][3] = v[k][4] = v[k][5] = 1;
  }
  for (long n = (long)blockIdx.x * 256 + threadIdx.x; n < a.nc; n += (long)gridDim.x * 256) {
    if (!(phi[n] >= -d_ref)) continue;
    const int x = (int)(n % a.nx), y = (int)((n / a.nx) % a.ny), z = (int)(n / ((long)a.nx * a.ny));
    int best = 0;
    long bd = -1;
    for (int k = 0; k < sd.n; ++k) {
      const long dx = x - sd.p[k][0], dy = y - sd.p[k][1], dz = z - sd.p[k][2];
      const long dd = dx * dx + dy * dy + dz * dz;
      if (bd < 0 || dd < bd) {
        bd = dd;
        best = k;
      }
    }
#pragma unroll
    for (int k = 0; k < kMaxSeeds; ++k)
      if (best == k) {
        v[k][0] = min(v[k][0], x);
        v[k][1] = min(v[k][1], y);
        v[k][2] = min(v[k][2], z);
        v[k][3] = min(v[k][3], -x);
        v[k][4] = min(v[k][4], -y);
        v[k][5] = min(v[k][5], -z);
      }
  }
  for (int k = 0; k < sd.n; ++k) {
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      int w = v[0][d];  // v[k][d] without a runtime index into the registers
#pragma unroll
      for (int j = 1; j < kMaxSeeds; ++j) w = j == k ? v[j][d] : w;
      const int m = block_min(w, sh);
      if (threadIdx.x == 0) part[((long)blockIdx.x * kMaxSeeds + k) * 6 + d] = m;
    }
  }
}

// reduces nslots boxes over nparts blocks: part [block][slot][6] -> box [slot][6]
__global__ __launch_bounds__(256) void k_ref_sensor_final(int nparts, int nslots, int stride, const int* part, int* box) {
  __shared__ int sh[4];
  for (int k = 0; k < nslots; ++k)
    for (int d = 0; d < 6; ++d) {
      int v = 0x7fffffff;
      for (int b = threadIdx.x; b < nparts; b += 256) v = min(v, part[((long)b * stride + k) * 6 + d]);
      v = block_min(v, sh);
      if (threadIdx.x == 0) box[k * 6 + d] = d < 3 ? v : -v;
    }
}

// Re-meshing of one refined level (state at the end of a coarse step, the
// parent already re-meshed): new nodes at positions the old level covered
// keep the old populations; the others take the parent's post-collision
// populations interpolated like the perimeter's (the mean of the 2, 4 or 8
// parent nodes around an off-grid node), the non-equilibrium part scaled by
// (tau_f - 1) / (2 (tau_c - 1)) about the equilibrium of the interpolated
// moments (the equilibrium alone at tau_c = 1).  Old geometry: o (its
// buffer off); sx, sy, sz: how far the parent's first node moved, in this
// level's spacing (0 for level 1).
template <int LAT>
__global__ __launch_bounds__(256) void k_ref_remesh_fine(RefArgs a, RefArgs o, int sx, int sy, int sz,
                                                         const double* off, double* ff) {
  using L = Lat<LAT>;
  constexpr int Q = L::Q;
  const long n1 = (long)(a.mx + 1) * (a.my + 1) * (a.mz + 1);
  const bool flat = a.tc == 1.0;
  const double up = flat ? 0.0 : (a.tf - 1.0) / (2.0 * (a.tc - 1.0));
  for (long n = (long)blockIdx.x * 256 + threadIdx.x; n < n1; n += (long)gridDim.x * 256) {
    const int i = (int)(n % (a.mx + 1)), j = (int)((n / (a.mx + 1)) % (a.my + 1));
    const int k = (int)(n / ((long)(a.mx + 1) * (a.my + 1)));
    const int X2 = 2 * a.ia + i, Y2 = 2 * a.ja + j, Z2 = 2 * a.ka + k;  // twice the parent-unit position
    const int oi = X2 - 2 * o.ia + sx, oj = Y2 - 2 * o.ja + sy, ok = Z2 - 2 * o.ka + sz;
    const long p = fine_index(a, i, j, k);
    if (oi >= 0 && oi <= o.mx && oj >= 0 && oj <= o.my && ok >= 0 && ok <= o.mz) {
      const long op = fine_index(o, oi, oj, ok);
#pragma unroll
      for (int q = 0; q < Q; ++q) ff[q * a.nf + p] = off[q * o.nf + op];
      continue;
    }
    const int ox = X2 & 1, oy = Y2 & 1, oz = Z2 & 1;
    const double s = (ox ? 0.5 : 1.0) * (oy ? 0.5 : 1.0) * (oz ? 0.5 : 1.0);
    double H[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) H[q] = 0.0;
    for (int dz = 0; dz <= oz; ++dz)
      for (int dy = 0; dy <= oy; ++dy)
        for (int dx = 0; dx <= ox; ++dx) {
          const long m = a.po + ((long)((Z2 - oz) / 2 + dz) * a.ph + (Y2 - oy) / 2 + dy) * a.pw + (X2 - ox) / 2 + dx;
#pragma unroll
          for (int q = 0; q < Q; ++q) H[q] += s * a.fc_in[q * a.nc + m];
        }
    double rho, ux, uy, uz;
    moments<LAT>(H, rho, ux, uy, uz);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const double e = equilibrium<LAT>(q, rho, ux, uy, uz);
      ff[q * a.nf + p] = e + up * (H[q] - e);
    }
  }
}

// the new perimeter's pre-collision sets G(t) from the parent's
// post-collision populations, inverting the BGK step:
// f_eq + tau_c / (tau_c - 1) (f - f_eq) (f_eq at tau_c = 1)
template <int LAT>
__global__ __launch_bounds__(256) void k_ref_remesh_g(RefArgs a, double* g) {
  using L = Lat<LAT>;
  constexpr int Q = L::Q;
  const long nbox = (long)a.bw * a.bh * a.bd;
  const bool flat = a.tc == 1.0;
  const double down = flat ? 0.0 : a.tc / (a.tc - 1.0);
  for (long n = (long)blockIdx.x * 256 + threadIdx.x; n < nbox; n += (long)gridDim.x * 256) {
    const int I = a.ia + (int)(n % a.bw), J = a.ja + (int)((n / a.bw) % a.bh), K = a.ka + (int)(n / ((long)a.bw * a.bh));
    if (covered(a, I, J, K)) continue;
    const long m = a.po + ((long)K * a.ph + J) * a.pw + I;
    double f[Q], v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) f[q] = a.fc_in[q * a.nc + m];
    double rho, ux, uy, uz;
    moments<LAT>(f, rho, ux, uy, uz);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const double e = equilibrium<LAT>(q, rho, ux, uy, uz);
      v[q] = e + down * (f[q] - e);
    }
    store_faces<Q>(a, g, I, J, K, v);
  }
}

// derived geometry of a patch (ia, ib, ja, jb, ka, kb)
void set_patch(RefArgs& a, const int* patch) {
  const bool three = a.D == 3;
  a.ia = patch[0];
  a.ib = patch[1];
  a.ja = patch[2];
  a.jb = patch[3];
  a.ka = three ? patch[4] : 0;
  a.kb = three ? patch[5] : 0;
  a.mx = 2 * (a.ib - a.ia);
  a.my = 2 * (a.jb - a.ja);
  a.mz = 2 * (a.kb - a.ka);
  a.bw = a.ib - a.ia + 1;
  a.bh = a.jb - a.ja + 1;
  a.bd = a.kb - a.ka + 1;
  a.fw = row_pitch(a.mx);
  a.fh = a.my + 3;
  a.nf = (long)a.fw * a.fh * (three ? a.mz + 3 : 1);
  // face sizes: x faces bh x bd, y faces bw x bd, z faces (3D) bw x bh
  const long sz[6] = {(long)a.bh * a.bd, (long)a.bh * a.bd, (long)a.bw * a.bd, (long)a.bw * a.bd,
                      three ? (long)a.bw * a.bh : 0L, three ? (long)a.bw * a.bh : 0L};
  long o = 0;
  for (int f = 0; f < 6; ++f) {
    a.fo[f] = o;
    o += sz[f];
  }
  a.nb = o;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int fail(int code, const std::string& msg) {
  lsb::set_error(msg);
  return code;
}

int q_of(int lattice) { return lattice == LSB_D2Q9 ? 9 : (lattice == LSB_D3Q19 ? 19 : 27); }

}  // namespace

constexpr int kMaxGrids = LSB_REF_MAX_BOXES + 1;

struct lsb_ref {
  lsb_ref_params P;
  RefArgs base;  // the coarse grid and box 1
  int L = 2;     // grids: the coarse grid and L - 1 boxes
  int par[kMaxGrids] = {};      // par[b]: the grid box b refines (0: the coarse grid)
  bool chain = true;            // every box refines the one before it
  RefArgs deep[kMaxGrids];      // deep[b], b >= 2: box b and its parent
  int Q = 9;
  int ext[3] = {0, 0, 0};  // largest patch extents (coarse cells per axis) the workspace holds
  long fcap = 0, bcap = 0;  // fine nodes with the shell, box-surface nodes, at those extents
  int* sens = nullptr;      // sensor partial boxes (kSensorBlocks x 15 x 6) and the reduced boxes (15 x 6)
  char* ws = nullptr;
  size_t ws_bytes = 0;
  double* fc[2] = {nullptr, nullptr};
  double* ff[2] = {nullptr, nullptr};
  double* g[2] = {nullptr, nullptr};
  int dext[kMaxGrids][3] = {};  // capacity extents (parent cells) of boxes 2 ..
  long dcap[kMaxGrids] = {}, dbcap[kMaxGrids] = {};
  double* dff[kMaxGrids][2] = {};
  double* dg[kMaxGrids][2] = {};
  int cur = 0;  // fc[cur] and g[cur] are the current coarse state and box 1's G(t); ff[0] box 1's state
  int dcur[kMaxGrids] = {};  // dg[b][dcur[b]] is box b's G(t); dff[b][0] its state
  bool inited = false;
  // One coarse step as a HIP graph per parity of the buffer state (the
  // state repeats every two steps), captured on first use on a private
  // stream and launched on the caller's; rebuilt after a re-mesh.
  bool use_graphs = true;
  bool graphs_ready = false;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int after_cur[2] = {0, 0};
  int after_dcur[2][kMaxGrids] = {};
  ~lsb_ref() {
    for (int k = 0; k < 2; ++k)
      if (gexec[k]) (void)hipGraphExecDestroy(gexec[k]);
  }
};

namespace {
size_t sizes(const lsb_ref* r, size_t* fcb, size_t* ffb, size_t* gb) {
  *fcb = align256(sizeof(double) * r->Q * (size_t)r->base.nc);
  *ffb = align256(sizeof(double) * r->Q * (size_t)r->fcap);
  *gb = align256(sizeof(double) * r->Q * (size_t)r->bcap);
  size_t t = 2 * (*fcb + *ffb + *gb) + align256(sizeof(int) * 6 * kMaxSeeds * (kSensorBlocks + 1));
  for (int l = 2; l < r->L; ++l)
    t += 2 * (align256(sizeof(double) * r->Q * (size_t)r->dcap[l]) + align256(sizeof(double) * r->Q * (size_t)r->dbcap[l]));
  return t;
}

// the pair args of box l >= 1 (with its parent)
const RefArgs& pair_of(const lsb_ref* r, int l) { return l == 1 ? r->base : r->deep[l]; }

// the coarse grid (as described by box 1's args) as a box's parent
void set_parent_root(RefArgs& a, const RefArgs& b) {
  a.nx = b.nx;
  a.ny = b.ny;
  a.nz = b.nz;
  a.pw = b.nx;
  a.ph = b.ny;
  a.po = 0;
  a.nc = b.nc;
  a.tc = b.tc;
  a.tf = b.tf;
}

// a box (pair args pp) as the parent of another
void set_parent(RefArgs& a, const RefArgs& pp) {
  a.nx = pp.mx + 1;
  a.ny = pp.my + 1;
  a.nz = pp.mz + 1;
  a.pw = pp.fw;
  a.ph = pp.fh;
  a.po = (pp.D == 3 ? (long)pp.fh * pp.fw : 0L) + pp.fw + kRowOrigin;
  a.nc = pp.nf;
  a.tc = pp.tf;
  a.tf = 2.0 * pp.tf - 0.5;
}

Grid grid_of(const lsb_ref* r, int l) {
  if (l == 0) {
    const RefArgs& b = r->base;
    return Grid{b.nx, b.ny, b.nz, b.nx, b.ny, 0L, b.nc};
  }
  const RefArgs& a = pair_of(r, l);
  return Grid{a.mx + 1, a.my + 1, a.mz + 1, a.fw, a.fh, (a.D == 3 ? (long)a.fh * a.fw : 0L) + a.fw + kRowOrigin, a.nf};
}

int check_launch() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LSB_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return LSB_OK;
}

unsigned grid_for(long n) {
  const long g = (n + 255) / 256;
  return (unsigned)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}

// box b's perimeter sets: G(t) (next = 0) or G(t+1) (next = 1)
double* gbuf(const lsb_ref* r, int b, int next) { return b == 1 ? r->g[r->cur ^ next] : r->dg[b][r->dcur[b] ^ next]; }

// the boxes refining grid gi, with the perimeter-set buffers of time level next
Kids kids_of(const lsb_ref* r, int gi, int next) {
  Kids k{};
  for (int b = 1; b < r->L; ++b) {
    if (r->par[b] != gi) continue;
    const RefArgs& a = pair_of(r, b);
    KidBox& c = k.k[k.n++];
    c.D = a.D;
    c.ia = a.ia;
    c.ib = a.ib;
    c.ja = a.ja;
    c.jb = a.jb;
    c.ka = a.ka;
    c.kb = a.kb;
    c.bw = a.bw;
    c.bh = a.bh;
    for (int f = 0; f < 6; ++f) c.fo[f] = a.fo[f];
    c.nb = a.nb;
    c.g = gbuf(r, b, next);
  }
  return k;
}

template <int LAT>
void launch_init(lsb_ref* r, const double* const* rho, const double* const* u, hipStream_t st) {
  for (int l = 0; l < r->L; ++l) {
    const Grid g = grid_of(r, l);
    double* f = l == 0 ? r->fc[0] : (l == 1 ? r->ff[0] : r->dff[l][0]);
    k_ref_init_level<LAT><<<grid_for((long)g.sx * g.sy * g.sz), 256, 0, st>>>(g, rho[l], u[l], f, kids_of(r, l, 0));
  }
}

// While a step is captured into a graph, the boxes refining one grid run on
// branches of their own (they share no data within a parent step: each
// reads its own perimeter sets and writes its own arrays and the parent
// nodes it covers): box c on stream s[c], forked from and joined to the
// parent's stream with events.
struct Cap {
  hipStream_t s[kMaxGrids];
  hipEvent_t fork[kMaxGrids], done[kMaxGrids];
};

template <int LAT>
void advance(lsb_ref* r, int l, double* parent_out, hipStream_t st, Cap* cap);

// the boxes refining grid gi, their two sub-steps each, after the grid's
// step or sub-step (new populations parent_out)
template <int LAT>
void run_kids(lsb_ref* r, int gi, double* parent_out, hipStream_t st, Cap* cap) {
  int n = 0;
  for (int c = 1; c < r->L; ++c) n += r->par[c] == gi;
  if (!cap || n < 2) {
    for (int c = 1; c < r->L; ++c)
      if (r->par[c] == gi) advance<LAT>(r, c, parent_out, st, cap);
    return;
  }
  (void)hipEventRecord(cap->fork[gi], st);
  for (int c = 1; c < r->L; ++c) {
    if (r->par[c] != gi) continue;
    (void)hipStreamWaitEvent(cap->s[c], cap->fork[gi], 0);
    advance<LAT>(r, c, parent_out, cap->s[c], cap);
    (void)hipEventRecord(cap->done[c], cap->s[c]);
    (void)hipStreamWaitEvent(st, cap->done[c], 0);
  }
}

// the two sub-steps of box l within one step of its parent (whose new
// populations, parent_out, receive the restriction), each followed by the
// two sub-steps of each of its own boxes
template <int LAT>
void advance(lsb_ref* r, int l, double* parent_out, hipStream_t st, Cap* cap) {
  RefArgs A = pair_of(r, l);
  double** ffl = l == 1 ? r->ff : r->dff[l];
  A.g0 = gbuf(r, l, 0);
  A.g1 = gbuf(r, l, 1);
  A.fc_out = parent_out;
  const int sf = (A.mx + 1 + 255) / 256;
  const unsigned gf = (unsigned)((long)sf * (A.my + 1) * (A.mz + 1));
  const long surf = 2L * (A.my + 1) * (A.mz + 1) + 2L * (A.mx - 1) * (A.mz + 1) +
                    (A.D == 3 ? 2L * (A.mx - 1) * (A.my - 1) : 0L);
  // inward populations of both sub-steps: G halfway in time, then G(t+1)
  k_ref_edge<LAT><<<dim3((unsigned)((surf + 255) / 256), 2), 256, 0, st>>>(A, ffl[0], ffl[1]);
  for (int s = 0; s < 2; ++s) {
    A.ff_in = ffl[s];
    A.ff_out = ffl[s ^ 1];
    // sub-step 2 also restricts onto the parent's covered nodes
    const Kids K = kids_of(r, l, 1);
    if (K.n > 0) {
      k_ref_fine<LAT, true><<<gf, 256, 0, st>>>(A, K, sf, s);
      run_kids<LAT>(r, l, ffl[s ^ 1], st, cap);
      for (int c = 2; c < r->L; ++c)
        if (r->par[c] == l) r->dcur[c] ^= 1;
    } else {
      k_ref_fine<LAT, false><<<gf, 256, 0, st>>>(A, K, sf, s);
    }
  }
}

template <int LAT>
void launch_steps(lsb_ref* r, int nsteps, hipStream_t st, Cap* cap = nullptr) {
  const RefArgs& b = r->base;
  const int sc = (b.nx + 255) / 256;
  const unsigned gc = (unsigned)((long)sc * b.ny * b.nz);
  for (int s = 0; s < nsteps; ++s) {
    RefArgs a = b;
    a.fc_in = r->fc[r->cur];
    a.fc_out = r->fc[r->cur ^ 1];
    k_ref_coarse<LAT><<<gc, 256, 0, st>>>(a, kids_of(r, 0, 1), sc);
    run_kids<LAT>(r, 0, r->fc[r->cur ^ 1], st, cap);
    for (int c = 2; c < r->L; ++c)
      if (r->par[c] == 0) r->dcur[c] ^= 1;
    r->cur ^= 1;  // box 1's perimeter sets turn with the coarse state
  }
}

void drop_graphs(lsb_ref* r) {
  for (int k = 0; k < 2; ++k)
    if (r->gexec[k]) {
      (void)hipGraphExecDestroy(r->gexec[k]);
      r->gexec[k] = nullptr;
    }
  r->graphs_ready = false;
}

// captures one coarse step from each parity of the state (capturing runs
// nothing on the device but moves the host's buffer bookkeeping as the step
// does; two captures bring it back to where it started, which is checked)
template <int LAT>
int build_graphs(lsb_ref* r) {
  const int cur0 = r->cur;
  int dcur0[kMaxGrids];
  for (int b = 0; b < kMaxGrids; ++b) dcur0[b] = r->dcur[b];
  auto restore = [&]() {
    r->cur = cur0;
    for (int b = 0; b < kMaxGrids; ++b) r->dcur[b] = dcur0[b];
  };
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(LSB_EDEVICE, "stream creation failed");
  Cap cap{};
  int made = 0;
  bool ok = true;
  for (; made < r->L && ok; ++made)
    ok = hipStreamCreateWithFlags(&cap.s[made], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&cap.fork[made], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&cap.done[made], hipEventDisableTiming) == hipSuccess;
  int rc = ok ? LSB_OK : fail(LSB_EDEVICE, "stream or event creation failed");
  for (int k = 0; k < 2 && rc == LSB_OK; ++k) {
    const int p = r->cur;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      rc = fail(LSB_EDEVICE, "graph capture failed to start");
      break;
    }
    launch_steps<LAT>(r, 1, cs, &cap);
    if (hipStreamEndCapture(cs, &graph) != hipSuccess || !graph) {
      rc = fail(LSB_EDEVICE, "graph capture failed");
      break;
    }
    if (hipGraphInstantiate(&r->gexec[p], graph, nullptr, nullptr, 0) != hipSuccess) {
      r->gexec[p] = nullptr;
      rc = fail(LSB_EDEVICE, "graph instantiation failed");
    }
    (void)hipGraphDestroy(graph);
    r->after_cur[p] = r->cur;
    for (int b = 0; b < kMaxGrids; ++b) r->after_dcur[p][b] = r->dcur[b];
  }
  (void)hipStreamDestroy(cs);
  for (int k = 0; k < made; ++k) {
    if (cap.s[k]) (void)hipStreamDestroy(cap.s[k]);
    if (cap.fork[k]) (void)hipEventDestroy(cap.fork[k]);
    if (cap.done[k]) (void)hipEventDestroy(cap.done[k]);
  }
  bool back = r->cur == cur0;
  for (int b = 0; b < kMaxGrids; ++b) back = back && r->dcur[b] == dcur0[b];
  restore();
  if (rc != LSB_OK || !back || !r->gexec[0] || !r->gexec[1]) {
    drop_graphs(r);
    return rc != LSB_OK ? rc : fail(LSB_EDEVICE, "graph capture did not return to the starting state");
  }
  r->graphs_ready = true;
  return LSB_OK;
}

// nsteps coarse steps: graph launches, or plain launches when graphs are off
template <int LAT>
int run_steps(lsb_ref* r, int nsteps, hipStream_t st) {
  if (!r->use_graphs) {
    launch_steps<LAT>(r, nsteps, st);
    return check_launch();
  }
  if (!r->graphs_ready)
    if (int e = build_graphs<LAT>(r)) return e;
  for (int s = 0; s < nsteps; ++s) {
    const int p = r->cur;
    if (hipGraphLaunch(r->gexec[p], st) != hipSuccess) return fail(LSB_EDEVICE, "graph launch failed");
    r->cur = r->after_cur[p];
    for (int b = 0; b < kMaxGrids; ++b) r->dcur[b] = r->after_dcur[p][b];
  }
  return LSB_OK;
}

// the sensor's reduction: the bounding box of the tagged coarse nodes (lo x,
// y, z then hi x, y, z); *tagged false when none is
int sensor_bbox(lsb_ref* r, const double* phi, double d_ref, hipStream_t st, int* box, bool* tagged) {
  const RefArgs& a = r->base;
  k_ref_sensor<<<kSensorBlocks, 256, 0, st>>>(a, phi, d_ref, r->sens);
  k_ref_sensor_final<<<1, 256, 0, st>>>(kSensorBlocks, 1, 1, r->sens, r->sens + 6 * kMaxSeeds * kSensorBlocks);
  if (int e = check_launch()) return e;
  if (hipMemcpyAsync(box, r->sens + 6 * kMaxSeeds * kSensorBlocks, 6 * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(LSB_EDEVICE, "sensor read-back failed");
  *tagged = box[0] < a.nx;
  return LSB_OK;
}

// level 1's box from the tagged box: grown by margin, clamped one node
// inside the grid, at least two cells per axis; the current patch when
// nothing is tagged
void level1_box(const lsb_ref* r, const int* box, bool tagged, int margin, int* patch) {
  const RefArgs& a = r->base;
  const int cur[6] = {a.ia, a.ib, a.ja, a.jb, a.ka, a.kb};
  if (!tagged) {
    for (int d = 0; d < 6; ++d) patch[d] = cur[d];
    return;
  }
  const int n[3] = {a.nx, a.ny, a.nz};
  int out[6] = {0, 0, 0, 0, 0, 0};
  for (int d = 0; d < a.D; ++d) {
    int lo = box[d] - margin, hi = box[3 + d] + margin;
    if (lo < 1) lo = 1;
    if (hi > n[d] - 2) hi = n[d] - 2;
    while (hi - lo < 2) {  // at least two cells (n >= 5 holds: the grid took a valid patch)
      if (hi < n[d] - 2) ++hi;
      else --lo;
    }
    out[2 * d] = lo;
    out[2 * d + 1] = hi;
  }
  for (int d = 0; d < 6; ++d) patch[d] = out[d];
}

// re-meshing of every box onto boxes (6 ints per box, in the parent's node
// coordinates), box 1 first, each inside its re-meshed parent (the shape of
// a chain or tree stays)
int remesh_levels(lsb_ref* r, const int* boxes, hipStream_t st) {
  drop_graphs(r);
  const RefArgs& b = r->base;
  const int D = b.D;
  int last[kMaxGrids][3] = {};  // each grid's last node index per axis, after the re-mesh
  last[0][0] = b.nx - 1;
  last[0][1] = b.ny - 1;
  last[0][2] = b.nz - 1;
  for (int l = 1; l < r->L; ++l) {
    const int* bx = boxes + 6 * (l - 1);
    const int* cap = l == 1 ? r->ext : r->dext[l];
    const int p = r->par[l];
    for (int d = 0; d < D; ++d) {
      const int lo = bx[2 * d], hi = bx[2 * d + 1];
      if (lo < 1 || hi > last[p][d] - 1 || hi - lo < 2)
        return fail(LSB_EINVAL, "a box must lie inside its parent with one node to spare and span >= 2 cells per axis");
      if (hi - lo > cap[d]) return fail(LSB_EINVAL, "box larger than the workspace's maximum extents");
    }
    for (int o = 1; o < l; ++o) {
      if (r->par[o] != p) continue;
      const int* w = boxes + 6 * (o - 1);
      bool apart = false;
      for (int d = 0; d < D; ++d) apart = apart || bx[2 * d + 1] + 2 <= w[2 * d] || w[2 * d + 1] + 2 <= bx[2 * d];
      if (!apart) return fail(LSB_EINVAL, "boxes refining one grid must be at least one node apart");
    }
    for (int d = 0; d < D; ++d) last[l][d] = 2 * (bx[2 * d + 1] - bx[2 * d]);
  }
  RefArgs O[kMaxGrids], A[kMaxGrids];
  for (int l = 1; l < r->L; ++l) O[l] = pair_of(r, l);
  int shift[kMaxGrids][3] = {};  // how far box l's parent's first node moved, in box l's spacing
  for (int l = 1; l < r->L; ++l) {
    const int p = r->par[l];
    A[l] = O[l];
    if (p == 0) set_parent_root(A[l], r->base);
    else set_parent(A[l], A[p]);
    set_patch(A[l], boxes + 6 * (l - 1));
    A[l].fc_in = p == 0 ? r->fc[r->cur] : (p == 1 ? r->ff[0] : r->dff[p][0]);
    if (p != 0) {
      shift[l][0] = 2 * (shift[p][0] + 2 * (A[p].ia - O[p].ia));
      shift[l][1] = 2 * (shift[p][1] + 2 * (A[p].ja - O[p].ja));
      shift[l][2] = 2 * (shift[p][2] + 2 * (A[p].ka - O[p].ka));
    }
    double** buf = l == 1 ? r->ff : r->dff[l];
    double* g = gbuf(r, l, 0);
    const int* sh = shift[l];
    const long n1 = (long)(A[l].mx + 1) * (A[l].my + 1) * (A[l].mz + 1), nbox = (long)A[l].bw * A[l].bh * A[l].bd;
    switch (r->P.lattice) {
      case LSB_D2Q9:
        k_ref_remesh_fine<LSB_D2Q9><<<grid_for(n1), 256, 0, st>>>(A[l], O[l], sh[0], sh[1], sh[2], buf[0], buf[1]);
        k_ref_remesh_g<LSB_D2Q9><<<grid_for(nbox), 256, 0, st>>>(A[l], g);
        break;
      case LSB_D3Q19:
        k_ref_remesh_fine<LSB_D3Q19><<<grid_for(n1), 256, 0, st>>>(A[l], O[l], sh[0], sh[1], sh[2], buf[0], buf[1]);
        k_ref_remesh_g<LSB_D3Q19><<<grid_for(nbox), 256, 0, st>>>(A[l], g);
        break;
      default:
        k_ref_remesh_fine<LSB_D3Q27><<<grid_for(n1), 256, 0, st>>>(A[l], O[l], sh[0], sh[1], sh[2], buf[0], buf[1]);
        k_ref_remesh_g<LSB_D3Q27><<<grid_for(nbox), 256, 0, st>>>(A[l], g);
        break;
    }
    if (int e = check_launch()) return e;
    double* t = buf[0];
    buf[0] = buf[1];
    buf[1] = t;
  }
  for (int l = 1; l < r->L; ++l) {
    A[l].fc_in = nullptr;
    if (l == 1) r->base = A[l];
    else r->deep[l] = A[l];
  }
  for (int d = 0; d < 6; ++d) r->P.patch[d] = D == 3 || d < 4 ? boxes[d] : 0;
  if (r->chain)  // the parameter block describes chains only
    for (int l = 2; l < r->L && l < LSB_REF_MAX_LEVELS; ++l)
      for (int d = 0; d < 6; ++d) r->P.inner[l - 2][d] = D == 3 || d < 4 ? boxes[6 * (l - 1) + d] : 0;
  return LSB_OK;
}


// Validates a tree of boxes and creates the handle.  Box 1 takes P's grid,
// tau_c and max_extent; with inner_caps, box b >= 2 (a chain) is sized by
// P->max_inner_extent[b - 2], else by its own extent.
int create_tree(const lsb_ref_params* P, int nbox, const int* parents, const int* boxes, bool inner_caps,
                lsb_ref** out) {
  *out = nullptr;
  if (P->lattice != LSB_D2Q9 && P->lattice != LSB_D3Q19 && P->lattice != LSB_D3Q27)
    return fail(LSB_EINVAL, "unknown lattice");
  if (nbox < 1 || nbox > LSB_REF_MAX_BOXES) return fail(LSB_EINVAL, "1 .. LSB_REF_MAX_BOXES boxes");
  if (parents[0] != 0) return fail(LSB_EINVAL, "box 1 must refine the coarse grid");
  const bool three = P->lattice != LSB_D2Q9;
  const int dims = three ? 3 : 2;
  const int nx = P->nx, ny = P->ny, nz = three ? P->nz : 1;
  const int* b1 = boxes;
  const int ia = b1[0], ib = b1[1], ja = b1[2], jb = b1[3];
  const int ka = three ? b1[4] : 0, kb = three ? b1[5] : 0;
  if (nx < 4 || ny < 4 || (three && nz < 4) || (!three && P->nz != 1))
    return fail(LSB_EINVAL, "coarse grid must be at least 4 nodes per axis (nz = 1 in 2D)");
  if (ia < 1 || ib > nx - 2 || ib - ia < 2 || ja < 1 || jb > ny - 2 || jb - ja < 2 ||
      (three && (ka < 1 || kb > nz - 2 || kb - ka < 2)))
    return fail(LSB_EINVAL, "patch must lie inside the coarse grid with one node to spare and span >= 2 cells per axis");
  if (!(P->tau_c > 0.5)) return fail(LSB_EINVAL, "tau_c must exceed 1/2");
  if ((long)nx * ny * nz > (1L << 31)) return fail(LSB_EINVAL, "grid too large");
  int ext[3] = {ib - ia, jb - ja, three ? kb - ka : 0};
  for (int d = 0; d < dims; ++d) {
    const int n = d == 0 ? nx : (d == 1 ? ny : nz);
    if (P->max_extent[d] < 0 || P->max_extent[d] > n - 3) return fail(LSB_EINVAL, "max_extent outside [0, n - 3]");
    if (P->max_extent[d] > ext[d]) ext[d] = P->max_extent[d];
  }
  const long cap = (long)row_pitch(2 * ext[0]) * (2L * ext[1] + 3) * (three ? 2L * ext[2] + 3 : 1);
  if (cap > (1L << 31)) return fail(LSB_EINVAL, "grid too large");
  lsb_ref* r = new lsb_ref();
  r->P = *P;
  r->Q = q_of(P->lattice);
  for (int d = 0; d < 3; ++d) r->ext[d] = ext[d];
  r->fcap = cap;
  r->bcap = 2L * (ext[1] + 1) * (ext[2] + 1) + 2L * (ext[0] + 1) * (ext[2] + 1) +
            (three ? 2L * (ext[0] + 1) * (ext[1] + 1) : 0L);
  RefArgs& a = r->base;
  a = RefArgs{};
  a.D = three ? 3 : 2;
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  a.nc = (long)nx * ny * nz;
  a.tc = P->tau_c;
  a.tf = 2.0 * P->tau_c - 0.5;
  a.pw = nx;
  a.ph = ny;
  a.po = 0;
  set_patch(a, b1);
  r->L = nbox + 1;
  r->par[1] = 0;
  auto refuse = [&](const char* msg) {
    delete r;
    return fail(LSB_EINVAL, msg);
  };
  int nkids[kMaxGrids] = {};
  nkids[0] = 1;
  for (int l = 2; l < r->L; ++l) {
    const int p = parents[l - 1];
    if (p < 0 || p >= l) return refuse("a box's parent must be the coarse grid or an earlier box");
    if (++nkids[p] > kMaxKids) return refuse("too many boxes refine one grid");
    r->par[l] = p;
    if (p != l - 1) r->chain = false;
    const int* bx = boxes + 6 * (l - 1);
    int m[3];
    if (p == 0) {
      m[0] = nx - 1;
      m[1] = ny - 1;
      m[2] = nz - 1;
    } else {
      const RefArgs& pp = pair_of(r, p);
      m[0] = pp.mx;
      m[1] = pp.my;
      m[2] = pp.mz;
    }
    for (int d = 0; d < dims; ++d)
      if (bx[2 * d] < 1 || bx[2 * d + 1] > m[d] - 1 || bx[2 * d + 1] - bx[2 * d] < 2)
        return refuse("an inner patch must lie inside its parent with one node to spare and span >= 2 cells per axis");
    // siblings at least one parent node apart on some axis
    for (int o = 1; o < l; ++o) {
      if (r->par[o] != p) continue;
      const RefArgs& w = pair_of(r, o);
      const int wl[3] = {w.ia, w.ja, w.ka}, wh[3] = {w.ib, w.jb, w.kb};
      bool apart = false;
      for (int d = 0; d < dims; ++d) apart = apart || bx[2 * d + 1] + 2 <= wl[d] || wh[d] + 2 <= bx[2 * d];
      if (!apart) return refuse("boxes refining one grid must be at least one node apart");
    }
    RefArgs& c = r->deep[l];
    c = RefArgs{};
    c.D = a.D;
    if (p == 0) set_parent_root(c, a);
    else set_parent(c, pair_of(r, p));
    set_patch(c, bx);
    // capacity: the larger of the box and max_inner_extent (chains), at most
    // what the parent's capacity admits
    int* e = r->dext[l];
    for (int d = 0; d < 3; ++d) e[d] = d < dims ? bx[2 * d + 1] - bx[2 * d] : 0;
    if (inner_caps) {
      const int* pe = p == 1 ? r->ext : r->dext[p];
      for (int d = 0; d < dims; ++d) {
        const int mx = P->max_inner_extent[l - 2][d];
        if (mx < 0 || mx > 2 * pe[d] - 2)
          return refuse("max_inner_extent outside [0, twice the parent's largest extent - 2]");
        if (mx > e[d]) e[d] = mx;
      }
    }
    r->dcap[l] = (long)row_pitch(2 * e[0]) * (2L * e[1] + 3) * (three ? 2L * e[2] + 3 : 1);
    r->dbcap[l] = 2L * (e[1] + 1) * (e[2] + 1) + 2L * (e[0] + 1) * (e[2] + 1) + (three ? 2L * (e[0] + 1) * (e[1] + 1) : 0L);
    if (r->dcap[l] > (1L << 31)) return refuse("grid too large");
  }
  *out = r;
  return LSB_OK;
}

}  // namespace

extern "C" {

int lsb_ref_create_tree(const lsb_ref_params* P, int nbox, const int* parents, const int* boxes, lsb_ref** out) {
  if (!P || !out || !parents || !boxes) return fail(LSB_EINVAL, "null pointer");
  return create_tree(P, nbox, parents, boxes, false, out);
}

int lsb_ref_create(const lsb_ref_params* P, lsb_ref** out) {
  if (!P || !out) return fail(LSB_EINVAL, "null pointer");
  *out = nullptr;
  const int L = P->levels == 0 ? 2 : P->levels;
  if (L < 2 || L > LSB_REF_MAX_LEVELS) return fail(LSB_EINVAL, "levels must be 2 .. LSB_REF_MAX_LEVELS");
  int parents[LSB_REF_MAX_LEVELS], boxes[6 * LSB_REF_MAX_LEVELS];
  for (int b = 1; b < L; ++b) {
    parents[b - 1] = b - 1;
    for (int d = 0; d < 6; ++d) boxes[6 * (b - 1) + d] = b == 1 ? P->patch[d] : P->inner[b - 2][d];
  }
  return create_tree(P, L - 1, parents, boxes, true, out);
}

void lsb_ref_destroy(lsb_ref* r) { delete r; }

int lsb_ref_workspace_bytes(const lsb_ref* r, size_t* bytes) {
  if (!r || !bytes) return fail(LSB_EINVAL, "null pointer");
  size_t a, b, c;
  *bytes = sizes(r, &a, &b, &c);
  return LSB_OK;
}

int lsb_ref_bind(lsb_ref* r, void* ws, size_t bytes) {
  if (!r || !ws) return fail(LSB_EINVAL, "null pointer");
  size_t fcb, ffb, gb;
  if (bytes < sizes(r, &fcb, &ffb, &gb)) return fail(LSB_ENOMEM, "workspace too small");
  char* p = static_cast<char*>(ws);
  for (int k = 0; k < 2; ++k) {
    r->fc[k] = reinterpret_cast<double*>(p);
    p += fcb;
    r->ff[k] = reinterpret_cast<double*>(p);
    p += ffb;
    r->g[k] = reinterpret_cast<double*>(p);
    p += gb;
  }
  r->sens = reinterpret_cast<int*>(p);
  p += align256(sizeof(int) * 6 * kMaxSeeds * (kSensorBlocks + 1));
  for (int l = 2; l < r->L; ++l)
    for (int k = 0; k < 2; ++k) {
      r->dff[l][k] = reinterpret_cast<double*>(p);
      p += align256(sizeof(double) * r->Q * (size_t)r->dcap[l]);
      r->dg[l][k] = reinterpret_cast<double*>(p);
      p += align256(sizeof(double) * r->Q * (size_t)r->dbcap[l]);
    }
  r->ws = static_cast<char*>(ws);
  r->ws_bytes = bytes;
  drop_graphs(r);
  r->inited = false;
  return LSB_OK;
}

int lsb_ref_init_levels(lsb_ref* r, const double* const* rho, const double* const* u, void* stream) {
  if (!r || !rho || !u) return fail(LSB_EINVAL, "null pointer");
  for (int l = 0; l < r->L; ++l)
    if (!rho[l] || !u[l]) return fail(LSB_EINVAL, "null pointer");
  if (!r->ws) return fail(LSB_ESTATE, "lsb_ref_init before lsb_ref_bind");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  r->cur = 0;
  for (int l = 0; l < kMaxGrids; ++l) r->dcur[l] = 0;
  drop_graphs(r);
  switch (r->P.lattice) {
    case LSB_D2Q9: launch_init<LSB_D2Q9>(r, rho, u, st); break;
    case LSB_D3Q19: launch_init<LSB_D3Q19>(r, rho, u, st); break;
    default: launch_init<LSB_D3Q27>(r, rho, u, st); break;
  }
  if (int e = check_launch()) return e;
  r->inited = true;
  return LSB_OK;
}

int lsb_ref_init(lsb_ref* r, const double* rho_c, const double* u_c, const double* rho_f, const double* u_f,
                 void* stream) {
  if (!r || !rho_c || !u_c || !rho_f || !u_f) return fail(LSB_EINVAL, "null pointer");
  if (r->L != 2) return fail(LSB_EINVAL, "lsb_ref_init takes two levels; use lsb_ref_init_levels");
  const double* rho[2] = {rho_c, rho_f};
  const double* u[2] = {u_c, u_f};
  return lsb_ref_init_levels(r, rho, u, stream);
}

int lsb_ref_step(lsb_ref* r, int nsteps, void* stream) {
  if (!r) return fail(LSB_EINVAL, "null pointer");
  if (!r->inited) return fail(LSB_ESTATE, "lsb_ref_step before lsb_ref_init");
  if (nsteps < 0) return fail(LSB_EINVAL, "negative step count");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  switch (r->P.lattice) {
    case LSB_D2Q9: return run_steps<LSB_D2Q9>(r, nsteps, st);
    case LSB_D3Q19: return run_steps<LSB_D3Q19>(r, nsteps, st);
    default: return run_steps<LSB_D3Q27>(r, nsteps, st);
  }
}

int lsb_ref_set_graphs(lsb_ref* r, int on) {
  if (!r) return fail(LSB_EINVAL, "null pointer");
  r->use_graphs = on != 0;
  if (!r->use_graphs) drop_graphs(r);
  return LSB_OK;
}

int lsb_ref_get_populations(lsb_ref* r, double* coarse, double* fine, void* stream) {
  if (!r) return fail(LSB_EINVAL, "null pointer");
  if (!r->inited) return fail(LSB_ESTATE, "lsb_ref_get_populations before lsb_ref_init");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (coarse && hipMemcpyAsync(coarse, r->fc[r->cur], sizeof(double) * r->Q * (size_t)r->base.nc,
                               hipMemcpyDeviceToDevice, st) != hipSuccess)
    return fail(LSB_EDEVICE, "copy of the coarse populations failed");
  if (fine) {
    const RefArgs& b = r->base;
    const long n1 = (long)(b.mx + 1) * (b.my + 1) * (b.mz + 1);
    k_ref_unpad<<<grid_for(r->Q * n1), 256, 0, st>>>(b, r->Q, r->ff[0], fine);
    if (int e = check_launch()) return e;
  }
  return LSB_OK;
}

int lsb_ref_get_level(lsb_ref* r, int level, double* out, void* stream) {
  if (!r || !out) return fail(LSB_EINVAL, "null pointer");
  if (level < 0 || level >= r->L) return fail(LSB_EINVAL, "level outside [0, levels)");
  if (!r->inited) return fail(LSB_ESTATE, "lsb_ref_get_level before lsb_ref_init");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (level == 0) return lsb_ref_get_populations(r, out, nullptr, stream);
  const RefArgs& a = pair_of(r, level);
  const long n1 = (long)(a.mx + 1) * (a.my + 1) * (a.mz + 1);
  k_ref_unpad<<<grid_for(r->Q * n1), 256, 0, st>>>(a, r->Q, level == 1 ? r->ff[0] : r->dff[level][0], out);
  return check_launch();
}

int lsb_ref_sensor(lsb_ref* r, const double* phi, double d_ref, int margin, int* patch, void* stream) {
  if (!r || !phi || !patch) return fail(LSB_EINVAL, "null pointer");
  if (!r->ws) return fail(LSB_ESTATE, "lsb_ref_sensor before lsb_ref_bind");
  if (margin < 0) return fail(LSB_EINVAL, "negative margin");
  int box[6];
  bool tagged = false;
  if (int e = sensor_bbox(r, phi, d_ref, reinterpret_cast<hipStream_t>(stream), box, &tagged)) return e;
  level1_box(r, box, tagged, margin, patch);
  return LSB_OK;
}

int lsb_ref_sensor_seeded(lsb_ref* r, const double* phi, double d_ref, int margin, int nseeds, const int* seeds,
                          int* boxes, int* nboxes, void* stream) {
  if (!r || !phi || !seeds || !boxes || !nboxes) return fail(LSB_EINVAL, "null pointer");
  if (!r->ws) return fail(LSB_ESTATE, "lsb_ref_sensor_seeded before lsb_ref_bind");
  if (margin < 0) return fail(LSB_EINVAL, "negative margin");
  if (nseeds < 1 || nseeds > kMaxSeeds) return fail(LSB_EINVAL, "1 .. LSB_REF_MAX_BOXES seeds");
  const RefArgs& a = r->base;
  const int n[3] = {a.nx, a.ny, a.nz};
  Seeds sd{};
  sd.n = nseeds;
  for (int k = 0; k < nseeds; ++k)
    for (int d = 0; d < 3; ++d) sd.p[k][d] = d < a.D ? seeds[3 * k + d] : 0;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int* out = r->sens + 6 * kMaxSeeds * kSensorBlocks;
  k_ref_sensor_seeded<<<kSensorBlocks, 256, 0, st>>>(a, phi, d_ref, sd, r->sens);
  k_ref_sensor_final<<<1, 256, 0, st>>>(kSensorBlocks, nseeds, kMaxSeeds, r->sens, out);
  if (int e = check_launch()) return e;
  int bb[kMaxSeeds][6];
  if (hipMemcpyAsync(bb, out, sizeof(int) * 6 * nseeds, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(LSB_EDEVICE, "sensor read-back failed");
  // one box per seed with tagged nodes, grown, clamped one node inside the
  // grid, at least two cells per axis
  int nb = 0;
  int bx[kMaxSeeds][6];
  for (int k = 0; k < nseeds; ++k) {
    if (bb[k][0] >= a.nx) continue;  // no node of this seed
    for (int d = 0; d < 6; ++d) bx[nb][d] = 0;
    for (int d = 0; d < a.D; ++d) {
      int lo = bb[k][d] - margin, hi = bb[k][3 + d] + margin;
      if (lo < 1) lo = 1;
      if (hi > n[d] - 2) hi = n[d] - 2;
      while (hi - lo < 2) {
        if (hi < n[d] - 2) ++hi;
        else --lo;
      }
      bx[nb][2 * d] = lo;
      bx[nb][2 * d + 1] = hi;
    }
    ++nb;
  }
  // boxes closer than one node apart merge into their union (in the earlier
  // one's place) until every pair is apart
  for (bool merged = true; merged;) {
    merged = false;
    for (int i = 0; i < nb && !merged; ++i)
      for (int j = i + 1; j < nb && !merged; ++j) {
        bool apart = false;
        for (int d = 0; d < a.D; ++d) apart = apart || bx[i][2 * d + 1] + 2 <= bx[j][2 * d] || bx[j][2 * d + 1] + 2 <= bx[i][2 * d];
        if (apart) continue;
        for (int d = 0; d < a.D; ++d) {
          bx[i][2 * d] = std::min(bx[i][2 * d], bx[j][2 * d]);
          bx[i][2 * d + 1] = std::max(bx[i][2 * d + 1], bx[j][2 * d + 1]);
        }
        for (int m = j; m + 1 < nb; ++m)
          for (int d = 0; d < 6; ++d) bx[m][d] = bx[m + 1][d];
        --nb;
        merged = true;
      }
  }
  for (int k = 0; k < nb; ++k)
    for (int d = 0; d < 6; ++d) boxes[6 * k + d] = bx[k][d];
  *nboxes = nb;
  return LSB_OK;
}

int lsb_ref_sensor_levels(lsb_ref* r, const double* phi, double d_ref, const int* margins, int* boxes,
                          void* stream) {
  if (!r || !phi || !margins || !boxes) return fail(LSB_EINVAL, "null pointer");
  if (!r->ws) return fail(LSB_ESTATE, "lsb_ref_sensor_levels before lsb_ref_bind");
  if (!r->chain) return fail(LSB_EINVAL, "the sensor's boxes need a chain of nested levels, not a tree");
  for (int l = 1; l < r->L; ++l)
    if (margins[l - 1] < 0) return fail(LSB_EINVAL, "negative margin");
  int box[6];
  bool tagged = false;
  if (int e = sensor_bbox(r, phi, d_ref, reinterpret_cast<hipStream_t>(stream), box, &tagged)) return e;
  if (!tagged) {  // nothing tagged: every level stays
    for (int l = 1; l < r->L; ++l) {
      const RefArgs& a = pair_of(r, l);
      const int cur[6] = {a.ia, a.ib, a.ja, a.jb, a.ka, a.kb};
      for (int d = 0; d < 6; ++d) boxes[6 * (l - 1) + d] = cur[d];
    }
    return LSB_OK;
  }
  level1_box(r, box, true, margins[0], boxes);
  // deeper levels: the tagged box grown by the level's margin, in the
  // parent's node coordinates (coarse X -> parent node scale X - org)
  const int D = r->base.D;
  long org[3] = {0, 0, 0};
  long scale = 1;
  for (int l = 2; l < r->L; ++l) {
    const int* pb = boxes + 6 * (l - 2);
    int* ob = boxes + 6 * (l - 1);
    scale *= 2;
    for (int d = 0; d < 6; ++d) ob[d] = 0;
    for (int d = 0; d < D; ++d) {
      org[d] = 2 * (org[d] + pb[2 * d]);
      const long last = 2L * (pb[2 * d + 1] - pb[2 * d]);  // the parent's last node
      long lo = scale * (box[d] - margins[l - 1]) - org[d], hi = scale * (box[3 + d] + margins[l - 1]) - org[d];
      if (lo < 1) lo = 1;
      if (hi > last - 1) hi = last - 1;
      while (hi - lo < 2) {  // the parent spans >= 2 cells, so >= 4 of this level's
        if (hi < last - 1) ++hi;
        else --lo;
      }
      ob[2 * d] = (int)lo;
      ob[2 * d + 1] = (int)hi;
    }
  }
  return LSB_OK;
}

int lsb_ref_remesh(lsb_ref* r, const int* patch, void* stream) {
  if (!r || !patch) return fail(LSB_EINVAL, "null pointer");
  if (!r->inited) return fail(LSB_ESTATE, "lsb_ref_remesh before lsb_ref_init");
  if (r->L != 2) return fail(LSB_EINVAL, "re-meshing takes a two-level hierarchy; use lsb_ref_remesh_levels");
  return remesh_levels(r, patch, reinterpret_cast<hipStream_t>(stream));
}

int lsb_ref_remesh_levels(lsb_ref* r, const int* boxes, int nboxes, void* stream) {
  if (!r || !boxes) return fail(LSB_EINVAL, "null pointer");
  if (nboxes != r->L - 1) return fail(LSB_EINVAL, "lsb_ref_remesh_levels: the number of boxes differs from the refined grids");
  if (!r->inited) return fail(LSB_ESTATE, "lsb_ref_remesh_levels before lsb_ref_init");
  return remesh_levels(r, boxes, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
