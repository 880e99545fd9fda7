// refine.hip -- two-level static grid refinement of the lattice Boltzmann
// solver (D2Q9, BGK, FP64, ratio 2) behind the C ABI of lsb_refine.h.
//
// The coupling of the levels follows the approach the paper adopts for its
// refinement jumps (Sec. 2, lattice Boltzmann method): populations missing
// at the jump come from the other level by interpolation in space and time,
// and the collision frequency eq. (omega) is taken per level for a single
// viscosity (tau_f = 2 tau_c - 1/2).  lsb_refine.h states the steps.
//
// Per coarse step, bandwidth-bound FP64 streams (72 B read and 72 B written
// per node update) and one small perimeter launch:
//   k_ref_coarse  pull + BGK on the uncovered coarse nodes; the perimeter
//                 nodes also keep their pre-collision sets (G(t+1));
//   k_ref_edge    per fine perimeter node, the populations whose source lies
//                 outside the patch, from G, stored where the pull reads
//                 them: a one-node ghost ring around the fine arrays;
//   k_ref_fine    pull + BGK on the fine nodes (no branch on the perimeter);
//                 the second sub-step restricts onto the covered coarse
//                 nodes.
// One row segment of 256 nodes per block (x along the lanes), so every
// population plane is read and written in contiguous 2 KB runs; blocks are
// ordered so that each XCD streams a contiguous band of rows.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/lsb_refine.h"

namespace lsb {
void set_error(const std::string& msg);
}

namespace {

constexpr int Q = 9;
// D2Q9 in the paper's ordering, rest direction last
__device__ constexpr int CX[Q] = {-1, 1, 0, 0, -1, -1, 1, 1, 0};
__device__ constexpr int CY[Q] = {0, 0, -1, 1, -1, 1, 1, -1, 0};
__device__ constexpr double WQ[Q] = {1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 4.0 / 9};

struct RefArgs {
  int nx, ny, ia, ib, ja, jb, mx, my;  // fine nodes (mx + 1) x (my + 1)
  int bw;                              // patch box width ib - ia + 1
  int fw;                              // fine row pitch with the ghost ring, mx + 3
  long nc, nf, nb;                     // nodes: coarse, fine (with the ghost ring), patch box
  double tc, tf;
  const double* fc_in;
  double* fc_out;
  const double* ff_in;
  double* ff_out;
  const double* g0;  // coarse pre-collision sets over the patch box, time t
  double* g1;        // time t + 1
};

// Blocks are dispatched round-robin over the 8 XCDs; logical block L of a
// row-major (row, segment) order goes to one XCD's contiguous share, so the
// rows a block pulls from (y - 1, y, y + 1) sit in the same L2.  A bijection
// of [0, nb) for any nb.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned x = b & 7u, k = b >> 3, q = nb >> 3, r = nb & 7u;
  return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ void moments(const double* f, double& rho, double& ux, double& uy) {
  rho = 0.0;
  double mx = 0.0, my = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    rho += f[q];
    mx += CX[q] * f[q];
    my += CY[q] * f[q];
  }
  ux = mx / rho;
  uy = my / rho;
}

// eq. (feq), c_s^2 = 1/3
__device__ __forceinline__ void equilibrium(double rho, double ux, double uy, double* e) {
  const double uu = ux * ux + uy * uy;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double cu = CX[q] * ux + CY[q] * uy;
    e[q] = WQ[q] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

__global__ __launch_bounds__(256) void k_ref_init(RefArgs a, const double* rho_c, const double* u_c,
                                                  const double* rho_f, const double* u_f, double* fc, double* ff,
                                                  double* g0) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  double e[Q];
  if (blockIdx.z == 0) {
    if (x >= a.nx || y >= a.ny) return;
    const long n = (long)y * a.nx + x;
    equilibrium(rho_c[n], u_c[2 * n], u_c[2 * n + 1], e);
#pragma unroll
    for (int q = 0; q < Q; ++q) fc[q * a.nc + n] = e[q];
    const bool inb = x >= a.ia && x <= a.ib && y >= a.ja && y <= a.jb;
    if (inb && (x == a.ia || x == a.ib || y == a.ja || y == a.jb)) {
      const long b = (long)(y - a.ja) * a.bw + (x - a.ia);
#pragma unroll
      for (int q = 0; q < Q; ++q) g0[q * a.nb + b] = e[q];
    }
  } else {
    if (x > a.mx || y > a.my) return;
    const long n = (long)y * (a.mx + 1) + x;
    equilibrium(rho_f[n], u_f[2 * n], u_f[2 * n + 1], e);
    const long p = (long)(y + 1) * a.fw + x + 1;
#pragma unroll
    for (int q = 0; q < Q; ++q) ff[q * a.nf + p] = e[q];
  }
}

// uncovered coarse nodes: pull (periodic), keep the perimeter's pre-collision
// set, collide with tau_c
__global__ __launch_bounds__(256) void k_ref_coarse(RefArgs a, int segs) {
  const int L = (int)xcd_block(blockIdx.x, gridDim.x);
  const int y = L / segs, x = (L - y * segs) * 256 + (int)threadIdx.x;
  if (x >= a.nx) return;
  const bool inb = x >= a.ia && x <= a.ib && y >= a.ja && y <= a.jb;
  if (inb && x > a.ia && x < a.ib && y > a.ja && y < a.jb) return;  // covered: restricted from the fine level
  const int xs[3] = {x + 1 == a.nx ? 0 : x + 1, x, x == 0 ? a.nx - 1 : x - 1};  // source x for c_x = -1, 0, 1
  const int ys[3] = {y + 1 == a.ny ? 0 : y + 1, y, y == 0 ? a.ny - 1 : y - 1};
  double f[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) f[q] = a.fc_in[q * a.nc + (long)ys[CY[q] + 1] * a.nx + xs[CX[q] + 1]];
  if (inb) {
    const long b = (long)(y - a.ja) * a.bw + (x - a.ia);
#pragma unroll
    for (int q = 0; q < Q; ++q) a.g1[q * a.nb + b] = f[q];
  }
  double rho, ux, uy, e[Q];
  moments(f, rho, ux, uy);
  equilibrium(rho, ux, uy, e);
  const long n = (long)y * a.nx + x;
#pragma unroll
  for (int q = 0; q < Q; ++q) a.fc_out[q * a.nc + n] = f[q] - (f[q] - e[q]) / a.tc;
}

// fine perimeter nodes: the populations whose source lies outside the patch
// (time weights wa on G(t), wb on G(t+1)), written into the ghost ring of the
// fine buffer that sub-step reads, where k_ref_fine pulls them from; both
// sub-steps in one launch (the ghost rings are disjoint from what the fine
// steps write, and G(t), G(t+1) are known once the coarse step is done).
// Thread t walks the perimeter: the rows j = 0 and j = my, then the columns
// i = 0 and i = mx.
__global__ __launch_bounds__(256) void k_ref_edge(RefArgs a, double* ff1, double* ff2) {
  // blockIdx.y = 0: sub-step 1 (t + 1/2, into ff1); 1: sub-step 2 (t + 1, into ff2)
  const double wa = blockIdx.y == 0 ? 0.5 : 0.0, wb = blockIdx.y == 0 ? 0.5 : 1.0;
  double* ff = blockIdx.y == 0 ? ff1 : ff2;
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int nr = a.mx + 1, ncol = a.my - 1;
  if (t >= 2 * nr + 2 * ncol) return;
  int i, j;
  if (t < 2 * nr) {
    i = t < nr ? t : t - nr;
    j = t < nr ? 0 : a.my;
  } else {
    const int u = t - 2 * nr;
    i = u < ncol ? 0 : a.mx;
    j = 1 + (u < ncol ? u : u - ncol);
  }
  // the coarse set at this node: one coarse node, or the mean of the two
  // beside an odd node along its edge
  double H[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) H[q] = 0.0;
  auto node = [&](int I, int J, double s) {
    const long b = (long)(J - a.ja) * a.bw + (I - a.ia);
#pragma unroll
    for (int q = 0; q < Q; ++q) H[q] += s * (wa * a.g0[q * a.nb + b] + wb * a.g1[q * a.nb + b]);
  };
  if (!(i & 1) && !(j & 1)) {
    node(a.ia + i / 2, a.ja + j / 2, 1.0);
  } else if (i & 1) {
    node(a.ia + (i - 1) / 2, a.ja + j / 2, 0.5);
    node(a.ia + (i + 1) / 2, a.ja + j / 2, 0.5);
  } else {
    node(a.ia + i / 2, a.ja + (j - 1) / 2, 0.5);
    node(a.ia + i / 2, a.ja + (j + 1) / 2, 0.5);
  }
  double rh, uxh, uyh, eh[Q];
  moments(H, rh, uxh, uyh);
  equilibrium(rh, uxh, uyh, eh);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int si = i - CX[q], sj = j - CY[q];
    if (si < 0 || si > a.mx || sj < 0 || sj > a.my)
      ff[q * a.nf + (long)(sj + 1) * a.fw + si + 1] = eh[q] + a.tf / (2.0 * a.tc) * (H[q] - eh[q]);
  }
}

// fine nodes: pull (the ghost ring holds the perimeter's inward populations),
// collide with tau_f; with restrict_ set, the fine nodes on covered coarse
// nodes write those nodes' post-collision populations
__global__ __launch_bounds__(256) void k_ref_fine(RefArgs a, int segs, int restrict_) {
  const int L = (int)xcd_block(blockIdx.x, gridDim.x);
  const int j = L / segs, i = (L - j * segs) * 256 + (int)threadIdx.x;
  if (i > a.mx) return;
  const long p = (long)(j + 1) * a.fw + i + 1;
  double f[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) f[q] = a.ff_in[q * a.nf + p - CY[q] * a.fw - CX[q]];
  double rho, ux, uy, e[Q];
  moments(f, rho, ux, uy);
  equilibrium(rho, ux, uy, e);
#pragma unroll
  for (int q = 0; q < Q; ++q) a.ff_out[q * a.nf + p] = f[q] - (f[q] - e[q]) / a.tf;
  if (restrict_ && !(i & 1) && !(j & 1)) {
    const int I = a.ia + i / 2, J = a.ja + j / 2;
    if (I > a.ia && I < a.ib && J > a.ja && J < a.jb) {
      const long m = (long)J * a.nx + I;
#pragma unroll
      for (int q = 0; q < Q; ++q) a.fc_out[q * a.nc + m] = e[q] + 2.0 * (a.tc - 1.0) / a.tf * (f[q] - e[q]);
    }
  }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int fail(int code, const std::string& msg) {
  lsb::set_error(msg);
  return code;
}

}  // namespace

struct lsb_ref {
  lsb_ref_params P;
  RefArgs base;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  double* fc[2] = {nullptr, nullptr};
  double* ff[2] = {nullptr, nullptr};
  double* g[2] = {nullptr, nullptr};
  int cur = 0;  // fc[cur] and g[cur] are the current coarse state and G(t); ff[0] the fine state
  bool inited = false;
};

namespace {
size_t sizes(const lsb_ref* r, size_t* fcb, size_t* ffb, size_t* gb) {
  *fcb = align256(sizeof(double) * Q * (size_t)r->base.nc);
  *ffb = align256(sizeof(double) * Q * (size_t)r->base.nf);
  *gb = align256(sizeof(double) * Q * (size_t)r->base.nb);
  return 2 * (*fcb + *ffb + *gb);
}

int check_launch() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LSB_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return LSB_OK;
}
}  // namespace

extern "C" {

int lsb_ref_create(const lsb_ref_params* P, lsb_ref** out) {
  if (!P || !out) return fail(LSB_EINVAL, "null pointer");
  *out = nullptr;
  const int nx = P->nx, ny = P->ny, ia = P->patch[0], ib = P->patch[1], ja = P->patch[2], jb = P->patch[3];
  if (nx < 4 || ny < 4 || ny > 65535) return fail(LSB_EINVAL, "coarse grid must be at least 4 x 4 with ny <= 65535");
  if (ia < 1 || ib > nx - 2 || ib - ia < 2 || ja < 1 || jb > ny - 2 || jb - ja < 2)
    return fail(LSB_EINVAL, "patch must lie inside the coarse grid with one node to spare and span >= 2 cells");
  if (2 * (jb - ja) >= 65535) return fail(LSB_EINVAL, "patch too tall");
  if (!(P->tau_c > 0.5)) return fail(LSB_EINVAL, "tau_c must exceed 1/2");
  lsb_ref* r = new lsb_ref();
  r->P = *P;
  RefArgs& a = r->base;
  a = RefArgs{};
  a.nx = nx;
  a.ny = ny;
  a.ia = ia;
  a.ib = ib;
  a.ja = ja;
  a.jb = jb;
  a.mx = 2 * (ib - ia);
  a.my = 2 * (jb - ja);
  a.bw = ib - ia + 1;
  a.fw = a.mx + 3;
  a.nc = (long)nx * ny;
  a.nf = (long)a.fw * (a.my + 3);
  a.nb = (long)a.bw * (jb - ja + 1);
  a.tc = P->tau_c;
  a.tf = 2.0 * P->tau_c - 0.5;
  *out = r;
  return LSB_OK;
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
  r->ws = static_cast<char*>(ws);
  r->ws_bytes = bytes;
  r->inited = false;
  return LSB_OK;
}

int lsb_ref_init(lsb_ref* r, const double* rho_c, const double* u_c, const double* rho_f, const double* u_f,
                 void* stream) {
  if (!r || !rho_c || !u_c || !rho_f || !u_f) return fail(LSB_EINVAL, "null pointer");
  if (!r->ws) return fail(LSB_ESTATE, "lsb_ref_init before lsb_ref_bind");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const RefArgs& a = r->base;
  const int w = a.nx > a.mx + 1 ? a.nx : a.mx + 1, h = a.ny > a.my + 1 ? a.ny : a.my + 1;
  r->cur = 0;
  k_ref_init<<<dim3((w + 255) / 256, h, 2), 256, 0, st>>>(a, rho_c, u_c, rho_f, u_f, r->fc[0], r->ff[0], r->g[0]);
  if (int e = check_launch()) return e;
  r->inited = true;
  return LSB_OK;
}

int lsb_ref_step(lsb_ref* r, int nsteps, void* stream) {
  if (!r) return fail(LSB_EINVAL, "null pointer");
  if (!r->inited) return fail(LSB_ESTATE, "lsb_ref_step before lsb_ref_init");
  if (nsteps < 0) return fail(LSB_EINVAL, "negative step count");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const RefArgs& b = r->base;
  const int sc = (b.nx + 255) / 256, sf = (b.mx + 1 + 255) / 256;
  const unsigned gc = (unsigned)(sc * b.ny), gf = (unsigned)(sf * (b.my + 1));
  const dim3 ge((unsigned)((2 * (b.mx + 1) + 2 * (b.my - 1) + 255) / 256), 2);
  for (int s = 0; s < nsteps; ++s) {
    RefArgs a = b;
    a.fc_in = r->fc[r->cur];
    a.fc_out = r->fc[r->cur ^ 1];
    a.g0 = r->g[r->cur];
    a.g1 = r->g[r->cur ^ 1];
    k_ref_coarse<<<gc, 256, 0, st>>>(a, sc);
    // inward populations of both fine sub-steps: G halfway in time, then G(t+1)
    k_ref_edge<<<ge, 256, 0, st>>>(a, r->ff[0], r->ff[1]);
    a.ff_in = r->ff[0];
    a.ff_out = r->ff[1];
    k_ref_fine<<<gf, 256, 0, st>>>(a, sf, 0);
    // sub-step 2 also restricts onto the covered coarse nodes
    a.ff_in = r->ff[1];
    a.ff_out = r->ff[0];
    k_ref_fine<<<gf, 256, 0, st>>>(a, sf, 1);
    r->cur ^= 1;
  }
  return check_launch();
}

int lsb_ref_get_populations(lsb_ref* r, double* coarse, double* fine, void* stream) {
  if (!r) return fail(LSB_EINVAL, "null pointer");
  if (!r->inited) return fail(LSB_ESTATE, "lsb_ref_get_populations before lsb_ref_init");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (coarse && hipMemcpyAsync(coarse, r->fc[r->cur], sizeof(double) * Q * (size_t)r->base.nc,
                               hipMemcpyDeviceToDevice, st) != hipSuccess)
    return fail(LSB_EDEVICE, "copy of the coarse populations failed");
  if (fine) {
    // the fine nodes without the ghost ring, plane by plane
    const RefArgs& b = r->base;
    const size_t w = sizeof(double) * (size_t)(b.mx + 1), h = (size_t)(b.my + 1);
    for (int q = 0; q < Q; ++q)
      if (hipMemcpy2DAsync(fine + (size_t)q * (b.mx + 1) * h, w, r->ff[0] + q * b.nf + b.fw + 1,
                           sizeof(double) * (size_t)b.fw, w, h, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(LSB_EDEVICE, "copy of the fine populations failed");
  }
  return LSB_OK;
}

}  // extern "C"
