// kernels.h -- HIP kernels of one time step, templated on the velocity set
// (LAT) and the population storage (ST).  Included by one translation unit
// per velocity set.
//
// Data layout in HBM (structure of arrays, cell index c = (z*ny + y)*nx + x):
//   A[i][c]     populations as deviations from w_i rho_ref of the cell's
//               phase (codec ST; 3D: chunks of 256 cells, [c/256][i][c%256])
//   phi[c]      level set; s1/s2 Runge-Kutta stages; p0 reinit reference
//   tag[c]      bit field (T_* in common.h)
//   M[m][c]     rho, u[3], S[6] of the last collision (LS-active cells)
//   G[m][c]     normal[3], curvature (LS-active cells)
//   ut[a][c]    extension velocity
// The level-set kernels run over a compact list of 32x4x4 (3D) or 16x16 (2D)
// tiles that hold LS-active cells, with a fixed grid that strides over the
// device-resident tile count.
#pragma once

#include <type_traits>

#include "common.h"

namespace lsb {

template <int LAT, int ST>
struct Step {
  using L = Lat<LAT>;
  using C = Codec<ST>;
  using T = typename C::T;
  using R = typename C::R;
  using Args = KArgs<T, R>;
  static constexpr int Q = L::Q;
  static constexpr int D = L::D;
};

// ---------------------------------------------------------------------------
// a2: moments, BGK collision with body force, store; moments to M on active
// cells.  d[] holds the incoming deviations f_i - w_i after streaming and
// bounce-back.  Opposite directions (i, opp(i)) share the even part of the
// equilibrium, w (rho - 1 + rho (9/2 (c.u)^2 - 3/2 u.u)), and flip the sign of
// the odd parts (3 w rho c.u and the force 3 w rho c.a).
// ---------------------------------------------------------------------------
// gas pressure baseline seen by a gas cell: the single baseline, or with
// several bubbles that of the cell's bubble
template <class Args>
__device__ __forceinline__ auto baseline(const Args& a, int c) {
  using R = typename std::remove_pointer<decltype(a.pbc)>::type;
  return a.use_pb == 2 ? a.pbc[c] : (R)a.scal[SC_PB];
}

// ---------------------------------------------------------------------------
// Cumulant collision (Sec. 2.1, D3Q27) with the paper's rates: omega_1 =
// omega_BGK for the shear (deviatoric second-order) cumulants, one for every
// other cumulant.  With those rates the post-collision cumulants of order
// three and more vanish and the second-order ones become
// cs^2 delta + (1 - omega) dev(kappa_2), so the post-collision central
// moments are those of a Gaussian with that covariance (sums over pairings),
// and the populations follow from the central moments by one inverse
// transform per axis (z, then y, then x), each a three-point relation on the
// lines of the 3x3x3 moment array.  Every quantity is carried as its
// deviation from the rest state (populations f - w, central moments minus
// their rest values), so FP32 arithmetic loses nothing to cancellation.
// Index of the moment array: a + 3 b + 9 c for the orders (a, b, c) in
// (x, y, z), or the position (cx + 1) + 3 (cy + 1) + 9 (cz + 1) once all
// three axes are transformed (the code of the direction).
// ---------------------------------------------------------------------------
namespace cum {
__host__ __device__ constexpr double rest_moment(int a) { return a == 0 ? 1.0 : (a == 1 ? 0.0 : 1.0 / 3.0); }
__host__ __device__ constexpr double rest_weight(int slot) { return slot == 1 ? 2.0 / 3.0 : 1.0 / 6.0; }

// One line: (g0, g1, g2) are the deviations of the central moments of
// orders 0, 1, 2 about velocity u (rest values k0r, 0, .); on return they
// are the deviations of the line's values at c = -1, 0, +1.
template <class R>
__device__ __forceinline__ void line(R k0r, R& g0, R& g1, R& g2, R u) {
  const R k0 = k0r + g0;
  const R m1 = g1 + u * k0;
  const R m2 = g2 + u * ((R)2 * g1 + u * k0);
  const R vm = (R)0.5 * (m2 - m1);
  const R vz = g0 - m2;
  const R vp = (R)0.5 * (m2 + m1);
  g0 = vm;
  g1 = vz;
  g2 = vp;
}
}  // namespace cum

// d: incoming deviations (paper order); out: post-collision deviations
// without the body force.
template <class R>
__device__ __forceinline__ void cumulant_collide(const R* d, R om, R* out) {
  using L = Lat<LSB_D3Q27>;
  R rp = 0, jx = 0, jy = 0, jz = 0, sxx = 0, syy = 0, szz = 0, sxy = 0, sxz = 0, syz = 0;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
    const R v = d[i];
    rp += v;
    if (cx) { jx += (R)cx * v; sxx += v; }
    if (cy) { jy += (R)cy * v; syy += v; }
    if (cz) { jz += (R)cz * v; szz += v; }
    if (cx * cy) sxy += (R)(cx * cy) * v;
    if (cx * cz) sxz += (R)(cx * cz) * v;
    if (cy * cz) syz += (R)(cy * cz) * v;
  }
  const R rho = (R)1 + rp;
  const R inv = (R)1 / rho;
  const R ux = jx * inv, uy = jy * inv, uz = jz * inv;
  const R third = (R)(1.0 / 3.0);
  // central second moments per unit density minus cs^2 delta
  const R rp3 = rp * third;
  const R exx = (sxx - rp3) * inv - ux * ux;
  const R eyy = (syy - rp3) * inv - uy * uy;
  const R ezz = (szz - rp3) * inv - uz * uz;
  const R exy = sxy * inv - ux * uy;
  const R exz = sxz * inv - ux * uz;
  const R eyz = syz * inv - uy * uz;
  // post-collision covariance minus cs^2 delta: relaxed deviatoric part
  // (the trace relaxes to cs^2 at rate one)
  const R oc = (R)1 - om;
  const R t3 = (exx + eyy + ezz) * third;
  const R axx = oc * (exx - t3), ayy = oc * (eyy - t3), azz = oc * (ezz - t3);
  const R axy = oc * exy, axz = oc * exz, ayz = oc * eyz;
  // deviations of the central moments (times rho) from the rest values
  R g[27];
#pragma unroll
  for (int m = 0; m < 27; ++m) g[m] = (R)0;
  g[0] = rp;
  g[2] = rp3 + rho * axx;
  g[6] = rp3 + rho * ayy;
  g[18] = rp3 + rho * azz;
  g[1 + 3] = rho * axy;
  g[1 + 9] = rho * axz;
  g[3 + 9] = rho * ayz;
  const R rp9 = rp * (R)(1.0 / 9.0);
  g[2 + 6] = rp9 + rho * ((axx + ayy) * third + axx * ayy + (R)2 * axy * axy);
  g[2 + 18] = rp9 + rho * ((axx + azz) * third + axx * azz + (R)2 * axz * axz);
  g[6 + 18] = rp9 + rho * ((ayy + azz) * third + ayy * azz + (R)2 * ayz * ayz);
  g[2 + 3 + 9] = rho * ((third + axx) * ayz + (R)2 * axy * axz);
  g[1 + 6 + 9] = rho * ((third + ayy) * axz + (R)2 * axy * ayz);
  g[1 + 3 + 18] = rho * ((third + azz) * axy + (R)2 * axz * ayz);
  g[2 + 6 + 18] = rp * (R)(1.0 / 27.0) +
                  rho * ((axx + ayy + azz) * (R)(1.0 / 9.0) + (axx * ayy + axx * azz + ayy * azz) * third +
                         axx * ayy * azz + (R)2 * (third + axx) * ayz * ayz + (R)2 * (third + ayy) * axz * axz +
                         (R)2 * (third + azz) * axy * axy + (R)8 * axy * axz * ayz);
  // inverse transforms: z orders -> z positions, then y, then x
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      cum::line((R)(cum::rest_moment(a) * cum::rest_moment(b)), g[a + 3 * b], g[a + 3 * b + 9], g[a + 3 * b + 18], uz);
#pragma unroll
  for (int zc = 0; zc < 3; ++zc)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      cum::line((R)(cum::rest_moment(a) * cum::rest_weight(zc)), g[a + 9 * zc], g[a + 3 + 9 * zc], g[a + 6 + 9 * zc], uy);
#pragma unroll
  for (int zc = 0; zc < 3; ++zc)
#pragma unroll
    for (int yc = 0; yc < 3; ++yc)
      cum::line((R)(cum::rest_weight(yc) * cum::rest_weight(zc)), g[3 * yc + 9 * zc], g[1 + 3 * yc + 9 * zc],
                g[2 + 3 * yc + 9 * zc], ux);
#pragma unroll
  for (int i = 0; i < 27; ++i) out[i] = g[detail::d3q27_code(i)];
}

// FORCE = false drops the body-force terms (a launch for zero acceleration);
// CUM = false leaves out the cumulant operator (a launch where both phases
// use BGK).
template <int LAT, int ST, bool FORCE = true, bool CUM = true>
__device__ __forceinline__ void collide_store(const typename Step<LAT, ST>::Args& a, int c, int k, bool active,
                                              typename Step<LAT, ST>::R* d) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using L = typename S::L;
  using C = typename S::C;
  constexpr int Q = S::Q;
  // moments from the pair sums and differences of opposite directions
  R rp = 0, m0 = 0, m1 = 0, m2 = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int j = opp<LAT>(i);
    if (j < i) continue;
    if (j == i) {
      rp += d[i];
      continue;
    }
    rp += d[i] + d[j];
    const R df = d[i] - d[j];
    if (L::cx(i) > 0) m0 += df; else if (L::cx(i) < 0) m0 -= df;
    if (L::cy(i) > 0) m1 += df; else if (L::cy(i) < 0) m1 -= df;
    if (L::cz(i) > 0) m2 += df; else if (L::cz(i) < 0) m2 -= df;
  }
  const R rho = sel2(a.rho_ref, k) + rp;  // deviations are carried relative to w rho_ref[k]
  const R inv = (R)1 / rho;
  const R ux = m0 * inv, uy = m1 * inv, uz = m2 * inv;
  const R uu15 = (R)1.5 * (ux * ux + uy * uy + uz * uz);
  const R om = sel2(a.omega, k);
  const R omc = (R)1 - om;
  const R fx = (R)3 * ACC(a, k, 0) * rho, fy = (R)3 * ACC(a, k, 1) * rho, fz = (R)3 * ACC(a, k, 2) * rho;
  const R ux3 = (R)3 * rho * ux, uy3 = (R)3 * rho * uy, uz3 = (R)3 * rho * uz;
  const R s = a.scale;
  const size_t N = a.N;
  const size_t pc = pop_cell<LAT>(c);  // the cell in the population layout
  bool cum_phase = false;
  if constexpr (LAT == LSB_D3Q27 && CUM) cum_phase = sel2(a.cum, k) != 0;
  if (cum_phase) {
    // the cumulant operator takes deviations from the rest state w_i
    const R rm1 = sel2(a.rref_m1, k);
    R da[Q], out[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) da[i] = d[i] + (R)wgt<LAT>(i) * rm1;
    cumulant_collide(da, om, out);
#pragma unroll
    for (int i = 0; i < Q; ++i) out[i] = out[i] - (R)wgt<LAT>(i) * rm1;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      R v = out[i];
      if (FORCE) {
        const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
        R ca = 0;
        if (cx) ca += (R)cx * fx;
        if (cy) ca += (R)cy * fy;
        if (cz) ca += (R)cz * fz;
        v += (R)wgt<LAT>(i) * ca;
      }
      store_pop(a.An + pc + pop_dir<LAT>(i, N), C::enc(v, (R)(1.0 / wgt<LAT>(i)), s));
    }
  } else {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int j = opp<LAT>(i);
    if (j < i) continue;
    const R w = (R)wgt<LAT>(i);
    const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
    R cu = 0, cu3 = 0, ca = 0;
    if (cx) { cu += (R)cx * ux; cu3 += (R)cx * ux3; if (FORCE) ca += (R)cx * fx; }
    if (cy) { cu += (R)cy * uy; cu3 += (R)cy * uy3; if (FORCE) ca += (R)cy * fy; }
    if (cz) { cu += (R)cz * uz; cu3 += (R)cz * uz3; if (FORCE) ca += (R)cz * fz; }
    const R even = w * (rp + rho * ((R)4.5 * cu * cu - uu15));
    if (j == i) {
      const R out = omc * d[i] + om * even;
      store_pop(a.An + pc + pop_dir<LAT>(i, N), C::enc(out, (R)(1.0 / wgt<LAT>(i)), s));
      continue;
    }
    const R odd = w * cu3;
    R out_i = omc * d[i] + om * (even + odd);
    R out_j = omc * d[j] + om * (even - odd);
    if (FORCE) {
      const R fo = w * ca;
      out_i = out_i + fo;
      out_j = out_j - fo;
    }
    store_pop(a.An + pc + pop_dir<LAT>(i, N), C::enc(out_i, (R)(1.0 / wgt<LAT>(i)), s));
    store_pop(a.An + pc + pop_dir<LAT>(j, N), C::enc(out_j, (R)(1.0 / wgt<LAT>(j)), s));
  }
  }
  if (active) {
    // strain rate from the second moment of f - f^eq (pairs: 2 x even part)
    R P0 = 0, P1 = 0, P2 = 0, P3 = 0, P4 = 0, P5 = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int j = opp<LAT>(i);
      if (j <= i) continue;
      const R w = (R)wgt<LAT>(i);
      const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
      R cu = 0;
      if (cx) cu += (R)cx * ux;
      if (cy) cu += (R)cy * uy;
      if (cz) cu += (R)cz * uz;
      const R even = w * (rp + rho * ((R)4.5 * cu * cu - uu15));
      const R fn2 = (d[i] + d[j]) - (R)2 * even;
      if (cx) P0 += fn2;
      if (cy) P1 += fn2;
      if (cz) P2 += fn2;
      if (cx * cy) P3 += (R)(cx * cy) * fn2;
      if (cx * cz) P4 += (R)(cx * cz) * fn2;
      if (cy * cz) P5 += (R)(cy * cz) * fn2;
    }
    const R fac = -(R)1.5 * om * inv;  // -omega / (2 rho cs^2)
    a.Mn[c] = rp + sel2(a.rref_m1, k);  // rho - 1
    a.Mn[N + c] = ux;
    a.Mn[2 * N + c] = uy;
    a.Mn[3 * N + c] = uz;
    a.Mn[4 * N + c] = fac * P0;
    a.Mn[5 * N + c] = fac * P1;
    a.Mn[6 * N + c] = fac * P2;
    a.Mn[7 * N + c] = fac * P3;
    a.Mn[8 * N + c] = fac * P4;
    a.Mn[9 * N + c] = fac * P5;
  }
}

// Reflection of direction i across the crossed axes (mask bit a = axis a).
template <int LAT>
__host__ __device__ constexpr int reflect_dir(int i, int mask) {
  return dir_of<LAT>((mask & 1) ? -Lat<LAT>::cx(i) : Lat<LAT>::cx(i), (mask & 2) ? -Lat<LAT>::cy(i) : Lat<LAT>::cy(i),
                     (mask & 4) ? -Lat<LAT>::cz(i) : Lat<LAT>::cz(i));
}

// a3: incoming deviation for a link whose source lies beyond a wall face.
// Halfway bounce-back with the moving-wall term if any crossed face is
// no-slip; specular reflection otherwise.  check_phase: a reflected source
// in the other phase falls back to plain bounce-back.
template <int LAT, int ST, bool check_phase>
__device__ __forceinline__ typename Step<LAT, ST>::R wall_pull(const typename Step<LAT, ST>::Args& a, int c, int x, int y,
                                                              int z, int i, int k) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using L = typename S::L;
  using C = typename S::C;
  const int cc[3] = {L::cx(i), L::cy(i), L::cz(i)};
  const int pos[3] = {x, y, z};
  const int n[3] = {a.nx, a.ny, a.nz};
  int mask = 0;
  int src[3];
  for (int ax = 0; ax < 3; ++ax) {
    int sv = pos[ax] - cc[ax];
    if (sv >= 0 && sv < n[ax]) { src[ax] = sv; continue; }
    if (sel3(a.per, ax)) { src[ax] = sv < 0 ? sv + n[ax] : sv - n[ax]; continue; }
    mask |= 1 << ax;
    src[ax] = pos[ax];
  }
  const R s = a.scale;
  const int j = opp<LAT>(i);
  const R wj = (R)wgt<LAT>(j);
  // across the face of a refined box: the coarser grid's population
  for (int ax = 0; ax < 3; ++ax)
    if ((mask & (1 << ax)) && sel6(a.bcf, 2 * ax + (pos[ax] - cc[ax] < 0 ? 0 : 1)) == kFaceInject)
      return a.ghost[(size_t)i * a.N + c];
  for (int ax = 0; ax < 3; ++ax) {
    if (!(mask & (1 << ax))) continue;
    const int face = 2 * ax + (pos[ax] - cc[ax] < 0 ? 0 : 1);
    if (sel6(a.bcf, face) == LSB_NOSLIP) {
      const R cu = (R)cc[0] * WALLU(a, face, 0) + (R)cc[1] * WALLU(a, face, 1) + (R)cc[2] * WALLU(a, face, 2);
      return C::dec(a.A[pidx<LAT>(j, c, a.N)], wj, a.inv_scale) + (R)6 * (R)wgt<LAT>(i) * cu;
    }
  }
  const int ir = reflect_dir<LAT>(i, mask);
  const int sc = (src[2] * a.ny + src[1]) * a.nx + src[0];
  if (check_phase && ((a.tag[sc] & T_GAS) != k)) return C::dec(a.A[pidx<LAT>(j, c, a.N)], wj, a.inv_scale);
  const R wr = (R)wgt<LAT>(ir);
  return C::dec(a.A[pidx<LAT>(ir, sc, a.N)], wr, a.inv_scale);
}

// ---------------------------------------------------------------------------
// Tile helpers for the level-set kernels.
// ---------------------------------------------------------------------------
template <int D, class Args>
__device__ __forceinline__ void tile_origin(const Args& a, int t, int& x0, int& y0, int& z0) {
  using TS = TileShape<D>;
  const int tx = t % a.ntile[0];
  const int ty = (t / a.ntile[0]) % a.ntile[1];
  const int tz = t / (a.ntile[0] * a.ntile[1]);
  x0 = tx << TS::SX;
  y0 = ty << TS::SY;
  z0 = tz << TS::SZ;
}

// Loop body over the cells of the listed tiles:  F(c, x, y, z).  Blocks of
// 256 threads; every lane runs the same number of iterations (tile sizes are
// multiples of the block size).
template <int D, class Args, class F>
__device__ __forceinline__ void for_tile_cells(const Args& a, const int* list, int count, F&& f) {
  using TS = TileShape<D>;
  constexpr int tcells = TS::X * TS::Y * TS::Z;
  static_assert(tcells % 256 == 0, "tile sizes are multiples of the block size");
  for (int e = blockIdx.x; e < count; e += gridDim.x) {
    int x0, y0, z0;
    // one tile per block: its origin is scalar arithmetic
    tile_origin<D>(a, __builtin_amdgcn_readfirstlane(list[e]), x0, y0, z0);
#pragma unroll
    for (int l = threadIdx.x; l < tcells; l += 256) {
      const int x = x0 + (l & (TS::X - 1));
      const int y = y0 + ((l >> TS::SX) & (TS::Y - 1));
      const int z = z0 + (l >> (TS::SX + TS::SY));
      if (x >= a.nx || y >= a.ny || z >= a.nz) continue;
      f((z * a.ny + y) * a.nx + x, x, y, z);
    }
  }
}

// The wall rule's source of link i at a cell on the x face that the link
// crosses (face 0 for c_x = +1, face 1 for c_x = -1), as an element offset
// into the populations: the own cell's opposite population at a no-slip
// face, the mirrored direction (-c_x, c_y, c_z) at the cell's own x in the
// source row (mirror_cell: element offset of (x, y - c_y, z - c_z)) at a
// free-slip face.
template <int LAT, class Args>
__device__ __forceinline__ size_t xwall_source(const Args& a, int i, int c, size_t mirror_cell) {
  using L = Lat<LAT>;
  const int face = L::cx(i) > 0 ? 0 : 1;
  if (sel6(a.bcf, face) == LSB_NOSLIP) return pop_dir<LAT>(opp<LAT>(i), a.N) + pop_cell<LAT>(c);
  return pop_dir<LAT>(dir_of<LAT>(-L::cx(i), L::cy(i), L::cz(i)), a.N) + mirror_cell;
}
// ... and the moving-wall term added at a no-slip face (zero at a free-slip
// one), 6 w_i (c_i . u_wall) as in wall_pull.
template <int LAT, class R, class Args>
__device__ __forceinline__ R xwall_term(const Args& a, int i) {
  using L = Lat<LAT>;
  const int face = L::cx(i) > 0 ? 0 : 1;
  if (sel6(a.bcf, face) != LSB_NOSLIP) return (R)0;
  const R cu = (R)L::cx(i) * WALLU(a, face, 0) + (R)L::cy(i) * WALLU(a, face, 1) + (R)L::cz(i) * WALLU(a, face, 2);
  return (R)6 * (R)wgt<LAT>(i) * cu;
}

// ---------------------------------------------------------------------------
// a2 for one cell with no lattice link to the other phase or through a wall:
// branch-free gather (per-direction base pointer plus a 32-bit cell offset).
// XW (3D grids with wall faces in x): cells tagged T_XWALL, whose only
// links through a wall cross an x face, are taken here too (every cell on
// an x face that reaches this point is one: the others are on the wall or
// interface lists).  On a link crossing the face the lane loads the wall
// rule's source instead (halfway bounce-back: the own cell's opposite
// population, plus the moving-wall term; free slip: the mirrored direction
// at (x, y - c_y, z - c_z)), so the gather stays one load per direction
// without divergence, and the rows stay coalesced, which the wall list
// cannot do for x faces (stride of a row).  The expressions are those of
// wall_pull.
// ---------------------------------------------------------------------------
template <int LAT, int ST, bool FORCE = true, bool CUM = true, bool XW = false>
__device__ __forceinline__ void fast_cell(const typename Step<LAT, ST>::Args& a, int c, int x, int y, int z, uint8_t t) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using T = typename S::T;
  using L = typename S::L;
  using C = typename S::C;
  constexpr int Q = S::Q;
  // source coordinate x - c for c = -1, 0, +1 (periodic wrap; no wall is crossed)
  const int xs[3] = {x + 1 == a.nx ? 0 : x + 1, x, x == 0 ? a.nx - 1 : x - 1};
  const int ys[3] = {y + 1 == a.ny ? 0 : y + 1, y, y == 0 ? a.ny - 1 : y - 1};
  const int zs[3] = {z + 1 == a.nz ? 0 : z + 1, z, z == 0 ? a.nz - 1 : z - 1};
  const R is = a.inv_scale;
  R d[Q];
  int rowoff[3][3];
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) rowoff[dz][dy] = (zs[dz] * a.ny + ys[dy]) * a.nx;
  // uniform per-direction base plus a per-lane offset of the source cell
  // (one array per direction: a 32-bit byte offset; chunked layout: the
  // chunk and position of the source cell)
  if constexpr (LAT == LSB_D2Q9) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int sc = rowoff[L::cz(i) + 1][L::cy(i) + 1] + xs[L::cx(i) + 1];
      const char* __restrict__ Ai = reinterpret_cast<const char*>(a.A + (size_t)i * a.N);
      d[i] = C::dec(*reinterpret_cast<const T*>(Ai + (unsigned)sc * (unsigned)sizeof(T)), (R)wgt<LAT>(i), is);
    }
  } else if ((a.nx & 255) == 0) {
    // rows start at chunk boundaries: a source cell's offset is its row's
    // chunk base plus the chunk offset of its x (9 + 3 terms, one add each)
    size_t rb[3][3], xo[3];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) rb[dz][dy] = (size_t)(rowoff[dz][dy] >> 8) * (size_t)(Q << 8);
#pragma unroll
    for (int k = 0; k < 3; ++k) xo[k] = pop_cell<LAT>(xs[k]);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if constexpr (XW) {
        if (L::cx(i) != 0) {
          const size_t off = pop_dir<LAT>(i, a.N) + rb[L::cz(i) + 1][L::cy(i) + 1] + xo[L::cx(i) + 1];
          const size_t woff = xwall_source<LAT>(a, i, c, rb[L::cz(i) + 1][L::cy(i) + 1] + xo[1]);
          const bool cross = L::cx(i) > 0 ? x == 0 : x == a.nx - 1;
          d[i] = C::dec(a.A[cross ? woff : off], (R)wgt<LAT>(i), is) + (cross ? xwall_term<LAT, R>(a, i) : (R)0);
          continue;
        }
      }
      const T* __restrict__ Ai = a.A + pop_dir<LAT>(i, a.N);
      d[i] = C::dec(Ai[rb[L::cz(i) + 1][L::cy(i) + 1] + xo[L::cx(i) + 1]], (R)wgt<LAT>(i), is);
    }
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int sc = rowoff[L::cz(i) + 1][L::cy(i) + 1] + xs[L::cx(i) + 1];
      if constexpr (XW && LAT != LSB_D2Q9) {
        if (L::cx(i) != 0) {
          const size_t off = pop_dir<LAT>(i, a.N) + pop_cell<LAT>(sc);
          const size_t woff = xwall_source<LAT>(a, i, c, pop_cell<LAT>(rowoff[L::cz(i) + 1][L::cy(i) + 1] + x));
          const bool cross = L::cx(i) > 0 ? x == 0 : x == a.nx - 1;
          d[i] = C::dec(a.A[cross ? woff : off], (R)wgt<LAT>(i), is) + (cross ? xwall_term<LAT, R>(a, i) : (R)0);
          continue;
        }
      }
      const T* __restrict__ Ai = a.A + pop_dir<LAT>(i, a.N);
      d[i] = C::dec(Ai[pop_cell<LAT>(sc)], (R)wgt<LAT>(i), is);
    }
  }
  collide_store<LAT, ST, FORCE, CUM>(a, c, t & T_GAS, (t & T_ACT) != 0, d);
}

// a2/a3 for a wall-adjacent cell with no lattice link to the other phase.
template <int LAT, int ST, bool CUM = true>
__device__ __forceinline__ void wall_cell(const typename Step<LAT, ST>::Args& a, int c, int x, int y, int z, uint8_t t) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using L = typename S::L;
  using C = typename S::C;
  constexpr int Q = S::Q;
  const int k = t & T_GAS;
  const int xs[3] = {lb_coord(x + 1, a.nx, a.per[0]), x, lb_coord(x - 1, a.nx, a.per[0])};
  const int ys[3] = {lb_coord(y + 1, a.ny, a.per[1]), y, lb_coord(y - 1, a.ny, a.per[1])};
  const int zs[3] = {lb_coord(z + 1, a.nz, a.per[2]), z, lb_coord(z - 1, a.nz, a.per[2])};
  const R is = a.inv_scale;
  R d[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int sx = xs[L::cx(i) + 1], sy = ys[L::cy(i) + 1], sz = zs[L::cz(i) + 1];
    if ((sx | sy | sz) >= 0) {
      d[i] = C::dec(a.A[pidx<LAT>(i, (sz * a.ny + sy) * a.nx + sx, a.N)], (R)wgt<LAT>(i), is);
    } else {
      d[i] = wall_pull<LAT, ST, false>(a, c, x, y, z, i, k);
    }
  }
  collide_store<LAT, ST, true, CUM>(a, c, k, (t & T_ACT) != 0, d);
}

// Tile of a cell.
template <int D, class Args>
__device__ __forceinline__ int tile_of(const Args& a, int x, int y, int z) {
  using TS = TileShape<D>;
  const int tz = D == 3 ? (z >> TS::SZ) : 0;
  return (tz * a.ntile[1] + (y >> TS::SY)) * a.ntile[0] + (x >> TS::SX);
}

// Bulk part of the collide-stream: one thread per cell, 256-cell blocks along
// x, XCD-aware block order.  Skips interface-adjacent cells (k_lb_iface) and
// wall-adjacent cells (k_lb_wall).  With SPLIT it also skips the candidate
// tiles of the previous step's classification (k_lb_band takes them): they
// hold every LS-active cell and, by more than one lattice link, every cell
// the interface or refill kernels update, so this part writes no moments and
// reads nothing the level-set chain writes except the LS-active bit of tags
// (masked).  It may run concurrently with the level-set chain.
// xchunks > 0: blocks of 256 cells of one x-row (nx a multiple of 256);
// xchunks == 0: blocks of 256 consecutive cells across rows (any nx, no idle
// threads at the row ends).
template <int LAT, int ST, bool SPLIT, bool FORCE, bool CUM, bool XW = false>
__global__ __launch_bounds__(256, (XW && sizeof(typename Step<LAT, ST>::R) == 4) ? 7 : 1) void k_lb_bulk(
    const typename Step<LAT, ST>::Args a, int xchunks) {
  // Block order (MI355X hands out consecutive workgroups round-robin over
  // its 8 XCDs).  Two-byte storage: dispatch order, so that the XCDs stream
  // neighbouring rows together: 2.51-2.52 against 2.60-2.62 ms per FP16
  // launch at 512^3 with each XCD given a contiguous range of rows, 2.67-2.78
  // ms with tiles of rows.  FP32 and FP64: each XCD a contiguous range
  // (5.08 against 5.35 ms, 9.58 against 10.61 ms).
  const unsigned b = sizeof(typename Step<LAT, ST>::T) == 2 ? blockIdx.x : remap_xcd(blockIdx.x, gridDim.x);
  int c, x, y, z;
  if (xchunks > 0) {
    const int row = (int)(b / (unsigned)xchunks);
    x = (int)(b - (unsigned)row * xchunks) * 256 + (int)threadIdx.x;
    if (x >= a.nx) return;
    y = row % a.ny;
    z = row / a.ny;
    c = row * a.nx + x;
  } else {
    c = (int)(b * 256u + threadIdx.x);
    if (c >= a.N) return;
    const int row = c / a.nx;
    x = c - row * a.nx;
    y = row % a.ny;
    z = row / a.ny;
  }
  if (SPLIT && a.cand_prev[tile_of<Step<LAT, ST>::D>(a, x, y, z)]) return;
  const uint8_t t = a.tag[c];
  if (t & (T_SPEC | T_WALL)) return;
  fast_cell<LAT, ST, FORCE, CUM, XW>(a, c, x, y, z, SPLIT ? (uint8_t)(t & ~T_ACT) : t);
}

// Band part of the collide-stream: the non-interface, non-wall cells of the
// candidate tiles of the previous step's classification (a superset of the
// LS-active tiles; the moments of LS-active cells feed the level-set kernels
// of the same step).
template <int LAT, int ST, bool CUM, bool XW = false>
__global__ __launch_bounds__(256) void k_lb_band(const typename Step<LAT, ST>::Args a) {
  for_tile_cells<Step<LAT, ST>::D>(a, a.cand_list, a.counters[CNT_CAND], [&](int c, int x, int y, int z) {
    const uint8_t t = a.tag[c];
    if (t & (T_SPEC | T_WALL)) return;
    fast_cell<LAT, ST, true, CUM, XW>(a, c, x, y, z, t);
  });
}

// The two wall planes of no-slip z faces when x and y are periodic and rows
// are whole 256-cell chunks (3D): streamed like the bulk, one 256-cell row
// chunk per block, with halfway bounce-back plus the moving-wall term on the
// links through the face (the pulls of k_lb_wall's wall_pull for this case).
// Skips interface-adjacent cells (k_lb_iface takes their wall links).
template <int LAT, int ST, bool FORCE, bool CUM>
__global__ __launch_bounds__(256) void k_lb_zwall(const typename Step<LAT, ST>::Args a, int xchunks) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using T = typename S::T;
  using L = typename S::L;
  using C = typename S::C;
  constexpr int Q = S::Q;
  const unsigned b = remap_xcd(blockIdx.x, gridDim.x);
  const int row = (int)(b / (unsigned)xchunks);  // 0 .. 2 ny - 1: bottom plane, then top
  const int x = (int)(b - (unsigned)row * xchunks) * 256 + (int)threadIdx.x;
  const bool top = row >= a.ny;
  const int y = top ? row - a.ny : row;
  const int z = top ? a.nz - 1 : 0;
  const int c = (z * a.ny + y) * a.nx + x;
  const uint8_t t = a.tag[c];
  if (t & T_SPEC) return;
  const int face = top ? 5 : 4;
  const R uw[3] = {WALLU(a, face, 0), WALLU(a, face, 1), WALLU(a, face, 2)};
  const int xs[3] = {x + 1 == a.nx ? 0 : x + 1, x, x == 0 ? a.nx - 1 : x - 1};
  const int ys[3] = {y + 1 == a.ny ? 0 : y + 1, y, y == 0 ? a.ny - 1 : y - 1};
  const int zs[3] = {z + 1, z, z - 1};  // the one beyond the face is not read
  const R is = a.inv_scale;
  R d[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int cz = L::cz(i);
    // through the face: the source z - cz lies outside [0, nz)
    const bool wall = top ? (cz < 0) : (cz > 0);
    const int src = wall ? c : (zs[cz + 1] * a.ny + ys[L::cy(i) + 1]) * a.nx + xs[L::cx(i) + 1];
    const int dir = wall ? opp<LAT>(i) : i;
    const T v = a.A[pop_dir<LAT>(dir, a.N) + pop_cell<LAT>(src)];
    R di = C::dec(v, (R)wgt<LAT>(i), is);
    if (wall) di += (R)6 * (R)wgt<LAT>(i) * ((R)L::cx(i) * uw[0] + (R)L::cy(i) * uw[1] + (R)cz * uw[2]);
    d[i] = di;
  }
  collide_store<LAT, ST, FORCE, CUM>(a, c, t & T_GAS, (t & T_ACT) != 0, d);
}

// Wall-adjacent cells (static list), except interface-adjacent ones.
template <int LAT, int ST, bool CUM>
__global__ __launch_bounds__(256) void k_lb_wall(const typename Step<LAT, ST>::Args a) {
  const ListSpan sp = xcd_list_span(a.counters[CNT_WALL]);
  for (int e = sp.e; e < sp.end; e += sp.stride) {
    const int c = a.wall_list[e];
    const uint8_t t = a.tag[c];
    if (t & T_SPEC) continue;
    const int x = c % a.nx, y = (c / a.nx) % a.ny, z = c / (a.nx * a.ny);
    wall_cell<LAT, ST, CUM>(a, c, x, y, z, t);
  }
}

// Marks wall-adjacent cells (a link leaves through a wall face) and lists them.
// Every lane of a wavefront runs the same iterations except in the last,
// where the lanes past N have left the loop (wave_append ballots the active
// lanes only).
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_mark_walls(const typename Step<LAT, ST>::Args a) {
  for (int c = blockIdx.x * 256 + threadIdx.x; c < a.N; c += gridDim.x * 256) {
    const int x = c % a.nx, y = (c / a.nx) % a.ny, z = c / (a.nx * a.ny);
    const bool wx = !a.per[0] && (x == 0 || x == a.nx - 1);
    const bool wy = !a.per[1] && (y == 0 || y == a.ny - 1);
    const bool wz = !a.per[2] && (z == 0 || z == a.nz - 1);
    // 3D cells with wall links through x faces only are left to the bulk
    // kernel (T_XWALL; see fast_cell), the others are listed; the x faces of
    // a refined box's level read its ghost array and stay on the list
    const bool xonly = LAT != LSB_D2Q9 && wx && !wy && !wz && sel6(a.bcf, x == 0 ? 0 : 1) != kFaceInject;
    const bool wall = (wx || wy || wz) && !xonly;
    a.tag[c] = (uint8_t)((a.tag[c] & ~(T_WALL | T_XWALL)) | (wall ? T_WALL : 0) | (xonly ? T_XWALL : 0));
    // one append per wavefront, lanes in cell order: the list comes in runs
    // of consecutive cells, which the wall kernel reads coalesced
    const int slot = wave_append(&a.counters[CNT_WALL], wall);
    if (wall) a.wall_list[slot] = c;
  }
}

// ---------------------------------------------------------------------------
// a4: interface bounce-back (eq:bb with the momentum term eq:bb_cc and the
// stress jump eq:Sdecomp).  Own cell c (phase k) pulls direction i from the
// other-phase cell sc = c - c_i.  Deviation form: all weights of the
// interpolation sum to one, so the rest state cancels.  Runtime direction
// index (constant-memory tables).
// ---------------------------------------------------------------------------
template <class R>
struct OwnCell {   // level set, previous moments and geometry of the own cell
  R phi, M[10], G[4];
};

// Interface record of a cell: phi, M[0..9], G[0..3] and a pad, one aligned
// 16-value slot per cell (written for the interface-adjacent cells only).
template <class R>
struct alignas(16 * sizeof(R) > 64 ? 64 : 16 * sizeof(R)) IfaceRec {
  R v[16];
};

template <class Args>
__device__ __forceinline__ auto load_rec(const Args& a, int c) {
  using R = typename std::remove_pointer<decltype(a.irec)>::type;
  return *reinterpret_cast<const IfaceRec<R>*>(a.irec + (size_t)16 * c);
}

// Operands of the bounce-back on one cut link (direction i, source sc in the
// other phase), loaded before any of them is used so that the loads of
// several links are in flight together.  The forward neighbour's tag and
// population are loaded whatever q turns out to be.
template <int LAT, int ST>
struct CutLink {
  using R = typename Step<LAT, ST>::R;
  using T = typename Step<LAT, ST>::T;
  IfaceRec<R> rs;  // phi, M, G of the other-phase cell
  R pb;            // gas baseline (one, or that of the gas endpoint's bubble)
  T dj, di, djf;   // stored populations: own cell at j and i, forward neighbour at j
  uint8_t ftag;    // forward neighbour's tag (T_WALL when it lies beyond a wall face)
};

template <int LAT, int ST>
__device__ __forceinline__ CutLink<LAT, ST> cut_fetch(const typename Step<LAT, ST>::Args& a, int c, int x, int y,
                                                      int z, int sc, int i, int k) {
  const size_t N = a.N;
  const int j = tab<LAT>.opp[i];
  CutLink<LAT, ST> L;
  L.rs = load_rec(a, sc);
  L.pb = (typename Step<LAT, ST>::R)a.scal[SC_PB];
  if (a.use_pb == 2) L.pb = a.pbc[k == 1 ? c : sc];
  L.dj = a.A[pidx<LAT>(j, c, N)];
  L.di = a.A[pidx<LAT>(i, c, N)];
  const int fx = lb_coord(x + tab<LAT>.cx[i], a.nx, a.per[0]);
  const int fy = lb_coord(y + tab<LAT>.cy[i], a.ny, a.per[1]);
  const int fz = lb_coord(z + tab<LAT>.cz[i], a.nz, a.per[2]);
  L.ftag = T_WALL;
  L.djf = L.dj;
  if ((fx | fy | fz) >= 0) {
    const int fc = (fz * a.ny + fy) * a.nx + fx;
    L.ftag = a.tag[fc] & T_GAS;
    L.djf = a.A[pidx<LAT>(j, fc, N)];
  }
  return L;
}

// Interface bounce-back with the stress jump for one cut link, from its
// fetched operands.
template <int LAT, int ST>
__device__ __forceinline__ typename Step<LAT, ST>::R cut_eval(const typename Step<LAT, ST>::Args& a,
                                                               const OwnCell<typename Step<LAT, ST>::R>& own,
                                                               const CutLink<LAT, ST>& L, int i, int k) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using C = typename S::C;
  const int cc[3] = {tab<LAT>.cx[i], tab<LAT>.cy[i], tab<LAT>.cz[i]};
  const R w = tw<LAT, R>(i);
  const IfaceRec<R>& rs = L.rs;
  const R px = own.phi, py = rs.v[0];
  const R q = px / (px - py);
  // interface velocity (linear interpolation of the previous moments)
  R uG[3], nG[3];
  for (int m = 0; m < 3; ++m) uG[m] = ((R)1 - q) * own.M[1 + m] + q * rs.v[2 + m];
  R nn = 0;
  for (int m = 0; m < 3; ++m) {
    nG[m] = ((R)1 - q) * own.G[m] + q * rs.v[11 + m];
    nn += nG[m] * nG[m];
  }
  const R nl = sqrt(nn);
  if (nl > (R)1e-30) {
    const R inl = (R)1 / nl;
    for (int m = 0; m < 3; ++m) nG[m] = nG[m] * inl;
  }
  const R kG = ((R)1 - q) * own.G[3] + q * rs.v[14];
  const int o = 1 - k;
  const R pb = L.pb;
  R p_own = sel2(a.iface_pc, k) * own.M[0] + (k == 1 ? pb : (R)0);
  R p_oth = sel2(a.iface_pc, o) * rs.v[1] + (o == 1 ? pb : (R)0);
  for (int m = 0; m < 3; ++m) {
    p_own = p_own + sel2(a.rho_phys, k) * ACC(a, k, m) * (R)(-cc[m]) * q;
    p_oth = p_oth + sel2(a.rho_phys, o) * ACC(a, o, m) * (R)cc[m] * ((R)1 - q);
  }
  const R p_l = (k == 0) ? p_own : p_oth;
  const R p_g = (k == 0) ? p_oth : p_own;
  // pressure part of the normal jump: divisor 2 eta_p with eta_p the mean
  // viscosity, raised to rho_max cs^2 / 4 where the mean viscosity is below
  // rho_max / 24, so that the lagged explicit pressure feedback has gain
  // k <= 1 (constants of the argument block)
  const R E = ((p_g - p_l) + a.sigma * kG) * a.iface_inv2etap;
  R Sb[6];
  for (int m = 0; m < 6; ++m) Sb[m] = (R)0.5 * (own.M[4 + m] + rs.v[5 + m]);
  const R acoef = a.iface_acoef;
  const R Sm[3][3] = {{Sb[0], Sb[3], Sb[4]}, {Sb[3], Sb[1], Sb[5]}, {Sb[4], Sb[5], Sb[2]}};
  const R cn = (R)cc[0] * nG[0] + (R)cc[1] * nG[1] + (R)cc[2] * nG[2];
  R nAn = 0, nAc = 0;
  for (int p = 0; p < 3; ++p)
    for (int r = 0; r < 3; ++r) {
      nAn = nAn + acoef * nG[p] * Sm[p][r] * nG[r];
      nAc = nAc + acoef * nG[p] * Sm[p][r] * (R)cc[r];
    }
  const R cSc = cn * cn * E + (R)2 * cn * nAc - cn * cn * nAn;
  const R s_own = (k == 0) ? (R)1 : (R)-1;
  const R cu = (R)cc[0] * uG[0] + (R)cc[1] * uG[1] + (R)cc[2] * uG[2];
  const R W = (R)6 * w * (cu + q * ((R)1 - q) * s_own * cSc);
  const R dj = C::dec(L.dj, w, a.inv_scale);
  if (q < (R)0.5) {
    if (L.ftag == k) {
      const R djf = C::dec(L.djf, w, a.inv_scale);
      return (R)2 * q * dj + ((R)1 - (R)2 * q) * djf + W;
    }
    return dj + W;
  }
  const R di = C::dec(L.di, w, a.inv_scale);
  const R i2q = (R)1 / ((R)2 * q);
  return dj * i2q + ((R)2 * q - (R)1) * i2q * di + W * i2q;
}

template <int LAT, int ST>
__device__ __forceinline__ typename Step<LAT, ST>::R iface_pull(const typename Step<LAT, ST>::Args& a,
                                                                  const OwnCell<typename Step<LAT, ST>::R>& own, int c,
                                                                  int x, int y, int z, int sc, int i, int k) {
  return cut_eval<LAT, ST>(a, own, cut_fetch<LAT, ST>(a, c, x, y, z, sc, i, k), i, k);
}

// Incoming deviation of direction i (runtime index) for an interface-adjacent
// cell: plain streaming, wall rule or interface bounce-back.
template <int LAT, int ST>
__device__ __forceinline__ typename Step<LAT, ST>::R pull_general(const typename Step<LAT, ST>::Args& a,
                                                                    const OwnCell<typename Step<LAT, ST>::R>& own, int c,
                                                                    int x, int y, int z, int i, int k) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using C = typename S::C;
  const R s = a.scale;
  const int cx = tab<LAT>.cx[i], cy = tab<LAT>.cy[i], cz = tab<LAT>.cz[i];
  const int sx = lb_coord(x - cx, a.nx, a.per[0]);
  const int sy = lb_coord(y - cy, a.ny, a.per[1]);
  const int sz = lb_coord(z - cz, a.nz, a.per[2]);
  const R w = tw<LAT, R>(i);
  if ((sx | sy | sz) < 0) {
    // a3 at an interface-adjacent cell: halfway bounce-back for any crossed
    // no-slip face, else specular reflection (bounce-back if the reflected
    // source lies in the other phase)
    const int pos[3] = {x, y, z};
    const int cc[3] = {cx, cy, cz};
    const int n[3] = {a.nx, a.ny, a.nz};
    const int sv3[3] = {sx, sy, sz};
    int src[3];
    int rc[3];
    const int j = tab<LAT>.opp[i];
    for (int ax = 0; ax < 3; ++ax) {
      src[ax] = sv3[ax] < 0 ? pos[ax] : sv3[ax];
      rc[ax] = sv3[ax] < 0 ? -cc[ax] : cc[ax];
    }
    for (int ax = 0; ax < 3; ++ax)
      if (sv3[ax] < 0 && sel6(a.bcf, 2 * ax + (pos[ax] - cc[ax] < 0 ? 0 : 1)) == kFaceInject)
        return a.ghost[(size_t)i * a.N + c];
    for (int ax = 0; ax < 3; ++ax) {
      if (sv3[ax] >= 0) continue;
      const int face = 2 * ax + (pos[ax] - cc[ax] < 0 ? 0 : 1);
      if (sel6(a.bcf, face) == LSB_NOSLIP) {
        const R cu = (R)cc[0] * WALLU(a, face, 0) + (R)cc[1] * WALLU(a, face, 1) + (R)cc[2] * WALLU(a, face, 2);
        return C::dec(a.A[pidx<LAT>(j, c, a.N)], w, a.inv_scale) + (R)6 * w * cu;
      }
    }
    const int sc = (src[2] * a.ny + src[1]) * a.nx + src[0];
    if ((a.tag[sc] & T_GAS) != k) return C::dec(a.A[pidx<LAT>(j, c, a.N)], w, a.inv_scale);
    int ir = 0;
    for (int m = 0; m < S::Q; ++m)
      if (tab<LAT>.cx[m] == rc[0] && tab<LAT>.cy[m] == rc[1] && tab<LAT>.cz[m] == rc[2]) ir = m;
    return C::dec(a.A[pidx<LAT>(ir, sc, a.N)], w, a.inv_scale);
  }
  const int sc = (sz * a.ny + sy) * a.nx + sx;
  if ((a.tag[sc] & T_GAS) == k) return C::dec(a.A[pidx<LAT>(i, sc, a.N)], w, a.inv_scale);
  return iface_pull<LAT, ST>(a, own, c, x, y, z, sc, i, k);
}

// a2-a4 for the listed interface-adjacent cells, in two parts: the gather
// of the incoming populations into LDS (column col of fl) and the collision.
// G lanes share a cell (G = 1 or 4): lane sub gathers the directions
// i = sub (mod G) and stores their post-collision populations; every lane
// sums the moments over all directions from LDS in the same order, so the
// result does not depend on G.
template <int LAT, int ST, int G>
__device__ __forceinline__ void iface_gather(const typename Step<LAT, ST>::Args& a,
                                             const OwnCell<typename Step<LAT, ST>::R>& own, int c, int x, int y,
                                             int z, int k, int sub, typename Step<LAT, ST>::R* fl, int col) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using C = typename S::C;
  using L = typename S::L;
  using T = typename S::T;
  constexpr int Q = S::Q;
  const size_t N = a.N;
  // pass 1 (directions unrolled, all loads issued together): plain
  // streaming from own-phase sources; cut links and links through a wall
  // face are marked
  unsigned cut = 0u, wall = 0u;
  {
    const R is = a.inv_scale;
    // source coordinate x - c for c = -1, 0, +1 (-1 beyond a wall face)
    const int xs[3] = {lb_coord(x + 1, a.nx, a.per[0]), x, lb_coord(x - 1, a.nx, a.per[0])};
    const int ys[3] = {lb_coord(y + 1, a.ny, a.per[1]), y, lb_coord(y - 1, a.ny, a.per[1])};
    const int zs[3] = {lb_coord(z + 1, a.nz, a.per[2]), z, lb_coord(z - 1, a.nz, a.per[2])};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (G > 1 && (i & (G - 1)) != sub) continue;
      const int sx = xs[L::cx(i) + 1], sy = ys[L::cy(i) + 1], sz = zs[L::cz(i) + 1];
      if ((sx | sy | sz) < 0) {
        wall |= 1u << i;
        continue;
      }
      const int sc = (sz * a.ny + sy) * a.nx + sx;
      const uint8_t ts = a.tag[sc];
      const T v = a.A[pidx<LAT>(i, sc, N)];
      if ((ts & T_GAS) != k) {
        cut |= 1u << i;
        continue;
      }
      fl[i * 256 + col] = C::dec(v, (R)wgt<LAT>(i), is);
    }
  }
  // pass 2: interface bounce-back on the cut links, one at a time (fewer
  // live registers: with FP32 arithmetic the kernel runs at five
  // wavefronts per SIMD, which hides more of the links' load latency than
  // two links in flight per thread did; measured 175 us against 205 us
  // at 512^3)
  while (cut) {
    const int i0 = __ffs(cut) - 1;
    cut &= cut - 1u;
    const int sx = lb_coord(x - tab<LAT>.cx[i0], a.nx, a.per[0]);
    const int sy = lb_coord(y - tab<LAT>.cy[i0], a.ny, a.per[1]);
    const int sz = lb_coord(z - tab<LAT>.cz[i0], a.nz, a.per[2]);
    const CutLink<LAT, ST> L0 = cut_fetch<LAT, ST>(a, c, x, y, z, (sz * a.ny + sy) * a.nx + sx, i0, k);
    fl[i0 * 256 + col] = cut_eval<LAT, ST>(a, own, L0, i0, k);
  }
  // pass 3: links through a wall face
  while (wall) {
    const int i = __ffs(wall) - 1;
    wall &= wall - 1u;
    fl[i * 256 + col] = pull_general<LAT, ST>(a, own, c, x, y, z, i, k);
  }
}

template <int LAT, int ST, bool CUM, int G>
__device__ __forceinline__ void iface_collide(const typename Step<LAT, ST>::Args& a, int c, int k, bool active,
                                              int sub, const typename Step<LAT, ST>::R* fl, int col) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using C = typename S::C;
  constexpr int Q = S::Q;
  const size_t N = a.N;
  const R s = a.scale;
  R rp = 0, m0 = 0, m1 = 0, m2 = 0;
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    const R f = fl[i * 256 + col];
    rp += f;
    m0 += (R)tab<LAT>.cx[i] * f;
    m1 += (R)tab<LAT>.cy[i] * f;
    m2 += (R)tab<LAT>.cz[i] * f;
  }
  const R rho = sel2(a.rho_ref, k) + rp;  // deviations relative to w rho_ref[k]
  const R inv = (R)1 / rho;
  const R ux = m0 * inv, uy = m1 * inv, uz = m2 * inv;
  const R uu = ux * ux + uy * uy + uz * uz;
  const R om = sel2(a.omega, k);
  const R fx = (R)3 * ACC(a, k, 0), fy = (R)3 * ACC(a, k, 1), fz = (R)3 * ACC(a, k, 2);
  bool cum_phase = false;
  if constexpr (LAT == LSB_D3Q27 && CUM) cum_phase = sel2(a.cum, k) != 0;
  // strain-rate moments of the incoming populations (lane 0 of the cell's
  // group); BGK stores here
  const bool lead = sub == 0;
  R P0 = 0, P1 = 0, P2 = 0, P3 = 0, P4 = 0, P5 = 0;
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    const bool mine = G == 1 || (i & (G - 1)) == sub;
    if (!lead && !mine) continue;
    const R f = fl[i * 256 + col];
    const R w = tw<LAT, R>(i);
    const R cx = (R)tab<LAT>.cx[i], cy = (R)tab<LAT>.cy[i], cz = (R)tab<LAT>.cz[i];
    const R cu = cx * ux + cy * uy + cz * uz;
    const R deq = w * (rp + rho * ((R)3 * cu + (R)4.5 * cu * cu - (R)1.5 * uu));
    const R fn = f - deq;
    P0 += cx * cx * fn; P1 += cy * cy * fn; P2 += cz * cz * fn;
    P3 += cx * cy * fn; P4 += cx * cz * fn; P5 += cy * cz * fn;
    if (cum_phase || !mine) continue;
    const R ca = cx * fx + cy * fy + cz * fz;
    store_pop(&a.An[pidx<LAT>(i, c, N)], C::enc(f - om * fn + w * rho * ca, twinv<LAT, R>(i), s));
  }
  if constexpr (LAT == LSB_D3Q27 && CUM) {
    if (cum_phase && lead) {
      // the cumulant operator takes deviations from the rest state w_i
      const R rm1 = sel2(a.rref_m1, k);
      R dl[Q], out[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) dl[i] = fl[i * 256 + col] + (R)wgt<LAT>(i) * rm1;
      cumulant_collide(dl, om, out);
#pragma unroll
      for (int i = 0; i < Q; ++i) out[i] = out[i] - (R)wgt<LAT>(i) * rm1;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        using L = typename S::L;
        R ca = 0;
        if (L::cx(i)) ca += (R)L::cx(i) * fx;
        if (L::cy(i)) ca += (R)L::cy(i) * fy;
        if (L::cz(i)) ca += (R)L::cz(i) * fz;
        store_pop(&a.An[pidx<LAT>(i, c, N)], C::enc(out[i] + (R)wgt<LAT>(i) * rho * ca, (R)(1.0 / wgt<LAT>(i)), s));
      }
    }
  }
  if (active && lead) {
    const R fac = -(R)1.5 * om * inv;
    a.Mn[c] = rp + sel2(a.rref_m1, k);  // rho - 1
    a.Mn[N + c] = ux;
    a.Mn[2 * N + c] = uy;
    a.Mn[3 * N + c] = uz;
    a.Mn[4 * N + c] = fac * P0;
    a.Mn[5 * N + c] = fac * P1;
    a.Mn[6 * N + c] = fac * P2;
    a.Mn[7 * N + c] = fac * P3;
    a.Mn[8 * N + c] = fac * P4;
    a.Mn[9 * N + c] = fac * P5;
  }
}

template <int LAT, int ST>
__device__ __forceinline__ void iface_cell(const typename Step<LAT, ST>::Args& a, int c, int& x, int& y, int& z,
                                           int& k, bool& active, OwnCell<typename Step<LAT, ST>::R>& own) {
  x = c % a.nx;
  y = (c / a.nx) % a.ny;
  z = c / (a.nx * a.ny);
  const uint8_t t = a.tag[c];
  k = t & T_GAS;
  active = (t & T_ACT) != 0;
  const IfaceRec<typename Step<LAT, ST>::R> ro = load_rec(a, c);
  own.phi = ro.v[0];
#pragma unroll
  for (int m = 0; m < 10; ++m) own.M[m] = ro.v[1 + m];
#pragma unroll
  for (int m = 0; m < 4; ++m) own.G[m] = ro.v[11 + m];
}

// G lanes per cell, 256 / G cells per block and pass, the list split over
// the XCDs as in xcd_list_span; every lane of a block runs the same passes
// (the gather and the collision meet at a block barrier).
template <int LAT, int ST, bool CUM, int G>
__device__ __forceinline__ void iface_grouped(const typename Step<LAT, ST>::Args& a, int n,
                                              typename Step<LAT, ST>::R* fl) {
  constexpr int CPB = 256 / G;
  const int col = (int)threadIdx.x / G, sub = (int)threadIdx.x & (G - 1);
  int lo = 0, end = n, first = (int)blockIdx.x * CPB, stride = (int)gridDim.x * CPB;
  if ((gridDim.x & 7u) == 0u) {
    const int per = (n + 7) >> 3;
    lo = (int)(blockIdx.x & 7u) * per;
    end = min(n, lo + per);
    first = lo + (int)(blockIdx.x >> 3) * CPB;
    stride = (int)(gridDim.x >> 3) * CPB;
  }
  for (int base = first; base < end; base += stride) {
    const int e = base + col;
    const bool valid = e < end;
    int c = 0, x = 0, y = 0, z = 0, k = 0;
    bool active = false;
    OwnCell<typename Step<LAT, ST>::R> own;
    if (valid) {
      c = a.spec_list[e];
      iface_cell<LAT, ST>(a, c, x, y, z, k, active, own);
      iface_gather<LAT, ST, G>(a, own, c, x, y, z, k, sub, fl, col);
    }
    __syncthreads();
    if (valid) iface_collide<LAT, ST, CUM, G>(a, c, k, active, sub, fl, col);
    __syncthreads();  // the next pass rewrites fl
  }
}

// One lane per cell, or (LG, for grids whose interface lists do not fill
// the GPU) four lanes per cell while the list has at most kIfaceLanes4 cells,
// which splits the chain of dependent loads of a cell's cut links: 55 -> 46 us
// per step for the bubble of radius 16 in 128x128x256.  LG is a separate
// kernel because the group path costs the one-lane path registers (512^3:
// 175 -> 181 us with both in one kernel).
constexpr int kIfaceLanes4 = 65536;

template <int LAT, int ST, bool CUM, bool LG>
__global__ __launch_bounds__(256, sizeof(typename Step<LAT, ST>::R) == 4 ? 5 : 1) void k_lb_iface(
    const typename Step<LAT, ST>::Args a) {
  using R = typename Step<LAT, ST>::R;
  constexpr int Q = Step<LAT, ST>::Q;
  const int n = a.counters[CNT_SPEC];
  __shared__ R fl[Q * 256];
  if constexpr (LG) {
    if (n <= kIfaceLanes4) {
      iface_grouped<LAT, ST, CUM, 4>(a, n, fl);
      return;
    }
  }
  const ListSpan sp = xcd_list_span(n);
  for (int e = sp.e; e < sp.end; e += sp.stride) {
    const int c = a.spec_list[e];
    int x, y, z, k;
    bool active;
    OwnCell<R> own;
    iface_cell<LAT, ST>(a, c, x, y, z, k, active, own);
    iface_gather<LAT, ST, 1>(a, own, c, x, y, z, k, 0, fl, (int)threadIdx.x);
    iface_collide<LAT, ST, CUM, 1>(a, c, k, active, 0, fl, (int)threadIdx.x);
  }
}

// Interface records of the current state (phi, moments, geometry) of every
// interface-adjacent cell, for the next step's interface coupling.
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_pack_iface(const typename Step<LAT, ST>::Args a) {
  using R = typename Step<LAT, ST>::R;
  const size_t N = a.N;
  const ListSpan sp = xcd_list_span(a.counters[CNT_SPEC]);
  for (int e = sp.e; e < sp.end; e += sp.stride) {
    const int c = a.spec_list[e];
    IfaceRec<R> r;
    r.v[0] = a.phi[c];
#pragma unroll
    for (int m = 0; m < 10; ++m) r.v[1 + m] = a.M[(size_t)m * N + c];
#pragma unroll
    for (int m = 0; m < 4; ++m) r.v[11 + m] = a.G[(size_t)m * N + c];
    r.v[15] = (R)0;
    *reinterpret_cast<IfaceRec<R>*>(a.irec + (size_t)16 * c) = r;
  }
}

// ---------------------------------------------------------------------------
// a6: velocity extension.  Seed from the new moments Mn.
// ---------------------------------------------------------------------------
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_ext_seed(const typename Step<LAT, ST>::Args a) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  const size_t N = a.N;
  for_tile_cells<S::D>(a, a.tile_list, a.counters[CNT_TILES], [&](int c, int x, int y, int z) {
    // every load (own tag, moments, phi, normal, both neighbours' tags on
    // each axis) is issued before the cell's class is known
    const uint8_t t = a.tag[c];
    R mn[3];
    for (int m = 0; m < 3; ++m) mn[m] = a.Mn[(1 + m) * N + c];
    const R ph = a.phi[c];
    const int pos[3] = {x, y, z};
    const int n[3] = {a.nx, a.ny, a.nz};
    R gv[3] = {0, 0, 0};
    bool act_lo[3] = {false, false, false}, act_hi[3] = {false, false, false};
    for (int ax = 0; ax < S::D; ++ax) {
      gv[ax] = a.G[ax * N + c];
      for (int sd = -1; sd <= 1; sd += 2) {
        // a neighbour beyond a wall reads the cell itself (no branch around
        // the load); beyond a free-slip face it is the cell's mirror image
        // (the sweep reverses its normal component), beyond a no-slip face
        // it counts as inactive
        const int sv = lb_coord(pos[ax] + sd, sel3(n, ax), sel3(a.per, ax));
        int p2[3] = {x, y, z};
        p2[ax] = sv >= 0 ? sv : pos[ax];
        const uint8_t tn = a.tag[(p2[2] * a.ny + p2[1]) * a.nx + p2[0]];
        const bool mirror = sel6(a.bcf, 2 * ax + (sd > 0 ? 1 : 0)) == LSB_FREESLIP;
        const bool on = ((sv >= 0) | mirror) & ((tn & T_ACT) != 0);
        (sd < 0 ? act_lo : act_hi)[ax] = on;
      }
    }
    if ((t & (T_ACT | T_SPEC)) != T_ACT) return;
    for (int m = 0; m < 3; ++m) a.ut_a[m * N + c] = mn[m];
    // coefficients of the sweeps (phi and n are fixed over them): dtau v_ax
    // with v = S(phi) n; 0 where v_ax is 0 or the upwind neighbour is beyond
    // a no-slip face or not LS-active
    const R sg = ph / sqrt(ph * ph + (R)1);
    for (int ax = 0; ax < S::D; ++ax) {
      const R v = sg * gv[ax];
      R kk = 0;
      if (v != (R)0 && (v > (R)0 ? act_lo[ax] : act_hi[ax])) kk = a.ext_dtau * v;
      a.ext_k[ax * N + c] = kk;
    }
  });
}

// Seed at the interface-adjacent cells: the mean over the cut links of the
// velocity interpolated to the interface.
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_ext_seed_iface(const typename Step<LAT, ST>::Args a) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using L = typename S::L;
  const size_t N = a.N;
  const ListSpan sp = xcd_list_span(a.counters[CNT_SPEC]);
  for (int e = sp.e; e < sp.end; e += sp.stride) {
    const int c = a.spec_list[e];
    const int x = c % a.nx;
    const int y = (c / a.nx) % a.ny;
    const int z = c / (a.nx * a.ny);
    const int k = a.tag[c] & T_GAS;
    const R pc = a.phi[c];
    const R uc[3] = {a.Mn[N + c], a.Mn[2 * N + c], a.Mn[3 * N + c]};
    // the neighbours' tags first, all in flight together (a source beyond a
    // wall reads the cell itself and is skipped), then the cut links' values
    int src[S::Q];
    uint8_t tn[S::Q];
#pragma unroll
    for (int i = 0; i < S::Q; ++i) {
      const int sx = lb_coord(x - L::cx(i), a.nx, a.per[0]);
      const int sy = lb_coord(y - L::cy(i), a.ny, a.per[1]);
      const int sz = lb_coord(z - L::cz(i), a.nz, a.per[2]);
      const bool in = (sx | sy | sz) >= 0;
      src[i] = in ? (sz * a.ny + sy) * a.nx + sx : -1;
      tn[i] = a.tag[in ? src[i] : c];
    }
    R acc[3] = {0, 0, 0};
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < S::Q; ++i) {
      if (c2<LAT>(i) == 0 || src[i] < 0 || (tn[i] & T_GAS) == k) continue;
      const int sc = src[i];
      const R q = pc / (pc - a.phi[sc]);
      for (int m = 0; m < 3; ++m) acc[m] += ((R)1 - q) * uc[m] + q * a.Mn[(1 + m) * N + sc];
      ++cnt;
    }
    for (int m = 0; m < 3; ++m) a.ut_a[m * N + c] = acc[m] / (R)cnt;
  }
}

// One forward-Euler sweep of the first-order upwind extension; interface
// cells are held.  Reads ut_a, writes ut_b.  The upwind neighbours'
// velocities of all axes are loaded together, with no branch on the
// coefficients (an axis with a zero coefficient reads the cell itself); the
// compiler still tests the tag first, which keeps inactive lanes from
// loading at all (issuing every load ahead of that test measured slower).
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_ext_iter(const typename Step<LAT, ST>::Args a) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  const size_t N = a.N;
  for_tile_cells<S::D>(a, a.tile_list, a.counters[CNT_TILES], [&](int c, int x, int y, int z) {
    const uint8_t t = a.tag[c];
    const R u[3] = {a.ut_a[c], a.ut_a[N + c], a.ut_a[2 * N + c]};
    R kk[S::D];
    for (int ax = 0; ax < S::D; ++ax) kk[ax] = a.ext_k[ax * N + c];
    const int pos[3] = {x, y, z};
    const int n[3] = {a.nx, a.ny, a.nz};
    R un[S::D][3];
    for (int ax = 0; ax < S::D; ++ax) {
      const int sv = lb_coord(pos[ax] + (kk[ax] > (R)0 ? -1 : 1), sel3(n, ax), sel3(a.per, ax));
      int p2[3] = {x, y, z};
      p2[ax] = ((kk[ax] != (R)0) & (sv >= 0)) ? sv : pos[ax];
      const int nc = (p2[2] * a.ny + p2[1]) * a.nx + p2[0];
      // beyond a face (a nonzero coefficient there means a free-slip face)
      // the neighbour is the cell's mirror image: normal component reversed
      for (int m = 0; m < 3; ++m) {
        const R w = a.ut_a[m * N + nc];
        un[ax][m] = (m == ax && sv < 0) ? -w : w;
      }
    }
    R out[3] = {u[0], u[1], u[2]};
    for (int ax = 0; ax < S::D; ++ax)
      for (int m = 0; m < 3; ++m) {
        const R diff = kk[ax] > (R)0 ? (u[m] - un[ax][m]) : (un[ax][m] - u[m]);
        const R v = out[m] - kk[ax] * diff;
        out[m] = kk[ax] != (R)0 ? v : out[m];
      }
    if (!(t & T_ACT)) return;
    const bool held = (t & T_SPEC) != 0;
    a.ut_b[c] = held ? u[0] : out[0];
    a.ut_b[N + c] = held ? u[1] : out[1];
    a.ut_b[2 * N + c] = held ? u[2] : out[2];
  });
}

// ---------------------------------------------------------------------------
// a6: TVD-RK3 stage of the transport equation with the fifth-order upwind
// stencil.  stage 1: s1 = phi + L(phi); stage 2: s2 = 3/4 phi + 1/4 (s1 +
// L(s1)); stage 3: phi = 1/3 phi + 2/3 (s2 + L(s2)), clamped to the band.
// Non-active cells keep phi = s1 = s2 (maintained by k_ls_sync).
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ R upwind5(R fm3, R fm2, R fm1, R f0, R fp1, R fp2, R fp3, bool positive) {
  const R r60 = (R)(1.0 / 60.0);
  if (positive) return ((R)-2 * fm3 + (R)15 * fm2 - (R)60 * fm1 + (R)20 * f0 + (R)30 * fp1 - (R)3 * fp2) * r60;
  return ((R)3 * fm2 - (R)30 * fm1 - (R)20 * f0 + (R)60 * fp1 - (R)15 * fp2 + (R)2 * fp3) * r60;
}

template <class Args>
__device__ __forceinline__ int ls_index(const Args& a, int x, int y, int z, int ax, int o) {
  int p[3] = {x, y, z};
  const int n[3] = {a.nx, a.ny, a.nz};
  p[ax] = ls_coord(p[ax] + o, n[ax], sel3(a.per, ax));
  return (p[2] * a.ny + p[1]) * a.nx + p[0];
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_rk3_stage(const typename Step<LAT, ST>::Args a, int stage, const typename Step<LAT, ST>::R* ut) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  const size_t N = a.N;
  const R* in = stage == 1 ? a.phi : (stage == 2 ? a.s1 : a.s2);
  R* out = stage == 1 ? a.s1 : (stage == 2 ? a.s2 : a.phi);
  // every load is issued before the cell's activity is known (the store
  // alone depends on it): one memory round trip per cell instead of three
  for_tile_cells<S::D>(a, a.tile_list, a.counters[CNT_TILES], [&](int c, int x, int y, int z) {
    const bool act = (a.tag[c] & T_ACT) != 0;
    R r = 0;
    for (int ax = 0; ax < S::D; ++ax) {
      const R u = ut[ax * N + c];
      const R dd = upwind5<R>(in[ls_index(a, x, y, z, ax, -3)], in[ls_index(a, x, y, z, ax, -2)],
                              in[ls_index(a, x, y, z, ax, -1)], in[c], in[ls_index(a, x, y, z, ax, 1)],
                              in[ls_index(a, x, y, z, ax, 2)], in[ls_index(a, x, y, z, ax, 3)], u >= (R)0);
      r = r - u * dd;
    }
    const R v = in[c] + r;
    R o;
    if (stage == 1) o = v;
    else if (stage == 2) o = (R)0.75 * a.phi[c] + (R)0.25 * v;
    else {
      o = ((R)1 / (R)3) * a.phi[c] + ((R)2 / (R)3) * v;
      // the band edge is held at exactly +-B (values within the snap width)
      if (o > a.band_snap) o = a.band;
      if (o < -a.band_snap) o = -a.band;
    }
    if (act) out[c] = o;
  });
}

// ---------------------------------------------------------------------------
// a7: constrained reinitialisation (see the oracle's reading): prep stores
// phi0 and the zero-set cells; each stage integrates
// -S(phi0)(|grad phi|_Godunov-WENO5 - 1) plus the crossing-ratio forcing.
// ---------------------------------------------------------------------------
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_reinit_prep(const typename Step<LAT, ST>::Args a) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  for_tile_cells<S::D>(a, a.tile_list, a.counters[CNT_TILES], [&](int c, int x, int y, int z) {
    if (!(a.tag[c] & T_ACT)) return;
    const R ph = a.phi[c];
    a.p0[c] = ph;
    const bool g0 = ph >= (R)0;
    uint8_t fix = 0;
    for (int ax = 0; ax < S::D; ++ax)
      for (int sg = -1; sg <= 1; sg += 2)
        if ((a.phi[ls_index(a, x, y, z, ax, sg)] >= (R)0) != g0) fix = 1;
    a.aux[c] = fix;
  });
}

template <class R>
__device__ __forceinline__ R weno5(R v1, R v2, R v3, R v4, R v5) {
  // constant divisors as multiplications (an IEEE division by a constant
  // is a long instruction sequence)
  const R eps = (R)1e-6;
  const R r3 = (R)(1.0 / 3.0), r6 = (R)(1.0 / 6.0), c76 = (R)(7.0 / 6.0), c116 = (R)(11.0 / 6.0), c56 = (R)(5.0 / 6.0);
  const R p0 = v1 * r3 - v2 * c76 + v3 * c116;
  const R p1 = -v2 * r6 + v3 * c56 + v4 * r3;
  const R p2 = v3 * r3 + v4 * c56 - v5 * r6;
  const R a0 = v1 - (R)2 * v2 + v3, b0 = v1 - (R)4 * v2 + (R)3 * v3;
  const R a1 = v2 - (R)2 * v3 + v4, b1 = v2 - v4;
  const R a2 = v3 - (R)2 * v4 + v5, b2 = (R)3 * v3 - (R)4 * v4 + v5;
  const R c1312 = (R)(13.0 / 12.0);
  const R s0 = c1312 * a0 * a0 + (R)0.25 * b0 * b0;
  const R s1 = c1312 * a1 * a1 + (R)0.25 * b1 * b1;
  const R s2 = c1312 * a2 * a2 + (R)0.25 * b2 * b2;
  const R w0 = (R)0.1 / ((eps + s0) * (eps + s0));
  const R w1 = (R)0.6 / ((eps + s1) * (eps + s1));
  const R w2 = (R)0.3 / ((eps + s2) * (eps + s2));
  return (w0 * p0 + w1 * p1 + w2 * p2) / (w0 + w1 + w2);
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_reinit_stage(const typename Step<LAT, ST>::Args a, int stage, int last) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  const R* in = stage == 1 ? a.phi : (stage == 2 ? a.s1 : a.s2);
  R* out = stage == 1 ? a.s1 : (stage == 2 ? a.s2 : a.phi);
  const R beta = (R)0.5;
  const R dt = a.reinit_dtau;
  // (unlike the RK3 stage, loading before the activity test loses here: the
  // WENO arithmetic would run on the inactive cells of active tiles too)
  for_tile_cells<S::D>(a, a.tile_list, a.counters[CNT_TILES], [&](int c, int x, int y, int z) {
    if (!(a.tag[c] & T_ACT)) return;
    const R ph0 = a.p0[c];
    const R S0 = ph0 / sqrt(ph0 * ph0 + (R)1);
    R h2 = 0;
    for (int ax = 0; ax < S::D; ++ax) {
      const R m3 = in[ls_index(a, x, y, z, ax, -3)], m2 = in[ls_index(a, x, y, z, ax, -2)];
      const R m1 = in[ls_index(a, x, y, z, ax, -1)], c0 = in[c];
      const R q1 = in[ls_index(a, x, y, z, ax, 1)], q2 = in[ls_index(a, x, y, z, ax, 2)];
      const R q3 = in[ls_index(a, x, y, z, ax, 3)];
      const R dm = weno5<R>(m2 - m3, m1 - m2, c0 - m1, q1 - c0, q2 - q1);
      const R dp = weno5<R>(q3 - q2, q2 - q1, q1 - c0, c0 - m1, m1 - m2);
      R t;
      if (S0 > (R)0) {
        const R aa = dm > (R)0 ? dm : (R)0;
        const R bb = dp < (R)0 ? dp : (R)0;
        t = aa * aa > bb * bb ? aa * aa : bb * bb;
      } else {
        const R aa = dm < (R)0 ? dm : (R)0;
        const R bb = dp > (R)0 ? dp : (R)0;
        t = aa * aa > bb * bb ? aa * aa : bb * bb;
      }
      h2 = h2 + t;
    }
    R rt = -S0 * (sqrt(h2) - (R)1);
    if (a.aux[c]) {
      const bool g0 = ph0 >= (R)0;
      R acc = 0;
      int cnt = 0;
      for (int ax = 0; ax < S::D; ++ax)
        for (int sg = -1; sg <= 1; sg += 2) {
          const int j = ls_index(a, x, y, z, ax, sg);
          if ((a.p0[j] >= (R)0) == g0) continue;
          acc = acc + ph0 * (in[c] - in[j]) / (ph0 - a.p0[j]);
          ++cnt;
        }
      rt = rt + beta * (acc / (R)cnt - in[c]);
    }
    const R v = in[c] + dt * rt;
    R o;
    if (stage == 1) o = v;
    else if (stage == 2) o = (R)0.75 * a.phi[c] + (R)0.25 * v;
    else {
      o = ((R)1 / (R)3) * a.phi[c] + ((R)2 / (R)3) * v;
      if (last) {
        if (o > a.band_snap) o = a.band;
        if (o < -a.band_snap) o = -a.band;
      }
    }
    out[c] = o;
  });
}

// Restore phi = s1 = s2 = p0 on the band after the level-set update.
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_ls_sync(const typename Step<LAT, ST>::Args a) {
  for_tile_cells<Step<LAT, ST>::D>(a, a.tile_list, a.counters[CNT_TILES], [&](int c, int, int, int) {
    const bool act = (a.tag[c] & T_ACT) != 0;
    const auto v = a.phi[c];
    if (!act) return;
    a.s1[c] = v;
    a.s2[c] = v;
    a.p0[c] = v;
  });
}

// ---------------------------------------------------------------------------
// a8: classification.  Candidate tiles = active tiles dilated by one tile.
// ---------------------------------------------------------------------------
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_reset_counters(const typename Step<LAT, ST>::Args a, int first, int n) {
  if ((int)threadIdx.x < n) a.counters[first + threadIdx.x] = 0;
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_clear_tiles(const typename Step<LAT, ST>::Args a) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < a.ntiles) {
    a.tile_act[t] = 0;
    a.tile_act_next[t] = 0;
  }
}

template <int LAT, int ST>
__global__ void k_set_scalar(const typename Step<LAT, ST>::Args a, int slot, double v) {
  a.scal[slot] = v;
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_dilate(const typename Step<LAT, ST>::Args a, int all) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  bool cand = all != 0 && t < a.ntiles;
  if (!cand && t < a.ntiles) {
    const int tx = t % a.ntile[0], ty = (t / a.ntile[0]) % a.ntile[1], tz = t / (a.ntile[0] * a.ntile[1]);
    const int zr = Step<LAT, ST>::D == 3 ? 1 : 0;
    for (int dz = -zr; dz <= zr && !cand; ++dz)
      for (int dy = -1; dy <= 1 && !cand; ++dy)
        for (int dx = -1; dx <= 1 && !cand; ++dx) {
          const int ux = lb_coord(tx + dx, a.ntile[0], a.per[0]);
          const int uy = lb_coord(ty + dy, a.ntile[1], a.per[1]);
          const int uz = lb_coord(tz + dz, a.ntile[2], a.per[2]);
          if ((ux | uy | uz) < 0) continue;
          if (a.tile_act[(uz * a.ntile[1] + uy) * a.ntile[0] + ux]) cand = true;
        }
  }
  const int slot = wave_append(&a.counters[CNT_CAND], cand);
  if (cand) a.cand_list[slot] = t;
  if (t < a.ntiles) {
    a.cand_next[t] = cand ? 1 : 0;
    if (!cand) a.tile_act_next[t] = 0;  // candidates get their flag from k_classify
  }
}

// Candidate tiles are classified up to kClassifyBatch at a time per block, and
// the block reserves the list slots of the whole batch with one atomic per list:
// atomics on one counter from every block serialise on the device (about
// 12 ns each on MI355X), so one per tile would cost more than the
// classification itself.
//
// The neighbourhood tests run on bit masks: one wavefront ballot per halo row
// (x along the lanes) gives the row's in-band, gas and liquid cells; OR-ing
// the 3^(D-1) rows around a tile row gives, bit by bit along x, what its
// cells' neighbourhoods hold, and a cell reads its three bits at its own x.
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_classify(const typename Step<LAT, ST>::Args a, int record_flips) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using TS = TileShape<S::D>;
  using u64 = unsigned long long;
  constexpr int tcells = TS::X * TS::Y * TS::Z;
  constexpr int ITER = tcells / 256;  // cells per thread
  constexpr int NW = 256 / 64;        // wavefronts per block
  constexpr int KT = kClassifyBatch;
  constexpr int hz = S::D == 3 ? 1 : 0;
  constexpr int LX = TS::X + 2, LY = TS::Y + 2, LZ = TS::Z + 2 * hz;
  constexpr int NR = LY * LZ;               // halo rows of a tile
  constexpr int RPW = (NR + NW - 1) / NW;   // halo rows per wavefront
  constexpr int TR = TS::Y * TS::Z;         // tile rows
  static_assert(LX <= 64, "a halo row must fit the lanes of one wavefront");
  static_assert(ITER * 256 == tcells, "tile size must be a multiple of the block size");
  static_assert(KT * ITER <= 32, "one flag word per thread holds a batch");
  static_assert(TR <= 256, "one thread per tile row");
  constexpr int NE = KT * ITER * NW;        // count entries of a batch
  static_assert(NE <= 64, "one lane of a wavefront per count entry");
  // per halo row: in-band, gas and liquid cells (cells beyond a wall face
  // are none of them: lattice-neighbour semantics, they are skipped)
  __shared__ u64 rowm[NR][3];
  // per tile row, over its 3^(D-1) neighbour rows: any in band; gas and
  // liquid in the rows that differ in at most one of y, z ("edge") and in
  // the rows that differ in both ("corner", whose lattice links D3Q19 lacks
  // except along x = 0)
  __shared__ u64 summ[TR][5];
  __shared__ int wcnt[2][KT][ITER][NW];  // spec / flip cells per tile, pass and wavefront
  __shared__ int wact[KT][NW];
  __shared__ int tiles[KT];
  __shared__ int pre[2][KT][ITER][NW];   // first list slot of each count entry
  const int count = a.counters[CNT_CAND];
  // wavefront index and tile origins are uniform: scalar arithmetic
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const R B = a.band;
  const R INVALID = (R)1e30;
  // tiles per block: up to KT, fewer where the candidates would otherwise
  // leave the GPU idle (small grids: about 1024 blocks, four per CU)
  const int kb = min(KT, max(1, (count + 1023) / 1024));
  for (int e0 = blockIdx.x * kb; e0 < count; e0 += gridDim.x * kb) {
    const int nk = min(kb, count - e0);
    if ((int)threadIdx.x < nk) tiles[threadIdx.x] = a.cand_list[e0 + threadIdx.x];
    __syncthreads();
    unsigned sbits = 0u, fbits = 0u;  // bit k * ITER + it: spec / flipped cell
    for (int k = 0; k < nk; ++k) {
      int x0, y0, z0;
      tile_origin<S::D>(a, __builtin_amdgcn_readfirstlane(tiles[k]), x0, y0, z0);
      // every load of the tile (halo rows along the lanes, previous tags)
      // is issued before the first is used; a row is a uniform base pointer
      // plus the lane's x
      const int gx = lane < LX ? lb_coord(x0 - 1 + lane, a.nx, a.per[0]) : -1;
      // lane j finds the start of the wavefront's row j (-1 beyond a wall)
      int roff = -1;
      {
        const int r = wave + NW * lane;
        const int gy = lb_coord(y0 - 1 + r % LY, a.ny, a.per[1]);
        const int gz = lb_coord(z0 - hz + r / LY, a.nz, a.per[2]);
        if (lane < RPW && r < NR && (gy | gz) >= 0) roff = (gz * a.ny + gy) * a.nx;
      }
      R hv[RPW];
#pragma unroll
      for (int j = 0; j < RPW; ++j) {
        const int off = __builtin_amdgcn_readlane(roff, j);
        hv[j] = INVALID;
        if (off >= 0 && gx >= 0) hv[j] = (a.phi + (size_t)(unsigned)off)[(unsigned)gx];
      }
      // the tile's cells: a uniform corner plus a per-lane offset
      uint8_t* const tag0 = a.tag + (size_t)(z0 * a.ny + y0) * a.nx + x0;
      uint8_t tprev[ITER];
#pragma unroll
      for (int it = 0; it < ITER; ++it) {
        const int l = threadIdx.x + it * 256;
        const int ix = l & (TS::X - 1), iy = (l >> TS::SX) & (TS::Y - 1), iz = l >> (TS::SX + TS::SY);
        tprev[it] = 0;
        if (record_flips && x0 + ix < a.nx && y0 + iy < a.ny && z0 + iz < a.nz)
          tprev[it] = tag0[(unsigned)((iz * a.ny + iy) * a.nx + ix)];
      }
#pragma unroll
      for (int j = 0; j < RPW; ++j) {
        const int r = wave + NW * j;
        const R v = hv[j];
        const bool in = v != INVALID;
        const u64 mi = __ballot((v < B && v > -B) ? 1 : 0);
        const u64 mg = __ballot((in && v >= (R)0) ? 1 : 0);
        const u64 ml = __ballot((in && v < (R)0) ? 1 : 0);
        if (lane == 0 && r < NR) {
          rowm[r][0] = mi;
          rowm[r][1] = mg;
          rowm[r][2] = ml;
        }
      }
      __syncthreads();
      if (threadIdx.x < TR) {
        const int iy = threadIdx.x % TS::Y, iz = threadIdx.x / TS::Y;
        u64 m[5] = {0ull, 0ull, 0ull, 0ull, 0ull};
#pragma unroll
        for (int dz = -hz; dz <= hz; ++dz)
#pragma unroll
          for (int dy = -1; dy <= 1; ++dy) {
            const int r = (iz + hz + dz) * LY + iy + 1 + dy;
            const int corner = (dy != 0 && dz != 0) ? 1 : 0;
            m[0] |= rowm[r][0];
            m[1 + corner] |= rowm[r][1];
            m[3 + corner] |= rowm[r][2];
          }
#pragma unroll
        for (int q = 0; q < 5; ++q) summ[threadIdx.x][q] = m[q];
      }
      __syncthreads();
      bool act_any = false;
#pragma unroll
      for (int it = 0; it < ITER; ++it) {
        const int l = threadIdx.x + it * 256;
        const int ix = l & (TS::X - 1), iy = (l >> TS::SX) & (TS::Y - 1), iz = l >> (TS::SX + TS::SY);
        const int x = x0 + ix, y = y0 + iy, z = z0 + iz;
        bool sp = false, fl = false;
        if (x < a.nx && y < a.ny && z < a.nz) {
          const int tr = iz * TS::Y + iy;
          // bits ix .. ix + 2 of a row mask are the cells x - 1 .. x + 1
          const int ph = (int)((rowm[(iz + hz) * LY + iy + 1][1] >> (ix + 1)) & 1ull);
          const bool act = ((summ[tr][0] >> ix) & 7ull) != 0ull;
          const u64 oe = summ[tr][ph ? 3 : 1], oc = summ[tr][ph ? 4 : 2];
          if (LAT == LSB_D3Q19) sp = (((oe >> ix) & 7ull) | ((oc >> ix) & 2ull)) != 0ull;
          else sp = (((oe | oc) >> ix) & 7ull) != 0ull;
          // a full classification (record_flips == 0) starts from no previous
          // tag: the tag memory may be uninitialised (state reload); the wall
          // bit is set afterwards by k_mark_walls
          const uint8_t told = record_flips ? tprev[it] : (uint8_t)ph;
          const int old = told & T_GAS;
          tag0[(unsigned)((iz * a.ny + iy) * a.nx + ix)] = (uint8_t)(ph | (act ? T_ACT : 0) | (sp ? T_SPEC : 0) | (told & (T_WALL | T_XWALL)) | (old ? T_OLDGAS : 0));
          act_any = act_any || act;
          fl = record_flips && ph != old;
        }
        if (sp) sbits |= 1u << (k * ITER + it);
        if (fl) fbits |= 1u << (k * ITER + it);
        const u64 sm = __ballot(sp ? 1 : 0), fm = __ballot(fl ? 1 : 0);
        if (lane == 0) {
          wcnt[0][k][it][wave] = __popcll(sm);
          wcnt[1][k][it][wave] = __popcll(fm);
        }
      }
      const u64 am = __ballot(act_any ? 1 : 0);
      if (lane == 0) wact[k][wave] = am != 0ull;
      __syncthreads();  // the next tile restages rowm and summ
    }
    // one reservation per list for the batch, made by wavefront 0: lane
    // (k * ITER + it) * NW + w holds the counts of tile k, pass it and
    // wavefront w, and an inclusive scan over the lanes gives each entry its
    // first slot.  counters[CNT_SPEC] (low word) and counters[CNT_TILES]
    // (high word) share one 64-bit atomic.
    if (wave == 0) {
      const bool ent = lane < NE && lane / (ITER * NW) < nk;
      const int vs = ent ? (&wcnt[0][0][0][0])[lane] : 0;
      const int vf = ent ? (&wcnt[1][0][0][0])[lane] : 0;
      int is = vs, ifl = vf;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int ts = __shfl_up(is, d), tf = __shfl_up(ifl, d);
        if (lane >= d) {
          is += ts;
          ifl += tf;
        }
      }
      const int ns = __shfl(is, 63), nf = __shfl(ifl, 63);
      // tiles with an active cell, in batch order
      int na = 0;
      if (lane < nk)
        for (int w = 0; w < NW; ++w) na |= wact[lane][w];
      const unsigned long long am = __ballot(na ? 1 : 0);
      const int nt = __popcll(am);
      unsigned long long old = 0ull;
      int fb = 0;
      if (lane == 0) {
        if (nt || ns)
          old = atomicAdd(reinterpret_cast<unsigned long long*>(&a.counters[CNT_SPEC]),
                          ((unsigned long long)nt << 32) | (unsigned long long)ns);
        if (nf) fb = atomicAdd(&a.counters[CNT_FLIP], nf);
      }
      old = __shfl(old, 0);
      fb = __shfl(fb, 0);
      if (lane < nk) {
        a.tile_act_next[tiles[lane]] = na ? 1 : 0;
        if (na) a.tile_list[(int)(old >> 32) + __popcll(am & ((1ull << lane) - 1ull))] = tiles[lane];
      }
      if (lane < NE) {
        (&pre[0][0][0][0])[lane] = (int)(old & 0xffffffffull) + is - vs;
        (&pre[1][0][0][0])[lane] = fb + ifl - vf;
      }
    }
    __syncthreads();
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int k = 0; k < nk; ++k) {
      int x0, y0, z0;
      tile_origin<S::D>(a, __builtin_amdgcn_readfirstlane(tiles[k]), x0, y0, z0);
#pragma unroll
      for (int it = 0; it < ITER; ++it) {
        const bool sp = (sbits >> (k * ITER + it)) & 1u, fl = (fbits >> (k * ITER + it)) & 1u;
        const unsigned long long sm = __ballot(sp ? 1 : 0), fm = __ballot(fl ? 1 : 0);
        if (sp || fl) {
          const int l = threadIdx.x + it * 256;
          const int x = x0 + (l & (TS::X - 1)), y = y0 + ((l >> TS::SX) & (TS::Y - 1)), z = z0 + (l >> (TS::SX + TS::SY));
          const int c = (z * a.ny + y) * a.nx + x;
          if (sp) a.spec_list[pre[0][k][it][wave] + __popcll(sm & below)] = c;
          if (fl) a.flip_list[pre[1][k][it][wave] + __popcll(fm & below)] = c;
        }
      }
    }
    __syncthreads();  // wcnt, wact, tiles and pre are reused by the next batch
  }
}

// ---------------------------------------------------------------------------
// a5: normal and curvature by central differences on the active cells.
// ---------------------------------------------------------------------------
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_geometry(const typename Step<LAT, ST>::Args a) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  const size_t N = a.N;
  // the stencil is loaded before the cell's activity is known (only the
  // stores depend on it)
  for_tile_cells<S::D>(a, a.tile_list, a.counters[CNT_TILES], [&](int c, int x, int y, int z) {
    const bool act = (a.tag[c] & T_ACT) != 0;
    auto at = [&](int dx, int dy, int dz) {
      const int sx = ls_coord(x + dx, a.nx, a.per[0]);
      const int sy = ls_coord(y + dy, a.ny, a.per[1]);
      const int sz = ls_coord(z + dz, a.nz, a.per[2]);
      return a.phi[(sz * a.ny + sy) * a.nx + sx];
    };
    const R p = a.phi[c];
    const R gx = (R)0.5 * (at(1, 0, 0) - at(-1, 0, 0));
    const R gy = (R)0.5 * (at(0, 1, 0) - at(0, -1, 0));
    R gz = 0, zz = 0, xz = 0, yz = 0;
    const R xx = at(1, 0, 0) - (R)2 * p + at(-1, 0, 0);
    const R yy = at(0, 1, 0) - (R)2 * p + at(0, -1, 0);
    const R xy = (R)0.25 * (at(1, 1, 0) - at(1, -1, 0) - at(-1, 1, 0) + at(-1, -1, 0));
    if (S::D == 3) {
      gz = (R)0.5 * (at(0, 0, 1) - at(0, 0, -1));
      zz = at(0, 0, 1) - (R)2 * p + at(0, 0, -1);
      xz = (R)0.25 * (at(1, 0, 1) - at(1, 0, -1) - at(-1, 0, 1) + at(-1, 0, -1));
      yz = (R)0.25 * (at(0, 1, 1) - at(0, 1, -1) - at(0, -1, 1) + at(0, -1, -1));
    }
    const R g2 = gx * gx + gy * gy + gz * gz;
    const R g = sqrt(g2);
    if (!act) return;
    if (g < (R)1e-12) {
      a.G[c] = 0; a.G[N + c] = 0; a.G[2 * N + c] = 0; a.G[3 * N + c] = 0;
      return;
    }
    a.G[c] = gx / g;
    a.G[N + c] = gy / g;
    a.G[2 * N + c] = gz / g;
    const R num = xx * (gy * gy + gz * gz) + yy * (gx * gx + gz * gz) + zz * (gx * gx + gy * gy) - (R)2 * gx * gy * xy -
                  (R)2 * gx * gz * xz - (R)2 * gy * gz * yz;
    a.G[3 * N + c] = num / (g2 * g);
  });
}

// ---------------------------------------------------------------------------
// a8: refill of cells whose phase changed (Sec. 2.4).  Reads only
// established cells, writes only flipped cells.
// ---------------------------------------------------------------------------
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_refill(const typename Step<LAT, ST>::Args a) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using L = typename S::L;
  using C = typename S::C;
  constexpr int Q = S::Q;
  const size_t N = a.N;
  const R s = a.scale;
  const ListSpan sp = xcd_list_span(a.counters[CNT_FLIP]);
  for (int e = sp.e; e < sp.end; e += sp.stride) {
    const int c = a.flip_list[e];
    const R pb = (R)baseline(a, c);
    const int x = c % a.nx, y = (c / a.nx) % a.ny, z = c / (a.nx * a.ny);
    const uint8_t t = a.tag[c];
    const int knew = t & T_GAS;
    const int kold = (t & T_OLDGAS) ? 1 : 0;
    const R rm1_new = sel2(a.rref_m1, knew);
    const R sgn = knew == 1 ? (R)1 : (R)-1;
    const R m0 = sgn * a.G[c], m1 = sgn * a.G[N + c], m2 = sgn * a.G[2 * N + c];
    // candidate directions by alignment with the normal into the new phase
    int order[Q];
    R score[Q];
    int nc = 0;
    for (int i = 0; i < Q; ++i) {
      const int cx = L::cx(i), cy = L::cy(i), cz = L::cz(i);
      const int l2 = cx * cx + cy * cy + cz * cz;
      if (l2 == 0) continue;
      const R sc = ((R)cx * m0 + (R)cy * m1 + (R)cz * m2) / sqrt((R)l2);
      if (!(sc > (R)0)) continue;
      int p = nc++;
      order[p] = i;
      score[p] = sc;
      while (p > 0 && score[p - 1] < sc) {
        order[p] = order[p - 1]; score[p] = score[p - 1];
        order[p - 1] = i; score[p - 1] = sc;
        --p;
      }
    }
    // LB densities are handled as deviations rho - 1 (as stored in M)
    const R rhoO = a.Mn[c];
    const R uG0 = a.Mn[N + c], uG1 = a.Mn[2 * N + c], uG2 = a.Mn[3 * N + c];
    const R pold = sel2(a.rho_phys, kold) / (R)3 * rhoO + (kold == 1 ? pb : (R)0);
    const R kap = a.G[3 * N + c];
    const R pnew = knew == 0 ? pold + a.sigma * kap : pold - a.sigma * kap;
    const R rhoG = (pnew - (knew == 1 ? pb : (R)0)) / (sel2(a.rho_phys, knew) / (R)3);
    auto established = [&](int sc) {
      const uint8_t ts = a.tag[sc];
      return (ts & T_GAS) == knew && ((ts & T_OLDGAS) ? 1 : 0) == knew;
    };
    bool done = false;
    for (int tt = 0; tt < nc && !done; ++tt) {
      const int i = order[tt];
      const int ex = L::cx(i), ey = L::cy(i), ez = L::cz(i);
      const int x1 = lb_coord(x + ex, a.nx, a.per[0]), y1 = lb_coord(y + ey, a.ny, a.per[1]),
                z1 = lb_coord(z + ez, a.nz, a.per[2]);
      if ((x1 | y1 | z1) < 0) continue;
      const int c1 = (z1 * a.ny + y1) * a.nx + x1;
      if (!established(c1)) continue;
      const int x2 = lb_coord(x + 2 * ex, a.nx, a.per[0]), y2 = lb_coord(y + 2 * ey, a.ny, a.per[1]),
                z2 = lb_coord(z + 2 * ez, a.nz, a.per[2]);
      int c2c = -1;
      if ((x2 | y2 | z2) >= 0) {
        const int cc2 = (z2 * a.ny + y2) * a.nx + x2;
        if (established(cc2)) c2c = cc2;
      }
      const bool two = c2c >= 0;
      R q;
      const int xm = lb_coord(x - ex, a.nx, a.per[0]), ym = lb_coord(y - ey, a.ny, a.per[1]),
                zm = lb_coord(z - ez, a.nz, a.per[2]);
      const R phc = a.phi[c];
      bool crossed = false;
      if ((xm | ym | zm) >= 0) {
        const R phm = a.phi[(zm * a.ny + ym) * a.nx + xm];
        if ((phm >= (R)0) != (phc >= (R)0)) { crossed = true; q = phc / (phc - phm); }
      }
      if (!crossed) {
        const R len = sqrt((R)(ex * ex + ey * ey + ez * ez));
        const R en = ((R)ex * a.G[c] + (R)ey * a.G[N + c] + (R)ez * a.G[2 * N + c]) / len;
        const R aen = fabs(en);
        if (aen < (R)1e-12) q = (R)1;
        else {
          q = fabs(phc) / (aen * len);
          if (q > (R)1) q = (R)1;
        }
      }
      R w0, w1, w2 = 0;
      if (two) {
        w0 = (R)2 / ((q + (R)1) * (q + (R)2));
        w1 = (R)2 * q / (q + (R)1);
        w2 = -q / (q + (R)2);
      } else {
        w0 = (R)1 / ((R)1 + q);
        w1 = q / ((R)1 + q);
      }
      // into a lighter phase the boundary density is the nearest new-phase cell's
      const R rhoB = sel2(a.rho_phys, knew) >= sel2(a.rho_phys, kold) ? rhoG : a.Mn[c1];
      const R rr = w0 * rhoB + w1 * a.Mn[c1] + (two ? w2 * a.Mn[c2c] : (R)0);
      R ur[3];
      const R uGv[3] = {uG0, uG1, uG2};
      for (int m = 0; m < 3; ++m)
        ur[m] = w0 * uGv[m] + w1 * a.Mn[(1 + m) * N + c1] + (two ? w2 * a.Mn[(1 + m) * N + c2c] : (R)0);
      const R r1 = a.Mn[c1];
      const R u1[3] = {a.Mn[N + c1], a.Mn[2 * N + c1], a.Mn[3 * N + c1]};
      const R uur = ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2];
      const R uu1 = u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2];
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const R w = (R)wgt<LAT>(k);
        const R cur = (R)L::cx(k) * ur[0] + (R)L::cy(k) * ur[1] + (R)L::cz(k) * ur[2];
        const R cu1 = (R)L::cx(k) * u1[0] + (R)L::cy(k) * u1[1] + (R)L::cz(k) * u1[2];
        // equilibria as deviations from the rest state
        const R de = w * (rr + ((R)1 + rr) * ((R)3 * cur + (R)4.5 * cur * cur - (R)1.5 * uur));
        const R de1 = w * (r1 + ((R)1 + r1) * ((R)3 * cu1 + (R)4.5 * cu1 * cu1 - (R)1.5 * uu1));
        const R d1 = C::dec(a.An[pidx<LAT>(k, c1, N)], w, a.inv_scale);
        // f(x_r) = feq(rho_r, u_r) + (f(x1) - feq(x1))
        a.An[pidx<LAT>(k, c, N)] = C::enc(de + (d1 - de1), (R)(1.0 / wgt<LAT>(k)), s);
      }
      a.Mn[c] = rr;
      for (int m = 0; m < 3; ++m) a.Mn[(1 + m) * N + c] = ur[m];
      for (int m = 0; m < 6; ++m) a.Mn[(4 + m) * N + c] = a.Mn[(4 + m) * N + c1];
      done = true;
    }
    if (!done) {
      const R uu = uG0 * uG0 + uG1 * uG1 + uG2 * uG2;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const R w = (R)wgt<LAT>(k);
        const R cu = (R)L::cx(k) * uG0 + (R)L::cy(k) * uG1 + (R)L::cz(k) * uG2;
        const R de = w * (rhoG + ((R)1 + rhoG) * ((R)3 * cu + (R)4.5 * cu * cu - (R)1.5 * uu));
        // stored relative to w rho_ref of the new phase
        a.An[pidx<LAT>(k, c, N)] = C::enc(de - w * rm1_new, (R)(1.0 / wgt<LAT>(k)), s);
      }
      a.Mn[c] = rhoG;
      for (int m = 0; m < 6; ++m) a.Mn[(4 + m) * N + c] = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// a9: Heaviside-weighted gas volume and centroid, deterministic two-pass
// reduction in FP64 over a fixed grid.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double heaviside_d(double phi, double eps) {
  if (phi < -eps) return 0.0;
  if (phi > eps) return 1.0;
  const double pi = 3.14159265358979323846;
  return 0.5 * (1.0 + phi / eps + sin(pi * phi / eps) / pi);
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* part) {
  __shared__ double sh[256];
  for (int m = 0; m < NV; ++m) {
    sh[threadIdx.x] = v[m];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[m] = sh[0];
    __syncthreads();
  }
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_centroid_partial(const typename Step<LAT, ST>::Args a) {
  double v[4] = {0, 0, 0, 0};
  const double eps = (double)a.heps;
  for (int c = blockIdx.x * 256 + threadIdx.x; c < a.N; c += gridDim.x * 256) {
    const double h = heaviside_d((double)a.phi[c], eps);
    if (h == 0.0) continue;
    const int x = c % a.nx, y = (c / a.nx) % a.ny, z = c / (a.nx * a.ny);
    v[0] += h;
    v[1] += h * (x + 0.5);
    v[2] += h * (y + 0.5);
    v[3] += h * (z + 0.5);
  }
  block_sum<4>(v, a.partial + 4 * blockIdx.x);
}

// mode 0: initial centroid -> SC_XC0; mode 1: centroid -> SC_XC and the
// pressure baseline Pb = pb0 + rho_l a_l . (x_c - x_c0).
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_centroid_final(const typename Step<LAT, ST>::Args a, int nparts, int mode,
                                                         double pb0, double rho_l, double al0, double al1, double al2) {
  double v[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nparts; b += 256)
    for (int m = 0; m < 4; ++m) v[m] += a.partial[4 * b + m];
  __shared__ double out[4];
  block_sum<4>(v, out);
  if (threadIdx.x == 0) {
    const double V = out[0];
    double xc[3];
    for (int m = 0; m < 3; ++m) xc[m] = V > 0 ? out[1 + m] / V : 0.0;
    a.scal[SC_V] = V;
    if (mode == 0) {
      for (int m = 0; m < 3; ++m) a.scal[SC_XC0 + m] = xc[m];
    } else {
      for (int m = 0; m < 3; ++m) a.scal[SC_XC + m] = xc[m];
      double pb = pb0;
      const double al[3] = {al0, al1, al2};
      for (int m = 0; m < 3; ++m) pb = pb + rho_l * al[m] * (xc[m] - a.scal[SC_XC0 + m]);
      a.scal[SC_PB] = pb;
    }
  }
}

// ---------------------------------------------------------------------------
// Several bubbles (use_pb = 2): the bubbles are the connected components of
// the smoothed Heaviside's support (phi > -eps) over the lattice links
// (periodic faces wrap, wall faces cut), each with the single-bubble
// baseline at its own centroid, Pb_k = pb0 + rho_l a_l . (x_c,k - x_c0).
// Union-find on the cells: every link joins the two roots by pointing the
// larger at the smaller (atomicMin), so parents only decrease, every chain
// ends, and each root is its component's smallest cell, which also fixes the
// bubbles' numbering (ascending roots).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int bub_parent(const int* lab, int c) {
  return __hip_atomic_load(lab + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// root of c with path halving (a cell's parent becomes its grandparent, by
// atomicMin, so parents still only decrease)
__device__ __forceinline__ int bub_find(int* lab, int c) {
  for (;;) {
    const int q = bub_parent(lab, c);
    if (q == c) return c;
    const int g = bub_parent(lab, q);
    if (g == q) return q;
    atomicMin(lab + c, g);
    c = g;  // g < q < c: strictly decreasing
  }
}
__device__ __forceinline__ void bub_unite(int* lab, int u, int v) {
  for (;;) {
    u = bub_find(lab, u);
    v = bub_find(lab, v);
    if (u == v) return;
    if (u > v) { const int t = u; u = v; v = t; }
    const int old = atomicMin(lab + v, u);
    if (old == v) return;  // v was a root and now hangs under u
    v = old;               // v had been linked meanwhile: join its new parent (old < v)
  }
}

// support cells start at the smallest support cell among themselves and
// their lattice neighbours (a first union step without atomics)
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_bub_init(const typename Step<LAT, ST>::Args a) {
  using L = typename Step<LAT, ST>::L;
  constexpr int Q = Step<LAT, ST>::Q;
  const typename Step<LAT, ST>::R eps = a.heps;
  for (int c = blockIdx.x * 256 + threadIdx.x; c < a.N; c += gridDim.x * 256) {
    if (!(a.phi[c] > -eps)) {
      a.blab[c] = -1;
      continue;
    }
    const int x = c % a.nx, y = (c / a.nx) % a.ny, z = c / (a.nx * a.ny);
    int m = c;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int sx = lb_coord(x - L::cx(i), a.nx, a.per[0]);
      const int sy = lb_coord(y - L::cy(i), a.ny, a.per[1]);
      const int sz = lb_coord(z - L::cz(i), a.nz, a.per[2]);
      if ((sx | sy | sz) < 0) continue;
      const int n = (sz * a.ny + sy) * a.nx + sx;
      if (n < m && a.phi[n] > -eps) m = n;
    }
    a.blab[c] = m;
  }
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_bub_union(const typename Step<LAT, ST>::Args a) {
  using L = typename Step<LAT, ST>::L;
  constexpr int Q = Step<LAT, ST>::Q;
  for (int c = blockIdx.x * 256 + threadIdx.x; c < a.N; c += gridDim.x * 256) {
    if (a.blab[c] < 0) continue;
    const int x = c % a.nx, y = (c / a.nx) % a.ny, z = c / (a.nx * a.ny);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (opp<LAT>(i) <= i) continue;  // one direction of each pair (the rest direction has opp == i)
      const int sx = lb_coord(x - L::cx(i), a.nx, a.per[0]);
      const int sy = lb_coord(y - L::cy(i), a.ny, a.per[1]);
      const int sz = lb_coord(z - L::cz(i), a.nz, a.per[2]);
      if ((sx | sy | sz) < 0) continue;  // through a wall face
      const int n = (sz * a.ny + sy) * a.nx + sx;
      if (a.blab[n] < 0) continue;
      bub_unite(a.blab, c, n);
    }
  }
}

// path compression (every cell of the support points at its root, which
// keeps each parent an ancestor) and the list of roots (at most
// kMaxBubbles stored; the count may exceed it)
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_bub_roots(const typename Step<LAT, ST>::Args a) {
  for (int c = blockIdx.x * 256 + threadIdx.x; c < a.N; c += gridDim.x * 256) {
    if (a.blab[c] < 0) continue;
    const int r = bub_find(a.blab, c);
    if (r == c) {
      const int k = atomicAdd(&a.counters[CNT_BUB], 1);
      if (k < kMaxBubbles) a.broots[k] = c;
    } else {
      a.blab[c] = r;
    }
  }
}

// sort the stored roots (one thread, at most kMaxBubbles); the count goes to
// SC_NBUB
template <int LAT, int ST>
__global__ void k_bub_sort(const typename Step<LAT, ST>::Args a) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const int n = a.counters[CNT_BUB];
  a.scal[SC_NBUB] = (double)n;
  const int m = n < kMaxBubbles ? n : kMaxBubbles;
  for (int i = 1; i < m; ++i) {
    const int v = a.broots[i];
    int j = i - 1;
    while (j >= 0 && a.broots[j] > v) {
      a.broots[j + 1] = a.broots[j];
      --j;
    }
    a.broots[j + 1] = v;
  }
}

// root -> bubble number (rank of the root); -2 for a bubble beyond the
// stored ones (the query calls report the overflow)
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_bub_number(const typename Step<LAT, ST>::Args a) {
  __shared__ int roots[kMaxBubbles];
  const int n = a.counters[CNT_BUB];
  const int m = n < kMaxBubbles ? n : kMaxBubbles;
  for (int i = threadIdx.x; i < m; i += 256) roots[i] = a.broots[i];
  __syncthreads();
  for (int c = blockIdx.x * 256 + threadIdx.x; c < a.N; c += gridDim.x * 256) {
    const int r = a.blab[c];
    if (r < 0) continue;
    int lo = 0, hi = m - 1, id = -2;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int v = roots[mid];
      if (v == r) { id = mid; break; }
      if (v < r) lo = mid + 1; else hi = mid - 1;
    }
    a.blab[c] = id;
  }
}

// per reduction block (a contiguous range of cells) and bubble: sum H and
// sum H x in a fixed order, one pass per bubble present in the range
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_bub_partial(const typename Step<LAT, ST>::Args a) {
  const int chunk = (a.N + (int)gridDim.x - 1) / (int)gridDim.x;
  const int c0 = blockIdx.x * chunk;
  const int c1 = c0 + chunk < a.N ? c0 + chunk : a.N;
  const double eps = (double)a.heps;
  __shared__ unsigned long long present;
  if (threadIdx.x == 0) present = 0ull;
  __syncthreads();
  unsigned long long mine = 0ull;
  for (int c = c0 + (int)threadIdx.x; c < c1; c += 256) {
    const int id = a.blab[c];
    if (id >= 0) mine |= 1ull << id;
  }
  if (mine) atomicOr(&present, mine);
  __syncthreads();
  const unsigned long long mask = present;
  double* part = a.bpart + (size_t)blockIdx.x * kMaxBubbles * 4;
  for (int i = threadIdx.x; i < kMaxBubbles * 4; i += 256)
    if (!((mask >> (i >> 2)) & 1ull)) part[i] = 0.0;
  for (unsigned long long mk = mask; mk; mk &= mk - 1ull) {
    const int k = __ffsll((long long)mk) - 1;
    double v[4] = {0, 0, 0, 0};
    for (int c = c0 + (int)threadIdx.x; c < c1; c += 256) {
      if (a.blab[c] != k) continue;
      const double h = heaviside_d((double)a.phi[c], eps);
      const int x = c % a.nx, y = (c / a.nx) % a.ny, z = c / (a.nx * a.ny);
      v[0] += h;
      v[1] += h * (x + 0.5);
      v[2] += h * (y + 0.5);
      v[3] += h * (z + 0.5);
    }
    block_sum<4>(v, part + 4 * k);
  }
}

// per bubble (one block each): volume, centroid and baseline, the partials
// summed in a fixed order
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_bub_final(const typename Step<LAT, ST>::Args a, int nparts, double pb0,
                                                   double rho_l, double al0, double al1, double al2) {
  const int k = blockIdx.x;
  if (k >= a.counters[CNT_BUB]) return;
  double v[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nparts; b += 256)
    for (int m = 0; m < 4; ++m) v[m] += a.bpart[((size_t)b * kMaxBubbles + k) * 4 + m];
  __shared__ double sum[4];
  block_sum<4>(v, sum);
  if (threadIdx.x != 0) return;
  const double al[3] = {al0, al1, al2};
  double pb = pb0;
  double* out = a.bres + 5 * k;
  out[0] = sum[0];
  for (int m = 0; m < 3; ++m) {
    const double xc = sum[0] > 0 ? sum[1 + m] / sum[0] : 0.0;
    out[1 + m] = xc;
    pb = pb + rho_l * al[m] * (xc - a.scal[SC_XC0 + m]);
  }
  out[4] = pb;
}

// per cell: the baseline of its bubble
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_bub_field(const typename Step<LAT, ST>::Args a) {
  using R = typename Step<LAT, ST>::R;
  for (int c = blockIdx.x * 256 + threadIdx.x; c < a.N; c += gridDim.x * 256) {
    const int id = a.blab[c];
    if (id >= 0) a.pbc[c] = (R)a.bres[5 * id + 4];  // only gas cells read it (all in the support)
  }
}


// ---------------------------------------------------------------------------
// Initialisation and output kernels.
// ---------------------------------------------------------------------------
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_init_phi(const typename Step<LAT, ST>::Args a, const double* phi0, int c0,
                                                  int c1) {
  using R = typename Step<LAT, ST>::R;
  for (int c = c0 + blockIdx.x * 256 + threadIdx.x; c < c1; c += gridDim.x * 256) {
    double p = phi0[c - c0];
    const double B = (double)a.band;
    if (p > B - kBandSnap) p = B;
    if (p < -(B - kBandSnap)) p = -B;
    const R v = (R)p;
    a.phi[c] = v; a.s1[c] = v; a.s2[c] = v; a.p0[c] = v;
    a.tag[c] = 0;
  }
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_init_pop(const typename Step<LAT, ST>::Args a, const double* rho0,
                                                  const double* u0, int hydro, int c0, int c1) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using L = typename S::L;
  using C = typename S::C;
  const size_t N = a.N;
  const R s = a.scale;
  for (int c = c0 + blockIdx.x * 256 + threadIdx.x; c < c1; c += gridDim.x * 256) {
    const int x = c % a.nx, y = (c / a.nx) % a.ny, z = c / (a.nx * a.ny);
    const int k = a.tag[c] & T_GAS;
    double rho;
    if (rho0) rho = rho0[c - c0];
    else {
      rho = 1.0;
      if (hydro) {
        // about the initial centroid; a gas cell of one of several bubbles
        // about its own bubble's
        const double pos[3] = {x + 0.5, y + 0.5, z + 0.5};
        const double* ref = a.scal + SC_XC0;
        if (a.use_pb == 2 && k == 1 && a.blab[c] >= 0) ref = a.bres + 5 * a.blab[c] + 1;
        for (int m = 0; m < 3; ++m) rho = rho + (double)ACC(a, k, m) * (pos[m] - ref[m]) / (1.0 / 3.0);
      }
    }
    double u[3] = {0, 0, 0};
    if (u0) for (int m = 0; m < 3; ++m) u[m] = u0[3 * (size_t)(c - c0) + m];
    if (S::D == 2) u[2] = 0;
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
    for (int i = 0; i < S::Q; ++i) {
      const double w = wgt<LAT>(i);
      const double cu = L::cx(i) * u[0] + L::cy(i) * u[1] + L::cz(i) * u[2];
      const double fe = w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
      // stored relative to w rho_ref of the cell's phase
      a.An[pidx<LAT>(i, c, N)] = C::enc((R)(fe - w * (double)sel2(a.rho_ref, k)), (R)(1.0 / w), s);
    }
    R* Ms[2] = {const_cast<R*>(a.M), a.Mn};
    for (int b = 0; b < 2; ++b) {
      Ms[b][c] = (R)(rho - 1.0);
      for (int m = 0; m < 3; ++m) Ms[b][(1 + m) * N + c] = (R)u[m];
      for (int m = 0; m < 6; ++m) Ms[b][(4 + m) * N + c] = 0;
    }
  }
}

// Macroscopic output from the current populations (a.A).
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_fields(const typename Step<LAT, ST>::Args a, double* rho_out, double* u_out,
                                                double* p_out, uint8_t* ph_out, int c0, int c1) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using L = typename S::L;
  using C = typename S::C;
  const R s = a.scale;
  for (int c = c0 + blockIdx.x * 256 + threadIdx.x; c < c1; c += gridDim.x * 256) {
    const int k = a.tag[c] & T_GAS;
    const double rref = (double)sel2(a.rho_ref, k);
    double rho = 0, m[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < S::Q; ++i) {
      const R w = (R)wgt<LAT>(i);
      const double f = wgt<LAT>(i) * rref + (double)C::dec(a.A[pidx<LAT>(i, c, a.N)], w, a.inv_scale);
      rho += f;
      m[0] += L::cx(i) * f; m[1] += L::cy(i) * f; m[2] += L::cz(i) * f;
    }
    const size_t o = (size_t)(c - c0);
    if (rho_out) rho_out[o] = rho;
    if (u_out)
      for (int d = 0; d < S::D; ++d) u_out[(size_t)S::D * o + d] = m[d] / rho - 0.5 * (double)ACC(a, k, d);
    if (p_out) p_out[o] = (double)sel2(a.rho_phys, k) / 3.0 * (rho - 1.0) + (k == 1 ? (double)baseline(a, c) : 0.0);
    if (ph_out) ph_out[o] = (uint8_t)k;
  }
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_populations(const typename Step<LAT, ST>::Args a, double* out, int i0, int i1,
                                                     int c0, int c1) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using C = typename S::C;
  const R s = a.scale;
  const size_t n = (size_t)(c1 - c0);
  for (int c = c0 + blockIdx.x * 256 + threadIdx.x; c < c1; c += gridDim.x * 256) {
    const double rref = (double)sel2(a.rho_ref, a.tag[c] & T_GAS);
    for (int i = i0; i < i1; ++i) {
      double w = 0;
      for (int k = 0; k < S::Q; ++k) if (k == i) w = wgt<LAT>(k);
      out[(size_t)(i - i0) * n + (c - c0)] = w * rref + (double)C::dec(a.A[pidx<LAT>(i, c, a.N)], (R)w, a.inv_scale);
    }
  }
}

// Integral quantities: per-block partials of mass[2], V, sum x H[3],
// sum u H[3], max |u|, bad-cell count.
template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_integrals_partial(const typename Step<LAT, ST>::Args a) {
  using S = Step<LAT, ST>;
  using R = typename S::R;
  using L = typename S::L;
  using C = typename S::C;
  const R s = a.scale;
  double v[13] = {0};  // ..., [11], [12]: cells of each phase
  double umax = 0;
  const double eps = (double)a.heps;
  for (int c = blockIdx.x * 256 + threadIdx.x; c < a.N; c += gridDim.x * 256) {
    const int k = a.tag[c] & T_GAS;
    const double rref = (double)sel2(a.rho_ref, k);
    double rho = 0, m[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < S::Q; ++i) {
      const R w = (R)wgt<LAT>(i);
      const double f = wgt<LAT>(i) * rref + (double)C::dec(a.A[pidx<LAT>(i, c, a.N)], w, a.inv_scale);
      rho += f;
      m[0] += L::cx(i) * f; m[1] += L::cy(i) * f; m[2] += L::cz(i) * f;
    }
    double u[3];
    for (int d = 0; d < 3; ++d) u[d] = m[d] / rho - 0.5 * (double)ACC(a, k, d);
    v[k] += rho;
    v[11 + k] += 1.0;
    const double h = heaviside_d((double)a.phi[c], eps);
    const int x = c % a.nx, y = (c / a.nx) % a.ny, z = c / (a.nx * a.ny);
    v[2] += h;
    v[3] += h * (x + 0.5); v[4] += h * (y + 0.5); v[5] += h * (z + 0.5);
    v[6] += h * u[0]; v[7] += h * u[1]; v[8] += h * u[2];
    const double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (!(rho > 0.0) || !(un <= 0.3) || !isfinite(rho)) v[10] += 1.0;
    if (un > umax) umax = un;
  }
  block_sum<13>(v, a.partial + 16 * blockIdx.x);
  // max of |u|
  __shared__ double sh[256];
  sh[threadIdx.x] = umax;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w && sh[threadIdx.x + w] > sh[threadIdx.x]) sh[threadIdx.x] = sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[16 * blockIdx.x + 9] = sh[0];
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_export_interface(const typename Step<LAT, ST>::Args a, double* phi, double* nrm,
                                                          double* kap, uint8_t* tags, int c0, int c1) {
  using S = Step<LAT, ST>;
  const size_t N = a.N;
  for (int c = c0 + blockIdx.x * 256 + threadIdx.x; c < c1; c += gridDim.x * 256) {
    const size_t o = (size_t)(c - c0);
    if (phi) phi[o] = (double)a.phi[c];
    if (nrm) for (int d = 0; d < S::D; ++d) nrm[(size_t)S::D * o + d] = (double)a.G[d * N + c];
    if (kap) kap[o] = (double)a.G[3 * N + c];
    if (tags) tags[o] = a.tag[c] & (T_GAS | T_ACT | T_SPEC);
  }
}

template <int LAT, int ST>
__global__ __launch_bounds__(256) void k_export_moments(const typename Step<LAT, ST>::Args a, double* out, int c0, int c1) {
  const size_t N = a.N;
  for (int c = c0 + blockIdx.x * 256 + threadIdx.x; c < c1; c += gridDim.x * 256)
    for (int m = 0; m < 10; ++m) out[10 * (size_t)(c - c0) + m] = (double)a.M[m * N + c] + (m == 0 ? 1.0 : 0.0);
}

}  // namespace lsb
