// common.h -- device-side building blocks shared by the HIP kernels:
// velocity sets, storage codecs, the kernel argument block, index helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <cstdint>

#include "../../include/lsb.h"

namespace lsb {

// Tag bits of one cell (one byte per cell).
enum : uint8_t {
  T_GAS = 1,      // phase: gas (phi >= 0)
  T_ACT = 2,      // LS-active: in the narrow band or next to it
  T_SPEC = 4,     // has a lattice link to a cell of the other phase
  T_WALL = 8,     // has a lattice link through a wall face (static)
  T_OLDGAS = 16,  // phase before the last classification (refill)
  T_XWALL = 32,   // 3D: lattice links through x faces only (the bulk kernel takes them, static)
};

// ---------------------------------------------------------------------------
// Velocity sets.  Direction order of the paper's velocity-set figure, rest
// last.  D3Q19 = D3Q27 directions 0..17 + rest.
// ---------------------------------------------------------------------------
template <int LAT>
struct Lat;

template <>
struct Lat<LSB_D2Q9> {
  static constexpr int D = 2, Q = 9;
  __host__ __device__ static constexpr int cx(int i) { return (i == 0 || i == 4 || i == 5) ? -1 : ((i == 1 || i == 6 || i == 7) ? 1 : 0); }
  __host__ __device__ static constexpr int cy(int i) { return (i == 2 || i == 4 || i == 7) ? -1 : ((i == 3 || i == 5 || i == 6) ? 1 : 0); }
  __host__ __device__ static constexpr int cz(int) { return 0; }
};

namespace detail {
// D3Q27 directions of the paper's figure, packed as (cx+1) + 3(cy+1) + 9(cz+1).
__host__ __device__ constexpr int d3q27_code(int i) {
  constexpr int code[27] = {12, 14, 10, 16, 4, 22, 9, 15, 11, 17, 3, 21, 5, 23, 1, 19, 7, 25,
                            0, 18, 6, 24, 2, 20, 8, 26, 13};
  return code[i];
}
}  // namespace detail

template <>
struct Lat<LSB_D3Q27> {
  static constexpr int D = 3, Q = 27;
  __host__ __device__ static constexpr int cx(int i) { return detail::d3q27_code(i) % 3 - 1; }
  __host__ __device__ static constexpr int cy(int i) { return (detail::d3q27_code(i) / 3) % 3 - 1; }
  __host__ __device__ static constexpr int cz(int i) { return detail::d3q27_code(i) / 9 - 1; }
};

template <>
struct Lat<LSB_D3Q19> {
  static constexpr int D = 3, Q = 19;
  __host__ __device__ static constexpr int cx(int i) { return i == 18 ? 0 : Lat<LSB_D3Q27>::cx(i); }
  __host__ __device__ static constexpr int cy(int i) { return i == 18 ? 0 : Lat<LSB_D3Q27>::cy(i); }
  __host__ __device__ static constexpr int cz(int i) { return i == 18 ? 0 : Lat<LSB_D3Q27>::cz(i); }
};

template <int LAT>
__host__ __device__ constexpr int c2(int i) {
  return Lat<LAT>::cx(i) * Lat<LAT>::cx(i) + Lat<LAT>::cy(i) * Lat<LAT>::cy(i) + Lat<LAT>::cz(i) * Lat<LAT>::cz(i);
}

// Lattice weights (Sec. 2.1; D3Q19 textbook).
template <int LAT>
__host__ __device__ constexpr double wgt(int i) {
  return LAT == LSB_D2Q9 ? (c2<LAT>(i) == 0 ? 4.0 / 9 : c2<LAT>(i) == 1 ? 1.0 / 9 : 1.0 / 36)
       : LAT == LSB_D3Q19 ? (c2<LAT>(i) == 0 ? 1.0 / 3 : c2<LAT>(i) == 1 ? 1.0 / 18 : 1.0 / 36)
       : (c2<LAT>(i) == 0 ? 8.0 / 27 : c2<LAT>(i) == 1 ? 2.0 / 27 : c2<LAT>(i) == 2 ? 1.0 / 54 : 1.0 / 216);
}

// ---------------------------------------------------------------------------
// Population layout.  D2Q9: one array per direction, [q][cell].  D3Q19 and
// D3Q27: the cells in chunks of 256 consecutive cells, [cell / 256][q]
// [cell % 256]: the directions of a chunk are stored together, so the
// loads and stores of a 256-cell block fall into few DRAM pages (the D3Q27
// FP16 pull pattern runs at 5.83 TB/s this way against 5.31 TB/s with one
// array per direction).  The 3D layout pads N to a multiple of 256.
// ---------------------------------------------------------------------------
template <int LAT>
__host__ __device__ __forceinline__ size_t pop_cell(int c) {  // element offset of cell c, direction 0
  if constexpr (LAT == LSB_D2Q9) return (size_t)c;
  else return (size_t)(c >> 8) * (size_t)(Lat<LAT>::Q << 8) + (size_t)(c & 255);
}
template <int LAT>
__host__ __device__ __forceinline__ size_t pop_dir(int i, size_t N) {  // element offset of direction i
  if constexpr (LAT == LSB_D2Q9) return (size_t)i * N;
  else return (size_t)i << 8;
}
template <int LAT>
__host__ __device__ __forceinline__ size_t pidx(int i, int c, size_t N) {
  return pop_dir<LAT>(i, N) + pop_cell<LAT>(c);
}
template <int LAT>
__host__ __device__ inline size_t pop_elems(size_t N) {  // elements of one population buffer
  return LAT == LSB_D2Q9 ? (size_t)Lat<LAT>::Q * N : (size_t)Lat<LAT>::Q * ((N + 255) / 256 * 256);
}

template <int LAT>
__host__ __device__ constexpr int opp(int i) {
  int j = 0;
  for (int k = 0; k < Lat<LAT>::Q; ++k)
    if (Lat<LAT>::cx(k) == -Lat<LAT>::cx(i) && Lat<LAT>::cy(k) == -Lat<LAT>::cy(i) && Lat<LAT>::cz(k) == -Lat<LAT>::cz(i)) j = k;
  return j;
}

template <int LAT>
__host__ __device__ constexpr int dir_of(int x, int y, int z) {
  int j = -1;
  for (int k = 0; k < Lat<LAT>::Q; ++k)
    if (Lat<LAT>::cx(k) == x && Lat<LAT>::cy(k) == y && Lat<LAT>::cz(k) == z) j = k;
  return j;
}

// Lattice tables for runtime direction indices (constant memory).
template <int LAT>
struct Tables {
  int cx[27], cy[27], cz[27], opp[27];
  float wf[27], wif[27];
  double wd[27], wid[27];
};

template <int LAT>
__host__ __device__ constexpr Tables<LAT> make_tables() {
  Tables<LAT> t{};
  for (int i = 0; i < Lat<LAT>::Q; ++i) {
    t.cx[i] = Lat<LAT>::cx(i);
    t.cy[i] = Lat<LAT>::cy(i);
    t.cz[i] = Lat<LAT>::cz(i);
    t.opp[i] = opp<LAT>(i);
    t.wd[i] = wgt<LAT>(i);
    t.wf[i] = (float)wgt<LAT>(i);
    t.wid[i] = 1.0 / wgt<LAT>(i);
    t.wif[i] = (float)(1.0 / wgt<LAT>(i));
  }
  return t;
}

template <int LAT>
__constant__ Tables<LAT> tab = make_tables<LAT>();

template <int LAT, class R>
__device__ __forceinline__ R tw(int i) {
  if constexpr (sizeof(R) == 8) return tab<LAT>.wd[i];
  else return tab<LAT>.wf[i];
}

template <int LAT, class R>
__device__ __forceinline__ R twinv(int i) {
  if constexpr (sizeof(R) == 8) return tab<LAT>.wid[i];
  else return tab<LAT>.wif[i];
}

// ---------------------------------------------------------------------------
// Storage codecs.  Populations are kept as deviations d_i = f_i - w_i from
// the rest state; the FP16/BF16 paths store s d_i / w_i.
// ---------------------------------------------------------------------------
template <int ST>
struct Codec;

// dec(v, w, 1/s) -> deviation; enc(d, 1/w, s) -> stored value (multiplies only).
template <>
struct Codec<LSB_F64> {
  using T = double;
  using R = double;
  __device__ static R dec(T v, R, R) { return v; }
  __device__ static T enc(R d, R, R) { return d; }
};

template <>
struct Codec<LSB_F32> {
  using T = float;
  using R = float;
  __device__ static R dec(T v, R, R) { return v; }
  __device__ static T enc(R d, R, R) { return d; }
};

template <>
struct Codec<LSB_F16DEV> {
  using T = uint16_t;
  using R = float;
  __device__ static R dec(T v, R w, R inv_s) { return __half2float(__ushort_as_half(v)) * (w * inv_s); }
  __device__ static T enc(R d, R inv_w, R s) { return __half_as_ushort(__float2half_rn(d * (s * inv_w))); }
};

template <>
struct Codec<LSB_BF16DEV> {
  using T = uint16_t;
  using R = float;
  __device__ static R dec(T v, R w, R inv_s) { return __uint_as_float(((unsigned)v) << 16) * (w * inv_s); }
  __device__ static T enc(R d, R inv_w, R s) {
    __hip_bfloat16 b = __float2bfloat16(d * (s * inv_w));  // round to nearest even
    return *reinterpret_cast<uint16_t*>(&b);
  }
};

// Population store of the collide-stream kernels: nontemporal, the written
// lattice is read again only in the next step (it does not fit any cache).
template <class T>
__device__ __forceinline__ void store_pop(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

// ---------------------------------------------------------------------------
// Kernel argument block (everything a kernel may need, by value).
// ---------------------------------------------------------------------------
template <class T, class R>
struct KArgs {
  int nx, ny, nz, N;
  int per[3];         // axis periodic?
  int bcf[6];         // face conditions
  R wall_u[6][3];
  R omega[2];
  int cum[2];         // phase uses the cumulant collision (D3Q27)
  R acc[2][3];
  R rho_phys[2];
  R eta[2];
  R sigma;
  R iface_pc[2];      // rho_phys_k / 3 (pressure per LB density deviation)
  R iface_inv2etap;   // 1 / (2 eta_p), eta_p the floored divisor of the pressure jump
  R iface_acoef;      // -[eta] / eta_bar
  R band;
  R band_snap;        // band - kBandSnap: beyond it (in magnitude) phi is held at +-band
  R ext_dtau, reinit_dtau;
  R heps;
  R scale;            // storage scale s
  R inv_scale;        // 1 / s
  // Reference density of each phase's stored deviations: a population of
  // phase k is stored as f - w_i rho_ref[k] (FP16 / BF16 storage: the
  // phase's mean initial LB density; 1 for FP32 / FP64 storage), and the
  // collide-stream kernels carry deviations in that frame.  rref_m1 =
  // rho_ref - 1 (exact).
  R rho_ref[2];
  R rref_m1[2];
  int use_pb;
  // tiles
  int tdim[3];        // tile extents
  int ntile[3];       // tiles per axis
  int ntiles;
  // state
  const T* __restrict__ A;  // populations read this step
  T* __restrict__ An;       // populations written this step
  R* phi;
  R* s1;
  R* s2;
  R* p0;
  uint8_t* tag;
  uint8_t* aux;
  const R* M;               // moments of the previous collision [10][N]
  R* Mn;                    // moments written this step
  R* G;                     // normal[3], kappa  [4][N]
  R* ut_a;
  R* ut_b;
  R* ext_k;                 // per LS-active cell and axis: dtau v_ax towards the upwind neighbour, 0 if none
  R* irec;                  // per interface-adjacent cell: phi, M[10], G[4] of the current state (16 values)
  // several bubbles (use_pb = 2)
  int* blab;                // per cell: union-find parent, then the bubble (-1 outside the Heaviside support)
  int* broots;              // roots of the bubbles, ascending (at most kMaxBubbles)
  double* bpart;            // per reduction block and bubble: sum H, sum H x[3]
  double* bres;             // per bubble: volume, centroid[3], baseline
  R* pbc;                   // per cell: the baseline of its bubble
  double* scal;             // device scalars (see SC_*)
  // lists
  int* counters;            // see CNT_*
  uint8_t* tile_act;        // per tile: has LS-active cells (this step)
  uint8_t* tile_act_next;   // the same after this step's classification
  uint8_t* cand_prev;       // per tile: candidate of the previous step's classification
  uint8_t* cand_next;       // per tile: candidate of this step's classification
  int* tile_list;           // active tiles
  int* cand_list;           // candidate tiles for classification
  int* spec_list;           // interface-adjacent cells
  int* flip_list;           // cells whose phase changed
  int* wall_list;           // cells with a link through a wall face
  double* partial;          // reduction partials
  const R* ghost;           // populations entering across injected faces [Q][N] (kFaceInject)
};

// device scalar slots (SC_NBUB: bubbles found, may exceed kMaxBubbles)
// SC_RREF: the codec's reference density of each phase (two slots)
enum { SC_PB = 0, SC_XC0 = 1, SC_XC = 4, SC_V = 7, SC_NBUB = 8, SC_RREF = 9, SC_COUNT = 16 };
constexpr int kMaxBubbles = LSB_MAX_BUBBLES;
constexpr int kBubbleParts = 16384;  // reduction blocks of the per-bubble sums
// counters: CNT_SPEC, CNT_TILES and CNT_FLIP are cleared before each
// classification, CNT_CAND before each dilation, CNT_WALL is static.
// CNT_SPEC and CNT_TILES form one aligned 64-bit word (one atomic reserves
// slots in both lists).
enum { CNT_SPEC = 0, CNT_TILES = 1, CNT_FLIP = 2, CNT_CAND = 3, CNT_WALL = 4, CNT_BUB = 5, CNT_NUM = 8 };

// Runtime selection from small arrays of the kernel argument block without
// indexing it dynamically (which would copy the block to scratch memory).
template <class V>
__device__ __forceinline__ V sel2(const V (&v)[2], int i) { return i ? v[1] : v[0]; }
template <class V>
__device__ __forceinline__ V sel3(const V (&v)[3], int i) { return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]); }
template <class V>
__device__ __forceinline__ V sel6(const V (&v)[6], int i) {
  return i < 3 ? (i == 0 ? v[0] : (i == 1 ? v[1] : v[2])) : (i == 3 ? v[3] : (i == 4 ? v[4] : v[5]));
}
// acceleration component m of phase k, wall velocity component m of face f
#define ACC(a, k, m) ((k) ? (a).acc[1][m] : (a).acc[0][m])
#define WALLU(a, f, m)                                                                                  \
  ((f) < 3 ? ((f) == 0 ? (a).wall_u[0][m] : ((f) == 1 ? (a).wall_u[1][m] : (a).wall_u[2][m]))           \
           : ((f) == 3 ? (a).wall_u[3][m] : ((f) == 4 ? (a).wall_u[4][m] : (a).wall_u[5][m])))

// Width of the band edge that is held at exactly +-B (cells): level-set
// values within it of +-B are set to +-B after transport and reinitialisation
// and at initialisation, so that drifts below a reduced-precision level
// set's resolution at |phi| = B never reach the reinitialisation stencils.
constexpr double kBandSnap = 1e-3;

// Face condition of a refined box's faces (internal; never accepted from a
// caller's lsb_params): a population whose source lies beyond the face is
// read from the ghost array the coarser grid fills, ghost[i N + c] (FP64 or
// FP32 like the moments, the deviation f - w_i rho_ref of the cell's phase).
constexpr int kFaceInject = 3;

// Level-set stencil coordinate: periodic wrap, or even mirror about a wall face.
__device__ __forceinline__ int ls_coord(int s, int n, int periodic) {
  if (s >= 0 && s < n) return s;
  if (periodic) return s < 0 ? s + n * ((-s + n - 1) / n) : s % n;
  return s < 0 ? -1 - s : 2 * n - 1 - s;
}

// Lattice neighbour coordinate: periodic wrap, -1 when leaving through a wall.
__device__ __forceinline__ int lb_coord(int s, int n, int periodic) {
  if (s >= 0 && s < n) return s;
  if (!periodic) return -1;
  return s < 0 ? s + n : s - n;
}

// Tiles of the narrow band: 32x4x4 cells in 3D (a 64-wide wavefront covers
// two full x-rows), 16x16 in 2D; log2 of the extents.
template <int D>
struct TileShape {
  static constexpr int SX = D == 3 ? 5 : 4, SY = D == 3 ? 2 : 4, SZ = D == 3 ? 2 : 0;
  static constexpr int X = 1 << SX, Y = 1 << SY, Z = 1 << SZ;
};
// largest tile plus one-cell halo, in cells, that the tile kernels accept
constexpr int kClassifyLds = 1280;
// most candidate tiles per block batch of the classification kernel
constexpr int kClassifyBatch = 8;

// Append for the lanes of a wavefront with pred set: one atomic per
// wavefront on the counter; lanes keep their order.  Returns the slot of
// the calling lane (meaningful where pred is set).  All active lanes of the
// wavefront must call it together.
__device__ __forceinline__ int wave_append(int* counter, bool pred) {
  const unsigned long long mask = __ballot(pred ? 1 : 0);
  if (mask == 0ull) return -1;
  const int lane = (int)__lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(mask));
  base = __shfl(base, leader);
  return base + __popcll(mask & ((1ull << lane) - 1ull));
}

__device__ __forceinline__ unsigned remap_xcd(unsigned b, unsigned nb) {
  // MI355X dispatches consecutive workgroups round-robin over 8 XCDs; give
  // each XCD a contiguous range of logical blocks so that neighbouring blocks
  // share one L2.
  if ((nb & 7u) != 0u) return b;
  return (b & 7u) * (nb >> 3) + (b >> 3);
}

// Entries of a list (0 .. n-1) that this thread takes: the list is split
// into 8 contiguous parts, one per XCD (workgroups are dispatched round-robin
// over the XCDs), each part strided over that XCD's blocks, so that list
// neighbours (cells of one tile batch, a run of one wall plane) share one L2.
struct ListSpan {
  int e, end, stride;
};
__device__ __forceinline__ ListSpan xcd_list_span(int n) {
  if ((gridDim.x & 7u) != 0u) return {(int)(blockIdx.x * 256u + threadIdx.x), n, (int)(gridDim.x * 256u)};
  const int xcd = (int)(blockIdx.x & 7u), j = (int)(blockIdx.x >> 3);
  const int per = (n + 7) >> 3;
  const int lo = xcd * per;
  return {lo + j * 256 + (int)threadIdx.x, min(n, lo + per), (int)(gridDim.x >> 3) * 256};
}

}  // namespace lsb
