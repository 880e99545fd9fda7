// driver.h -- host launch sequence of one time step and of the queries,
// templated on the velocity set and the storage.  Included by one
// translation unit per velocity set.
#pragma once

#include "kernels.h"
#include "plan.h"

namespace lsb {

template <int LAT, int ST>
struct Driver {
  using S = Step<LAT, ST>;
  using T = typename S::T;
  using R = typename S::R;
  using Args = typename S::Args;

  static Args args(lsb_plan* p, int cur) {
    Args a{};
    const lsb_params& P = p->P;
    a.nx = P.nx; a.ny = P.ny; a.nz = P.nz; a.N = p->N;
    for (int ax = 0; ax < 3; ++ax) a.per[ax] = P.bc[2 * ax] == LSB_PERIODIC;
    for (int f = 0; f < 6; ++f) {
      a.bcf[f] = P.bc[f];
      for (int m = 0; m < 3; ++m) a.wall_u[f][m] = (R)P.wall_u[f][m];
    }
    for (int k = 0; k < 2; ++k) {
      const double nu = (P.tau[k] - 0.5) / 3.0;
      a.omega[k] = (R)((1.0 / 3.0) / (nu + 0.5 / 3.0));
      a.cum[k] = P.collision[k] == LSB_CUMULANT;
      for (int m = 0; m < 3; ++m) a.acc[k][m] = (R)P.accel[k][m];
      a.rho_phys[k] = (R)P.rho_phys[k];
      a.eta[k] = (R)(P.rho_phys[k] * nu);
    }
    a.sigma = (R)P.sigma;
    {
      // interface-coupling constants: the pressure jump's divisor is the
      // mean viscosity where eta_bar >= rho_max / 24 (the lagged pressure
      // feedback then has gain <= 1), else rho_max cs^2 / 4 = rho_max / 12
      // (gain <= 1/2), see iface_pull
      const double eta_bar = 0.5 * (P.rho_phys[0] * (P.tau[0] - 0.5) / 3.0 + P.rho_phys[1] * (P.tau[1] - 0.5) / 3.0);
      const double rmax = P.rho_phys[0] > P.rho_phys[1] ? P.rho_phys[0] : P.rho_phys[1];
      const double eta_p = eta_bar >= rmax / 24.0 ? eta_bar : rmax / 12.0;
      for (int k = 0; k < 2; ++k) a.iface_pc[k] = (R)(P.rho_phys[k] / 3.0);
      a.iface_inv2etap = (R)(1.0 / (2.0 * eta_p));
      a.iface_acoef = (R)(-((double)a.eta[1] - (double)a.eta[0]) / eta_bar);
    }
    a.band = (R)P.band;
    a.band_snap = (R)(P.band - kBandSnap);
    a.ext_dtau = (R)P.ext_dtau;
    a.reinit_dtau = (R)P.reinit_dtau;
    a.heps = (R)P.heaviside_eps;
    a.scale = ST == LSB_F16DEV ? (R)ldexp(1.0, P.fp16_scale_log2) : (R)1;
    a.inv_scale = ST == LSB_F16DEV ? (R)ldexp(1.0, -P.fp16_scale_log2) : (R)1;
    for (int k = 0; k < 2; ++k) {
      const bool dev16 = ST == LSB_F16DEV || ST == LSB_BF16DEV;
      a.rho_ref[k] = dev16 ? (R)p->rho_ref[k] : (R)1;
      a.rref_m1[k] = (R)((double)a.rho_ref[k] - 1.0);
    }
    a.use_pb = P.use_pb;
    for (int ax = 0; ax < 3; ++ax) { a.tdim[ax] = p->tdim[ax]; a.ntile[ax] = p->ntile[ax]; }
    a.ntiles = p->ntiles;
    char* w = p->ws;
    a.A = reinterpret_cast<const T*>(w + p->off_A[cur]);
    a.An = reinterpret_cast<T*>(w + p->off_A[cur ^ 1]);
    a.phi = reinterpret_cast<R*>(w + p->off_phi);
    a.s1 = reinterpret_cast<R*>(w + p->off_s1);
    a.s2 = reinterpret_cast<R*>(w + p->off_s2);
    a.p0 = reinterpret_cast<R*>(w + p->off_p0);
    a.tag = reinterpret_cast<uint8_t*>(w + p->off_tag);
    a.aux = reinterpret_cast<uint8_t*>(w + p->off_aux);
    a.M = reinterpret_cast<const R*>(w + p->off_M[cur]);
    a.Mn = reinterpret_cast<R*>(w + p->off_M[cur ^ 1]);
    a.G = reinterpret_cast<R*>(w + p->off_G);
    a.ut_a = reinterpret_cast<R*>(w + p->off_ut[0]);
    a.ut_b = reinterpret_cast<R*>(w + p->off_ut[1]);
    a.ext_k = reinterpret_cast<R*>(w + p->off_ext_k);
    a.irec = reinterpret_cast<R*>(w + p->off_irec);
    a.blab = reinterpret_cast<int*>(w + p->off_blab);
    a.pbc = reinterpret_cast<R*>(w + p->off_pbc);
    a.broots = reinterpret_cast<int*>(w + p->off_broots);
    a.bpart = reinterpret_cast<double*>(w + p->off_bpart);
    a.bres = reinterpret_cast<double*>(w + p->off_bres);
    a.scal = reinterpret_cast<double*>(w + p->off_scal);
    a.counters = reinterpret_cast<int*>(w + p->off_cnt);
    a.tile_act = reinterpret_cast<uint8_t*>(w + (p->tcur ? p->off_tile_act2 : p->off_tile_act));
    a.tile_act_next = reinterpret_cast<uint8_t*>(w + (p->tcur ? p->off_tile_act : p->off_tile_act2));
    a.cand_next = reinterpret_cast<uint8_t*>(w + p->off_cflag[p->nstep & 1]);
    a.cand_prev = reinterpret_cast<uint8_t*>(w + p->off_cflag[(p->nstep + 1) & 1]);
    a.tile_list = reinterpret_cast<int*>(w + p->off_tile_list);
    a.cand_list = reinterpret_cast<int*>(w + p->off_cand_list);
    a.spec_list = reinterpret_cast<int*>(w + p->off_spec_list);
    a.flip_list = reinterpret_cast<int*>(w + p->off_flip_list);
    a.wall_list = reinterpret_cast<int*>(w + p->off_wall_list);
    a.partial = reinterpret_cast<double*>(w + p->off_partial);
    a.ghost = reinterpret_cast<const R*>(w + p->off_ghost);
    return a;
  }

  static int cell_grid(const lsb_plan* p) {
    long g = ((long)p->N + 255) / 256;
    return (int)(g < 8192 ? g : 8192);
  }

  // Classification of all tiles (initialisation and state reload), then the
  // candidate tiles around the resulting band, recorded as those of the
  // previous step (the next step's band collide-stream takes them).
  static void classify_all(lsb_plan* p, hipStream_t st) {
    Args a = args(p, p->cur);
    k_reset_counters<LAT, ST><<<1, 256, 0, st>>>(a, 0, CNT_WALL);
    k_dilate<LAT, ST><<<(p->ntiles + 255) / 256, 256, 0, st>>>(a, 1);
    k_classify<LAT, ST><<<p->grid_tiles, 256, 0, st>>>(a, 0);
    k_geometry<LAT, ST><<<p->grid_tiles, 256, 0, st>>>(a);
    p->tcur ^= 1;
    Args b = args(p, p->cur);
    b.cand_next = b.cand_prev;
    k_reset_counters<LAT, ST><<<1, 256, 0, st>>>(b, CNT_CAND, 1);
    k_dilate<LAT, ST><<<(p->ntiles + 255) / 256, 256, 0, st>>>(b, 0);
  }

  static void centroid(lsb_plan* p, int mode, hipStream_t st) {
    Args a = args(p, p->cur);
    k_centroid_partial<LAT, ST><<<p->red_blocks, 256, 0, st>>>(a);
    const lsb_params& P = p->P;
    k_centroid_final<LAT, ST><<<1, 256, 0, st>>>(a, p->red_blocks, mode, P.pb0, P.rho_phys[0], P.accel[0][0],
                                                 P.accel[0][1], P.accel[0][2]);
  }

  static void init_phi(lsb_plan* p, const double* phi0, int c0, int c1, hipStream_t st) {
    p->cur = 0;
    Args a = args(p, 0);
    const int g = (int)(((long)(c1 - c0) + 255) / 256 < 8192 ? ((long)(c1 - c0) + 255) / 256 : 8192);
    k_init_phi<LAT, ST><<<g > 0 ? g : 1, 256, 0, st>>>(a, phi0, c0, c1);
  }

  static void init_band(lsb_plan* p, hipStream_t st) {
    Args a = args(p, p->cur);
    k_clear_tiles<LAT, ST><<<(p->ntiles + 255) / 256, 256, 0, st>>>(a);
    k_reset_counters<LAT, ST><<<1, 256, 0, st>>>(a, 0, CNT_NUM);
    classify_all(p, st);
    k_mark_walls<LAT, ST><<<cell_grid(p), 256, 0, st>>>(a);
    centroid(p, 0, st);
    k_set_scalar<LAT, ST><<<1, 1, 0, st>>>(a, SC_PB, p->P.pb0);
    if (p->P.use_pb == 2) bubbles(p, st);
  }

  // Several bubbles: label the components of the Heaviside support, their
  // volumes, centroids and baselines, and the baseline field.
  static void bubbles(lsb_plan* p, hipStream_t st) {
    Args a = args(p, p->cur);
    const lsb_params& P = p->P;
    const int g = cell_grid(p);
    k_reset_counters<LAT, ST><<<1, 256, 0, st>>>(a, CNT_BUB, 1);
    k_bub_init<LAT, ST><<<g, 256, 0, st>>>(a);
    k_bub_union<LAT, ST><<<g, 256, 0, st>>>(a);
    k_bub_roots<LAT, ST><<<g, 256, 0, st>>>(a);
    k_bub_sort<LAT, ST><<<1, 64, 0, st>>>(a);
    k_bub_number<LAT, ST><<<g, 256, 0, st>>>(a);
    k_bub_partial<LAT, ST><<<kBubbleParts, 256, 0, st>>>(a);
    k_bub_final<LAT, ST><<<kMaxBubbles, 256, 0, st>>>(a, kBubbleParts, P.pb0, P.rho_phys[0], P.accel[0][0],
                                                     P.accel[0][1], P.accel[0][2]);
    k_bub_field<LAT, ST><<<g, 256, 0, st>>>(a);
  }

  // populations and both moment buffers of the current state (buffer 0)
  static void init_pop(lsb_plan* p, const double* rho0, const double* u0, int c0, int c1, hipStream_t st) {
    Args b = args(p, 1);  // b.An == buffer 0, b.M == buffer 1, b.Mn == buffer 0
    const int g = (int)(((long)(c1 - c0) + 255) / 256 < 8192 ? ((long)(c1 - c0) + 255) / 256 : 8192);
    k_init_pop<LAT, ST><<<g > 0 ? g : 1, 256, 0, st>>>(b, rho0, u0, p->P.init_hydrostatic, c0, c1);
  }

  // bulk collide-stream launch (with or without the body-force terms).  The
  // FP32-storage kernel reserves 32 KB of LDS per block it does not use: that
  // holds it at five blocks per CU, where its 54 streams run at 5.4 TB/s
  // against 4.7 TB/s at the full eight (measured); FP16 runs at seven (its
  // 66 registers; forcing eight spills and is 2.7% slower, holding it at six
  // or five is slower too), FP64 is held at four by its registers.
  // With wall faces in x (3D) the kernel also takes the x-face cells
  // (XW, T_XWALL).
  template <bool SPLIT, bool CUM, bool XW>
  static void bulk_launch(const Args& a, bool force, unsigned g, size_t dyn, int xchunks, hipStream_t st) {
    if (force) k_lb_bulk<LAT, ST, SPLIT, true, CUM, XW><<<g, 256, dyn, st>>>(a, xchunks);
    else k_lb_bulk<LAT, ST, SPLIT, false, CUM, XW><<<g, 256, dyn, st>>>(a, xchunks);
  }
  static bool xwall(const Args& a) { return LAT != LSB_D2Q9 && !a.per[0] && a.bcf[0] != kFaceInject; }
  template <bool SPLIT>
  static void bulk(const Args& a, bool force, int xchunks, int rows, hipStream_t st) {
    // whole 256-cell row chunks when nx allows, else consecutive cells
    if (xchunks * 256 != a.nx) xchunks = 0;
    const unsigned g = xchunks ? (unsigned)(xchunks * rows) : (unsigned)(((long)a.N + 255) / 256);
    const size_t dyn = ST == LSB_F32 ? 32768 : 0;
    const bool xw = xwall(a);
    if constexpr (LAT == LSB_D3Q27) {
      if (a.cum[0] || a.cum[1]) {
        if (xw) bulk_launch<SPLIT, true, true>(a, force, g, dyn, xchunks, st);
        else bulk_launch<SPLIT, true, false>(a, force, g, dyn, xchunks, st);
        return;
      }
    }
    if constexpr (LAT != LSB_D2Q9) {
      if (xw) {
        bulk_launch<SPLIT, false, true>(a, force, g, dyn, xchunks, st);
        return;
      }
    }
    bulk_launch<SPLIT, false, false>(a, force, g, dyn, xchunks, st);
  }

  // wall-adjacent cells: the two z planes streamed (k_lb_zwall) where the
  // only walls are no-slip z faces and rows are whole chunks, else the list
  static void walls(lsb_plan* p, const Args& a, bool cum, bool force, hipStream_t st) {
    if (p->n_wall_cells <= 0) return;
    if constexpr (LAT != LSB_D2Q9) {
      const int xchunks = a.nx / 256;
      if (a.per[0] && a.per[1] && !a.per[2] && a.bcf[4] == LSB_NOSLIP && a.bcf[5] == LSB_NOSLIP &&
          xchunks * 256 == a.nx) {
        const unsigned g = (unsigned)(xchunks * 2 * a.ny);
        if (cum) {
          if (force) k_lb_zwall<LAT, ST, true, true><<<g, 256, 0, st>>>(a, xchunks);
          else k_lb_zwall<LAT, ST, false, true><<<g, 256, 0, st>>>(a, xchunks);
        } else {
          if (force) k_lb_zwall<LAT, ST, true, false><<<g, 256, 0, st>>>(a, xchunks);
          else k_lb_zwall<LAT, ST, false, false><<<g, 256, 0, st>>>(a, xchunks);
        }
        return;
      }
    }
    if (cum) k_lb_wall<LAT, ST, true><<<p->grid_walls, 256, 0, st>>>(a);
    else k_lb_wall<LAT, ST, false><<<p->grid_walls, 256, 0, st>>>(a);
  }

  // copy of a step intermediate into the snapshot slot being recorded
  static void rec(lsb_plan* p, size_t off, const void* src, size_t bytes, hipStream_t st) {
    char* d = p->adj.ws + p->adj.o_snap + (size_t)p->adj.rec_slot * p->adj.stride + off;
    (void)hipMemcpyAsync(d, src, bytes, hipMemcpyDeviceToDevice, st);
  }

  // One step.  Serial schedule: the collide-stream (bulk, interface, walls)
  // and then the level-set chain, all on the caller's stream st.  Overlap
  // schedule: the library's side stream runs the bulk collide-stream of the
  // cells outside the previous step's candidate tiles; it needs only the
  // populations of the previous step's band, interface and wall parts and
  // its own previous launch, so it runs concurrently with the previous
  // step's level-set chain and with this step's band part.  The caller's
  // stream runs the band collide-stream (candidate tiles), the interface and
  // wall cells and the level-set chain.  Events order the two streams.
  static void step(lsb_plan* p, hipStream_t st) {
    const lsb_params& P = p->P;
    Args a = args(p, p->cur);
    const int xchunks = (P.nx + 255) / 256;
    const int rows = P.ny * P.nz;
    bool force = false;  // any body acceleration: the bulk launch with force terms
    for (int k = 0; k < 2; ++k)
      for (int m = 0; m < 3; ++m) force = force || P.accel[k][m] != 0.0;
    // a phase with the cumulant operator: the collide-stream variants with it
    const bool cum = LAT == LSB_D3Q27 && (a.cum[0] || a.cum[1]);
    // the populations of the previous step are complete (bulk part included)
    (void)hipStreamWaitEvent(st, p->ev_bulk_done, 0);
    if (p->schedule == LSB_SCHED_OVERLAP) {
      (void)hipStreamWaitEvent(p->side, p->ev_pop_done, 0);
      timing_begin(p, p->side);
      bulk<true>(a, force, xchunks, rows, p->side);
      timing_end(p, p->side);
      (void)hipEventRecord(p->ev_bulk_done, p->side);
      const bool xw = xwall(a);
      if (cum) {
        if (xw) k_lb_band<LAT, ST, true, true><<<p->grid_tiles, 256, 0, st>>>(a);
        else k_lb_band<LAT, ST, true, false><<<p->grid_tiles, 256, 0, st>>>(a);
      } else {
        if (xw) k_lb_band<LAT, ST, false, true><<<p->grid_tiles, 256, 0, st>>>(a);
        else k_lb_band<LAT, ST, false, false><<<p->grid_tiles, 256, 0, st>>>(a);
      }
    } else {
      timing_begin(p, st);
      bulk<false>(a, force, xchunks, rows, st);
      timing_end(p, st);
    }
    // candidate tiles of this step's classification (dilation of the
    // current LS-active tiles); their flags bound the next bulk part
    k_reset_counters<LAT, ST><<<1, 256, 0, st>>>(a, CNT_CAND, 1);
    k_dilate<LAT, ST><<<(p->ntiles + 255) / 256, 256, 0, st>>>(a, 0);
    // grids below 2^25 cells: the interface kernel with lane groups for
    // short lists (bit-identical results)
    const bool lg = p->N < (1 << 25);
    if (cum) {
      if (lg) k_lb_iface<LAT, ST, true, true><<<p->grid_cells, 256, 0, st>>>(a);
      else k_lb_iface<LAT, ST, true, false><<<p->grid_cells, 256, 0, st>>>(a);
    } else {
      if (lg) k_lb_iface<LAT, ST, false, true><<<p->grid_cells, 256, 0, st>>>(a);
      else k_lb_iface<LAT, ST, false, false><<<p->grid_cells, 256, 0, st>>>(a);
    }
    walls(p, a, cum, force, st);
    (void)hipEventRecord(p->ev_pop_done, st);
    const bool recording = p->adj.rec_slot >= 0;
    const size_t rb = sizeof(R), N = (size_t)p->N;
    if (recording) rec(p, p->adj.s_Mn, a.Mn, 10 * N * rb, st);
    // a6: extension (ut ping-pong), advection
    k_ext_seed<LAT, ST><<<p->grid_tiles, 256, 0, st>>>(a);
    k_ext_seed_iface<LAT, ST><<<p->grid_cells, 256, 0, st>>>(a);
    R* ua = a.ut_a;
    R* ub = a.ut_b;
    if (recording) rec(p, p->adj.s_ut, ua, 3 * N * rb, st);
    for (int it = 0; it < P.n_ext; ++it) {
      Args e = a;
      e.ut_a = ua;
      e.ut_b = ub;
      k_ext_iter<LAT, ST><<<p->grid_tiles, 256, 0, st>>>(e);
      R* t = ua; ua = ub; ub = t;
      if (recording) rec(p, p->adj.s_ut + (size_t)(it + 1) * 3 * N * rb, ua, 3 * N * rb, st);
    }
    for (int stage = 1; stage <= 3; ++stage) k_rk3_stage<LAT, ST><<<p->grid_tiles, 256, 0, st>>>(a, stage, ua);
    if (recording) {
      rec(p, p->adj.s_s1, a.s1, N * rb, st);
      rec(p, p->adj.s_s2, a.s2, N * rb, st);
    }
    // a7: reinitialisation
    if (P.reinit_every > 0 && P.n_reinit > 0 && ((p->nstep + 1) % P.reinit_every) == 0) {
      // recording: the level set before the reinitialisation, then each
      // stage's input (phi of the pseudo step, s1, s2)
      if (recording) rec(p, p->adj.s_p0, a.phi, N * rb, st);
      k_reinit_prep<LAT, ST><<<p->grid_tiles, 256, 0, st>>>(a);
      for (int it = 0; it < P.n_reinit; ++it)
        for (int stage = 1; stage <= 3; ++stage) {
          if (recording) {
            const R* in = stage == 1 ? a.phi : (stage == 2 ? a.s1 : a.s2);
            rec(p, p->adj.s_rein + (size_t)(3 * it + stage - 1) * N * rb, in, N * rb, st);
          }
          k_reinit_stage<LAT, ST><<<p->grid_tiles, 256, 0, st>>>(a, stage, it == P.n_reinit - 1 ? 1 : 0);
        }
    }
    k_ls_sync<LAT, ST><<<p->grid_tiles, 256, 0, st>>>(a);
    // a8: classification on the candidate tiles, geometry, refill
    k_reset_counters<LAT, ST><<<1, 256, 0, st>>>(a, 0, CNT_CAND);
    k_classify<LAT, ST><<<p->grid_tiles, 256, 0, st>>>(a, 1);
    k_geometry<LAT, ST><<<p->grid_tiles, 256, 0, st>>>(a);
    k_refill<LAT, ST><<<p->grid_cells, 256, 0, st>>>(a);
    p->cur ^= 1;
    p->tcur ^= 1;
    // a9: centroid and gas pressure baseline (one, or one per bubble)
    if (P.use_pb == 2) bubbles(p, st);
    else if (P.use_pb) centroid(p, 1, st);
    pack(p, st);
    ++p->nstep;
  }

  static void fields(lsb_plan* p, double* rho, double* u, double* pr, uint8_t* ph, int c0, int c1, hipStream_t st) {
    k_fields<LAT, ST><<<cell_grid(p), 256, 0, st>>>(args(p, p->cur), rho, u, pr, ph, c0, c1);
  }
  static void populations(lsb_plan* p, double* out, int i0, int i1, int c0, int c1, hipStream_t st) {
    k_populations<LAT, ST><<<cell_grid(p), 256, 0, st>>>(args(p, p->cur), out, i0, i1, c0, c1);
  }
  static void interface(lsb_plan* p, double* phi, double* nrm, double* kap, uint8_t* tags, int c0, int c1,
                        hipStream_t st) {
    k_export_interface<LAT, ST><<<cell_grid(p), 256, 0, st>>>(args(p, p->cur), phi, nrm, kap, tags, c0, c1);
  }
  static void moments(lsb_plan* p, double* out, int c0, int c1, hipStream_t st) {
    k_export_moments<LAT, ST><<<cell_grid(p), 256, 0, st>>>(args(p, p->cur), out, c0, c1);
  }
  static void integrals_partial(lsb_plan* p, double* partial, hipStream_t st) {
    Args a = args(p, p->cur);
    if (partial) a.partial = partial;
    k_integrals_partial<LAT, ST><<<p->red_blocks, 256, 0, st>>>(a);
  }
  // interface records of the current state (read by the next collide-stream)
  static void pack(lsb_plan* p, hipStream_t st) {
    k_pack_iface<LAT, ST><<<p->grid_cells, 256, 0, st>>>(args(p, p->cur));
  }

  static void rebuild(lsb_plan* p, hipStream_t st) {
    Args a = args(p, p->cur);
    k_clear_tiles<LAT, ST><<<(p->ntiles + 255) / 256, 256, 0, st>>>(a);
    k_reset_counters<LAT, ST><<<1, 256, 0, st>>>(a, 0, CNT_NUM);
    classify_all(p, st);
    k_mark_walls<LAT, ST><<<cell_grid(p), 256, 0, st>>>(a);
    if (p->P.use_pb == 2) bubbles(p, st);
  }

  static const Ops* table() {
    static const Ops ops = {init_phi, init_band, init_pop, step, fields, populations, interface, moments,
                            integrals_partial, rebuild, pack};
    return &ops;
  }
};

}  // namespace lsb

#define LSB_DEFINE_OPS(NAME, LAT)                                   \
  namespace lsb {                                                   \
  const Ops* NAME(int storage) {                                    \
    switch (storage) {                                              \
      case LSB_F64: return Driver<LAT, LSB_F64>::table();           \
      case LSB_F32: return Driver<LAT, LSB_F32>::table();           \
      case LSB_F16DEV: return Driver<LAT, LSB_F16DEV>::table();     \
      case LSB_BF16DEV: return Driver<LAT, LSB_BF16DEV>::table();   \
      default: return nullptr;                                      \
    }                                                               \
  }                                                                 \
  }
