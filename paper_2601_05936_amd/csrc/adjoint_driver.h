// adjoint_driver.h -- host side of the reverse mode (D2Q9): recording a
// checkpoint segment with the forward kernels, the reverse step sequence and
// the reverse of the initialisation.
#pragma once

#include "adjoint.h"
#include "driver.h"

namespace lsb {

template <int ST>
struct AdjDriver {
  using F = Driver<LSB_D2Q9, ST>;
  using R = typename F::R;
  using T = typename F::T;
  using Args = typename F::Args;
  using V = adj::View<R>;
  static_assert(sizeof(T) == sizeof(R), "the adjoint needs FP64 or FP32 population storage");

  static char* slot(lsb_plan* p, int k) { return p->adj.ws + p->adj.o_snap + (size_t)k * p->adj.stride; }
  static double* dbl(lsb_plan* p, size_t off) { return reinterpret_cast<double*>(p->adj.ws + off); }
  static double* sc(lsb_plan* p) { return dbl(p, p->adj.o_scal); }
  static int grid(const lsb_plan* p) {
    const int g = (p->N + 255) / 256;
    return g < 4096 ? g : 4096;
  }
  static int grid_units(const lsb_plan* p) { return adj::unit_blocks(p->N); }

  // state of the current step (before it runs) into snapshot slot k
  static void snapshot_state(lsb_plan* p, int k, hipStream_t st) {
    const AdjState& s = p->adj;
    char* d = slot(p, k);
    const size_t N = (size_t)p->N, rb = p->bytes_real;
    // one launch for the six arrays (six copies cost six launches)
    adj::CopySet z{};
    const std::pair<size_t, size_t> from[6] = {{p->off_A[p->cur], s.s_A}, {p->off_M[p->cur], s.s_M},
                                               {p->off_phi, s.s_phi},     {p->off_G, s.s_G},
                                               {p->off_tag, s.s_tag},     {p->off_scal, s.s_scal}};
    const size_t bytes[6] = {p->pop_bytes, 10 * N * rb, N * rb, 4 * N * rb, N, SC_COUNT * sizeof(double)};
    for (int j = 0; j < 6; ++j) {
      z.src[j] = p->ws + from[j].first;
      z.dst[j] = d + from[j].second;
      z.bytes[j] = (long)bytes[j];
    }
    z.count = 6;
    adj::k_copy_set<<<grid(p), 256, 0, st>>>(z);
  }

  static void record(lsb_plan* p, int nsteps, hipStream_t st) {
    const int sched = p->schedule;
    const lsb_params& P = p->P;
    p->schedule = LSB_SCHED_SERIAL;
    p->adj.reinit_at.assign((size_t)nsteps, 0);
    for (int k = 0; k < nsteps; ++k) {
      snapshot_state(p, k, st);
      p->adj.reinit_at[k] = P.reinit_every > 0 && P.n_reinit > 0 && ((p->nstep + 1) % P.reinit_every) == 0;
      p->adj.rec_slot = k;
      F::step(p, st);
      p->adj.rec_slot = -1;
    }
    snapshot_state(p, nsteps, st);
    p->adj.nrec = nsteps;
    p->schedule = sched;
  }

  static V view(lsb_plan* p, int n) {
    const AdjState& s = p->adj;
    const Args a = F::args(p, p->cur);
    V v{};
    char* s0 = slot(p, n);
    char* s1 = slot(p, n + 1 <= s.nrec ? n + 1 : n);
    v.val[adj::AR_AIN] = reinterpret_cast<const R*>(s0 + s.s_A);
    v.val[adj::AR_MIN] = reinterpret_cast<const R*>(s0 + s.s_M);
    v.val[adj::AR_PHI0] = reinterpret_cast<const R*>(s0 + s.s_phi);
    v.val[adj::AR_GIN] = reinterpret_cast<const R*>(s0 + s.s_G);
    v.val[adj::AR_MNEW] = reinterpret_cast<const R*>(s0 + s.s_Mn);
    v.val[adj::AR_ANEW] = reinterpret_cast<const R*>(s1 + s.s_A);
    v.val[adj::AR_PHI1] = reinterpret_cast<const R*>(s1 + s.s_phi);
    v.val[adj::AR_GNEW] = reinterpret_cast<const R*>(s1 + s.s_G);
    v.val[adj::AR_S1] = reinterpret_cast<const R*>(s0 + s.s_s1);
    v.val[adj::AR_S2] = reinterpret_cast<const R*>(s0 + s.s_s2);
    v.sval[adj::AR_PB] = reinterpret_cast<const double*>(s0 + s.s_scal) + SC_PB;
    v.sval[adj::AR_XC0] = reinterpret_cast<const double*>(s0 + s.s_scal) + SC_XC0;
    v.sval[adj::AR_SIG] = sc(p) + AdjState::SC_SIGMA;
    v.tag0 = reinterpret_cast<const uint8_t*>(s0 + s.s_tag);
    v.tag1 = reinterpret_cast<const uint8_t*>(s1 + s.s_tag);
    v.nx = a.nx; v.ny = a.ny; v.nz = a.nz; v.N = a.N;
    for (int m = 0; m < 3; ++m) v.per[m] = a.per[m];
    for (int f = 0; f < 6; ++f) {
      v.bcf[f] = a.bcf[f];
      for (int m = 0; m < 3; ++m) v.wall_u[f][m] = (double)a.wall_u[f][m];
    }
    for (int k = 0; k < 2; ++k) {
      v.omega[k] = (double)a.omega[k];
      v.rho_phys[k] = (double)a.rho_phys[k];
      v.eta[k] = (double)a.eta[k];
      for (int m = 0; m < 3; ++m) v.acc[k][m] = (double)a.acc[k][m];
    }
    v.band = (double)a.band;
    v.band_snap = (double)a.band_snap;
    v.ext_dtau = (double)a.ext_dtau;
    v.reinit_dtau = (double)a.reinit_dtau;
    v.heps = (double)a.heps;
    // adjoint roles: index r holds the adjoint of step n + 1's state, r ^ 1
    // receives that of step n
    const int r = s.role;
    v.bar[adj::AR_AIN] = dbl(p, s.o_Abar[r ^ 1]);
    v.bar[adj::AR_MIN] = dbl(p, s.o_Mbar[r ^ 1]);
    v.bar[adj::AR_PHI0] = dbl(p, s.o_phibar[r ^ 1]);
    v.bar[adj::AR_GIN] = dbl(p, s.o_Gbar[r ^ 1]);
    v.bar[adj::AR_PB] = sc(p) + AdjState::SC_PBBAR + (r ^ 1);
    v.bar[adj::AR_SIG] = sc(p) + AdjState::SC_SIGBAR;
    v.bar[adj::AR_XC0] = sc(p) + AdjState::SC_XC0BAR;
    v.bar[adj::AR_MNEW] = dbl(p, s.o_Mbar[r]);
    v.bar[adj::AR_ANEW] = dbl(p, s.o_Abar[r]);
    v.bar[adj::AR_PHI1] = dbl(p, s.o_phibar[r]);
    v.bar[adj::AR_GNEW] = dbl(p, s.o_Gbar[r]);
    v.bar[adj::AR_S1] = dbl(p, s.o_s1bar);
    v.bar[adj::AR_S2] = dbl(p, s.o_s2bar);
    return v;
  }

  static void zero(lsb_plan* p, size_t off, long n, hipStream_t st) {
    adj::k_zero<<<grid(p), 256, 0, st>>>(dbl(p, off), n);
  }

  // up to ZeroSet::kMax workspace arrays (offset, length) cleared in one launch
  static void zero_set(lsb_plan* p, std::initializer_list<std::pair<size_t, long>> arrays, hipStream_t st) {
    adj::ZeroSet z{};
    for (const auto& a : arrays) {
      z.p[z.count] = dbl(p, a.first);
      z.n[z.count] = a.second;
      ++z.count;
    }
    adj::k_zero_set<<<grid(p), 256, 0, st>>>(z);
  }

  static void zero_all(lsb_plan* p, hipStream_t st) {
    const AdjState& s = p->adj;
    const long N = p->N;
    for (int r = 0; r < 2; ++r) {
      zero(p, s.o_Abar[r], 9 * N, st);
      zero(p, s.o_Mbar[r], 10 * N, st);
      zero(p, s.o_phibar[r], N, st);
      zero(p, s.o_Gbar[r], 4 * N, st);
      zero(p, s.o_utbar[r], 3 * N, st);
    }
    zero(p, s.o_s1bar, N, st);
    zero(p, s.o_s2bar, N, st);
    adj::k_zero<<<1, 256, 0, st>>>(sc(p), AdjState::SC_NUM);
  }

  static void seed_centroid(lsb_plan* p, int axis, hipStream_t st) {
    const AdjState& s = p->adj;
    p->adj.role = 0;
    zero_all(p, st);
    const R* phi = reinterpret_cast<const R*>(slot(p, s.nrec) + s.s_phi);
    const double eps = p->P.heaviside_eps;
    adj::k_set_sigma<<<1, 1, 0, st>>>(sc(p) + AdjState::SC_SIGMA, p->P.sigma);
    adj::k_centroid1<R><<<1, 256, 0, st>>>(phi, p->P.nx, p->N, eps, sc(p) + AdjState::SC_XC, sc(p) + AdjState::SC_V);
    adj::k_set_unit<<<1, 1, 0, st>>>(sc(p) + AdjState::SC_W, axis);
    adj::k_centroid_adj<R><<<grid(p), 256, 0, st>>>(phi, dbl(p, s.o_phibar[0]), p->P.nx, p->N, eps,
                                                     sc(p) + AdjState::SC_XC, sc(p) + AdjState::SC_V,
                                                     sc(p) + AdjState::SC_W);
  }

  static void reverse_step(lsb_plan* p, int n, hipStream_t st) {
    AdjState& s = p->adj;
    const long N = p->N;
    const int r = s.role;
    const int g = grid(p), gu = grid_units(p);
    int* flag = reinterpret_cast<int*>(sc(p) + AdjState::SC_FLAG);
    V v = view(p, n);
    char* s0 = slot(p, n);
    char* s1 = slot(p, n + 1);
    // gas-pressure baseline of step n + 1 (a function of the centroid of phi_{n+1})
    if (p->P.use_pb) {
      adj::k_pb_weights<<<1, 1, 0, st>>>(sc(p) + AdjState::SC_PBBAR + r, p->P.rho_phys[0], p->P.accel[0][0],
                                         p->P.accel[0][1], sc(p) + AdjState::SC_W, sc(p) + AdjState::SC_XC0BAR);
      const double* s1sc = reinterpret_cast<const double*>(s1 + s.s_scal);
      adj::k_centroid_adj<R><<<g, 256, 0, st>>>(reinterpret_cast<const R*>(s1 + s.s_phi), dbl(p, s.o_phibar[r]),
                                                 p->P.nx, p->N, p->P.heaviside_eps, s1sc + SC_XC, s1sc + SC_V,
                                                 sc(p) + AdjState::SC_W);
    }
    adj::k_zero<<<1, 1, 0, st>>>(sc(p) + AdjState::SC_PBBAR + r, 1);
    // refill (cells whose phase changed), geometry of the new band
    adj::k_refill_take<R><<<g, 256, 0, st>>>(v, dbl(p, s.o_ytmp));
    adj::k_refill_adj<R><<<gu, 256, 0, st>>>(v, dbl(p, s.o_ytmp), flag);
    adj::k_geometry_adj<R><<<gu, 256, 0, st>>>(v, 1, adj::AR_PHI1, dbl(p, s.o_Gbar[r]), flag);
    // reinitialisation (on the steps that ran one)
    if (s.reinit_at[n]) reverse_reinit(p, n, v, st);
    // TVD-RK3 stages, velocity of the last extension sweep
    const size_t lvl = 3 * N * p->bytes_real;
    const int ne = p->P.n_ext;
    int u = 0;
    v.val[adj::AR_UTOUT] = reinterpret_cast<const R*>(s0 + s.s_ut + (size_t)ne * lvl);
    v.bar[adj::AR_UTOUT] = dbl(p, s.o_utbar[u]);
    adj::k_rk_adj<R><<<gu, 256, 0, st>>>(v, 3, dbl(p, s.o_phibar[r]), flag);
    adj::k_rk_adj<R><<<gu, 256, 0, st>>>(v, 2, dbl(p, s.o_s2bar), flag);
    adj::k_rk_adj<R><<<gu, 256, 0, st>>>(v, 1, dbl(p, s.o_s1bar), flag);
    // extension sweeps, last to first
    for (int k = ne; k >= 1; --k) {
      v.val[adj::AR_UTOUT] = reinterpret_cast<const R*>(s0 + s.s_ut + (size_t)k * lvl);
      v.bar[adj::AR_UTOUT] = dbl(p, s.o_utbar[u]);
      v.val[adj::AR_UT] = reinterpret_cast<const R*>(s0 + s.s_ut + (size_t)(k - 1) * lvl);
      v.bar[adj::AR_UT] = dbl(p, s.o_utbar[u ^ 1]);
      adj::k_sweep_adj<R><<<gu, 256, 0, st>>>(v, flag);  // clears utbar[u]
      u ^= 1;
    }
    // extension seed
    v.val[adj::AR_UTOUT] = reinterpret_cast<const R*>(s0 + s.s_ut);
    v.bar[adj::AR_UTOUT] = dbl(p, s.o_utbar[u]);
    adj::k_seed_adj<R><<<gu, 256, 0, st>>>(v, flag);  // clears utbar[u]
    // collide-stream with wall and interface bounce-back
    adj::k_collide_adj_plain<R><<<g, 256, 0, st>>>(v);
    adj::k_collide_adj<R><<<gu, 256, 0, st>>>(v, flag);
    // the adjoint of step n + 1's state is consumed
    zero_set(p, {{s.o_Abar[r], 9 * N}, {s.o_Mbar[r], 10 * N}, {s.o_phibar[r], N}, {s.o_Gbar[r], 4 * N},
                 {s.o_s1bar, N}, {s.o_s2bar, N}}, st);
    s.role = r ^ 1;
  }

  // Reverse of the reinitialisation of step n: pseudo steps last to first,
  // stages 3, 2, 1.  On entry phibar[role] holds the adjoint of its output
  // (phi_{n+1}); on return, on the LS-active cells, the adjoint of its
  // input (the level set after the advection).
  static void reverse_reinit(lsb_plan* p, int n, V v, hipStream_t st) {
    AdjState& s = p->adj;
    const long N = p->N;
    const int r = s.role;
    const int gu = grid_units(p);
    int* flag = reinterpret_cast<int*>(sc(p) + AdjState::SC_FLAG);
    char* s0 = slot(p, n);
    const size_t lvl = (size_t)N * p->bytes_real;
    const int nr = p->P.n_reinit;
    v.val[adj::AR_P0] = reinterpret_cast<const R*>(s0 + s.s_p0);
    v.bar[adj::AR_P0] = dbl(p, s.o_p0bar);
    v.bar[adj::AR_RS1] = dbl(p, s.o_rs1bar);
    v.bar[adj::AR_RS2] = dbl(p, s.o_rs2bar);
    zero(p, s.o_p0bar, N, st);
    const double* ob = dbl(p, s.o_phibar[r]);
    int cur = 0;
    for (int k = nr - 1; k >= 0; --k) {
      const char* base = s0 + s.s_rein + (size_t)3 * k * lvl;
      v.val[adj::AR_RPHI] = reinterpret_cast<const R*>(base);
      v.val[adj::AR_RS1] = reinterpret_cast<const R*>(base + lvl);
      v.val[adj::AR_RS2] = reinterpret_cast<const R*>(base + 2 * lvl);
      v.bar[adj::AR_RPHI] = dbl(p, s.o_rphibar[cur]);
      zero_set(p, {{s.o_rphibar[cur], N}, {s.o_rs1bar, N}, {s.o_rs2bar, N}}, st);
      adj::k_reinit_adj<R><<<gu, 256, 0, st>>>(v, 3, k == nr - 1 ? 1 : 0, ob, flag);
      adj::k_reinit_adj<R><<<gu, 256, 0, st>>>(v, 2, 0, dbl(p, s.o_rs2bar), flag);
      adj::k_reinit_adj<R><<<gu, 256, 0, st>>>(v, 1, 0, dbl(p, s.o_rs1bar), flag);
      ob = dbl(p, s.o_rphibar[cur]);
      cur ^= 1;
    }
    adj::k_reinit_finish<<<grid(p), 256, 0, st>>>(v.tag0, ob, dbl(p, s.o_p0bar), dbl(p, s.o_phibar[r]), p->N);
  }

  static void reverse(lsb_plan* p, hipStream_t st) {
    for (int n = p->adj.nrec - 1; n >= 0; --n) reverse_step(p, n, st);
  }

  // reverse of the initialisation (the recorded segment starts at step 0)
  static void initial(lsb_plan* p, const double* phi0, const double* u0, int hydro, double* dphi0, hipStream_t st) {
    AdjState& s = p->adj;
    const int r = s.role;
    const int g = grid(p);
    int* flag = reinterpret_cast<int*>(sc(p) + AdjState::SC_FLAG);
    V v = view(p, 0);
    // the state of step 0 is the "current" adjoint (index r)
    v.bar[adj::AR_PHI0] = dbl(p, s.o_phibar[r]);
    v.bar[adj::AR_AIN] = dbl(p, s.o_Abar[r]);
    v.bar[adj::AR_MIN] = dbl(p, s.o_Mbar[r]);
    // geometry of the initial band
    adj::k_geometry_adj<R><<<grid_units(p), 256, 0, st>>>(v, 0, adj::AR_PHI0, dbl(p, s.o_Gbar[r]), flag);
    // hydrostatic initial density about the initial centroid
    if (hydro) {
      adj::k_init_pop_adj<R><<<AdjState::kInitBlocks, 256, 0, st>>>(v, u0, dbl(p, s.o_partial));
      adj::k_sum_partials<<<1, 1, 0, st>>>(dbl(p, s.o_partial), AdjState::kInitBlocks, sc(p) + AdjState::SC_XC0BAR);
    }
    // the initial centroid (reference of the gas-pressure baseline)
    const double* s0sc = reinterpret_cast<const double*>(slot(p, 0) + s.s_scal);
    adj::k_centroid_adj<R><<<g, 256, 0, st>>>(reinterpret_cast<const R*>(slot(p, 0) + s.s_phi), dbl(p, s.o_phibar[r]),
                                               p->P.nx, p->N, p->P.heaviside_eps, s0sc + SC_XC0, s0sc + SC_V,
                                               sc(p) + AdjState::SC_XC0BAR);
    adj::k_phi0_grad<<<g, 256, 0, st>>>(dbl(p, s.o_phibar[r]), phi0, p->P.band, p->N, dphi0);
  }

  static const AdjOps* table() {
    static const AdjOps ops = {record, seed_centroid, reverse, initial};
    return &ops;
  }
};

}  // namespace lsb
