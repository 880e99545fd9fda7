// api.hip -- implementation of the C ABI declared in include/lsb.h: parameter
// validation, workspace layout, host-pointer staging, dispatch to the
// (velocity set, storage) launch table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "plan.h"

namespace {
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define LSB_HIP(x)                                                                                    \
  do {                                                                                                \
    hipError_t e_ = (x);                                                                              \
    if (e_ != hipSuccess) return fail(LSB_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Staging area for host-pointer calls: the non-current population buffer,
// which the next step overwrites completely.
size_t staging_bytes(const lsb_plan* p) { return (size_t)p->Q * p->N * p->bytes_pop; }
char* staging(lsb_plan* p) { return p->ws + p->off_A[p->cur ^ 1]; }

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LSB_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return LSB_OK;
}
}  // namespace

namespace lsb {
void set_error(const std::string& msg) { g_err = msg; }

static const int kEventPairs = 512;

static void timing_flush(lsb_plan* p) {
  if (p->ev_used == 0) return;
  (void)hipEventSynchronize(p->ev[2 * (p->ev_used - 1) + 1]);
  for (int k = 0; k < p->ev_used; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev[2 * k], p->ev[2 * k + 1]) == hipSuccess) {
      p->timing_ms += ms;
      ++p->timing_launches;
    }
  }
  p->ev_used = 0;
}

void timing_begin(lsb_plan* p, hipStream_t st) {
  if (!p->timing) return;
  if (p->ev_used == kEventPairs) timing_flush(p);
  (void)hipEventRecord(p->ev[2 * p->ev_used], st);
}

void timing_end(lsb_plan* p, hipStream_t st) {
  if (!p->timing) return;
  (void)hipEventRecord(p->ev[2 * p->ev_used + 1], st);
  ++p->ev_used;
}
}  // namespace lsb

extern "C" {

const char* lsb_last_error(void) { return g_err.c_str(); }

int lsb_create(const lsb_params* P, lsb_plan** out) { return lsb::create_plan(P, false, out); }
}  // extern "C"

int lsb::create_plan(const lsb_params* P, bool allow_inject, lsb_plan** out) {
  if (!P || !out) return fail(LSB_EINVAL, "null argument");
  *out = nullptr;
  if (P->lattice < LSB_D2Q9 || P->lattice > LSB_D3Q27) return fail(LSB_EINVAL, "unknown lattice");
  if (P->storage < LSB_F64 || P->storage > LSB_BF16DEV) return fail(LSB_EINVAL, "unknown storage");
  if (P->lattice == LSB_D2Q9 && P->nz != 1) return fail(LSB_EINVAL, "D2Q9 needs nz == 1");
  if (P->nx < 4 || P->ny < 4 || (P->lattice != LSB_D2Q9 && P->nz < 4) || P->nz < 1)
    return fail(LSB_EINVAL, "grid must have at least 4 cells per used axis");
  if ((double)P->nx * P->ny * P->nz > 2147483647.0 / 2) return fail(LSB_EINVAL, "grid too large for 32-bit cell indices");
  for (int a = 0; a < 3; ++a) {
    for (int s = 0; s < 2; ++s)
      if ((P->bc[2 * a + s] < LSB_PERIODIC || P->bc[2 * a + s] > LSB_FREESLIP) &&
          !(allow_inject && P->bc[2 * a + s] == lsb::kFaceInject))
        return fail(LSB_EINVAL, "unknown face condition");
    if ((P->bc[2 * a] == LSB_PERIODIC) != (P->bc[2 * a + 1] == LSB_PERIODIC))
      return fail(LSB_EINVAL, "paired faces must both be periodic or both walls");
  }
  if (P->lattice == LSB_D2Q9 && P->bc[4] != LSB_PERIODIC) return fail(LSB_EINVAL, "2D grids need periodic z faces");
  if (!(P->tau[0] > 0.5) || !(P->tau[1] > 0.5)) return fail(LSB_EINVAL, "tau must exceed 1/2");
  if (P->use_pb < 0 || P->use_pb > 2) return fail(LSB_EINVAL, "use_pb must be 0, 1 or 2");
  for (int k = 0; k < 2; ++k) {
    if (P->collision[k] != LSB_BGK && P->collision[k] != LSB_CUMULANT)
      return fail(LSB_EINVAL, "unknown collision operator");
    if (P->collision[k] == LSB_CUMULANT && P->lattice != LSB_D3Q27)
      return fail(LSB_EINVAL, "the cumulant collision needs D3Q27");
  }
  if (!(P->rho_phys[0] > 0) || !(P->rho_phys[1] > 0)) return fail(LSB_EINVAL, "physical densities must be positive");
  if (!(P->band >= 2.0)) return fail(LSB_EINVAL, "band must be at least 2 cells");
  if (P->n_ext < 0 || P->n_reinit < 0 || P->reinit_every < 0) return fail(LSB_EINVAL, "negative iteration count");
  if (!(P->heaviside_eps > 0)) return fail(LSB_EINVAL, "heaviside_eps must be positive");
  if (P->storage == LSB_F16DEV && (P->fp16_scale_log2 < 0 || P->fp16_scale_log2 > 20))
    return fail(LSB_EINVAL, "fp16_scale_log2 out of range");

  lsb_plan* p = new lsb_plan();
  p->P = *P;
  p->D = P->lattice == LSB_D2Q9 ? 2 : 3;
  p->Q = P->lattice == LSB_D2Q9 ? 9 : (P->lattice == LSB_D3Q19 ? 19 : 27);
  p->N = P->nx * P->ny * P->nz;
  p->bytes_pop = P->storage == LSB_F64 ? 8 : (P->storage == LSB_F32 ? 4 : 2);
  p->bytes_real = P->storage == LSB_F64 ? 8 : 4;
  if (p->D == 2) {
    p->tdim[0] = lsb::TileShape<2>::X; p->tdim[1] = lsb::TileShape<2>::Y; p->tdim[2] = 1;
  } else {
    p->tdim[0] = lsb::TileShape<3>::X; p->tdim[1] = lsb::TileShape<3>::Y; p->tdim[2] = lsb::TileShape<3>::Z;
  }
  // the classification kernel stages a tile plus a one-cell halo in LDS
  if ((p->tdim[0] + 2) * (p->tdim[1] + 2) * (p->tdim[2] + (p->D == 3 ? 2 : 0)) > lsb::kClassifyLds) {
    delete p;
    return fail(LSB_EINVAL, "internal: tile too large for the classification kernel");
  }
  const int n[3] = {P->nx, P->ny, P->nz};
  p->ntiles = 1;
  for (int a = 0; a < 3; ++a) {
    p->ntile[a] = (n[a] + p->tdim[a] - 1) / p->tdim[a];
    p->ntiles *= p->ntile[a];
  }
  // one block per listed tile (blocks beyond the list length exit at once)
  p->grid_tiles = std::min(p->ntiles, 32768);
  p->grid_cells = (int)std::min<long>(((long)p->N + 255) / 256, 4096);
  p->red_blocks = 512;
  switch (P->lattice) {
    case LSB_D2Q9:
      p->ops = lsb::ops_d2q9(P->storage);
      p->adj_ops = lsb::adj_ops_d2q9(P->storage);
      break;
    case LSB_D3Q19: p->ops = lsb::ops_d3q19(P->storage); break;
    default: p->ops = lsb::ops_d3q27(P->storage); break;
  }
  // workspace layout
  const size_t N = (size_t)p->N;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  // populations: one array per direction in 2D, 256-cell chunks in 3D
  const size_t npop = P->lattice == LSB_D2Q9 ? N : (N + 255) / 256 * 256;
  p->pop_bytes = (size_t)p->Q * npop * p->bytes_pop;
  for (int b = 0; b < 2; ++b) p->off_A[b] = take(p->pop_bytes);
  p->off_phi = take(N * p->bytes_real);
  p->off_s1 = take(N * p->bytes_real);
  p->off_s2 = take(N * p->bytes_real);
  p->off_p0 = take(N * p->bytes_real);
  p->off_tag = take(N);
  p->off_aux = take(N);
  for (int b = 0; b < 2; ++b) p->off_M[b] = take(10 * N * p->bytes_real);
  p->off_G = take(4 * N * p->bytes_real);
  for (int b = 0; b < 2; ++b) p->off_ut[b] = take(3 * N * p->bytes_real);
  p->off_ext_k = take((size_t)3 * N * p->bytes_real);
  p->off_irec = take((size_t)16 * N * p->bytes_real);
  p->off_scal = take(lsb::SC_COUNT * sizeof(double));
  p->off_cnt = take(lsb::CNT_NUM * sizeof(int));
  p->off_tile_act = take((size_t)p->ntiles);
  p->off_tile_act2 = take((size_t)p->ntiles);
  p->off_cflag[0] = take((size_t)p->ntiles);
  p->off_cflag[1] = take((size_t)p->ntiles);
  p->off_tile_list = take((size_t)p->ntiles * sizeof(int));
  p->off_cand_list = take((size_t)p->ntiles * sizeof(int));
  p->off_spec_list = take(N * sizeof(int));
  p->off_flip_list = take(N * sizeof(int));
  p->off_partial = take((size_t)p->red_blocks * 16 * sizeof(double));
  {
    // several bubbles: labels, baseline field, roots, partial sums, results
    const bool nb = P->use_pb == 2;
    p->off_blab = take(nb ? N * sizeof(int) : 0);
    p->off_pbc = take(nb ? N * p->bytes_real : 0);
    p->off_broots = take(nb ? lsb::kMaxBubbles * sizeof(int) : 0);
    p->off_bpart = take(nb ? (size_t)lsb::kBubbleParts * lsb::kMaxBubbles * 4 * sizeof(double) : 0);
    p->off_bres = take(nb ? (size_t)lsb::kMaxBubbles * 5 * sizeof(double) : 0);
  }
  {
    long nw = 0;
    const long ax[3] = {P->nx, P->ny, P->nz};
    for (int d = 0; d < 3; ++d)
      if (P->bc[2 * d] != LSB_PERIODIC) nw += 2 * (ax[(d + 1) % 3] * ax[(d + 2) % 3]);
    p->n_wall_cells = nw;
    p->grid_walls = (int)std::max<long>(1, std::min<long>((nw + 255) / 256, 4096));
    p->off_wall_list = take((size_t)(nw + 1) * sizeof(int));
  }
  {
    bool inject = false;
    for (int f = 0; f < 6; ++f) inject = inject || P->bc[f] == lsb::kFaceInject;
    p->off_ghost = take(inject ? (size_t)p->Q * N * p->bytes_real : 0);
  }
  p->total = o;
  *out = p;
  return LSB_OK;
}

extern "C" {

void lsb_destroy(lsb_plan* p) {
  if (!p) return;
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  if (p->side) {
    (void)hipStreamSynchronize(p->side);
    (void)hipStreamDestroy(p->side);
  }
  if (p->ev_pop_done) (void)hipEventDestroy(p->ev_pop_done);
  if (p->ev_bulk_done) (void)hipEventDestroy(p->ev_bulk_done);
  delete p;
}

int lsb_workspace_bytes(const lsb_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(LSB_EINVAL, "null argument");
  *bytes = p->total;
  return LSB_OK;
}

int lsb_bind(lsb_plan* p, void* ws, size_t bytes) {
  if (!p || !ws) return fail(LSB_EINVAL, "null argument");
  if (bytes < p->total) return fail(LSB_ENOMEM, "workspace too small: need " + std::to_string(p->total) + " bytes");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(LSB_EINVAL, "workspace must be 256-byte aligned");
  p->ws = static_cast<char*>(ws);
  p->bound = true;
  p->inited = false;
  if (!p->side) {
    // side stream of the bulk collide-stream (default priority) and the two
    // events that order it against the caller's stream
    LSB_HIP(hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
    LSB_HIP(hipEventCreateWithFlags(&p->ev_pop_done, hipEventDisableTiming));
    LSB_HIP(hipEventCreateWithFlags(&p->ev_bulk_done, hipEventDisableTiming));
  }
  return LSB_OK;
}

int lsb_init(lsb_plan* p, const double* phi0, const double* rho0, const double* u0, int on_device, void* stream) {
  if (!p) return fail(LSB_EINVAL, "null plan");
  if (!p->bound) return fail(LSB_ESTATE, "lsb_init before lsb_bind");
  if (!phi0) return fail(LSB_EINVAL, "phi0 is required");
  hipStream_t st = as_stream(stream);
  const int N = p->N;
  p->cur = 0;
  p->tcur = 0;
  p->nstep = 0;
  LSB_HIP(hipStreamSynchronize(p->side));
  // stage host arrays through the (not yet used) second population buffer
  char* stg = p->ws + p->off_A[1];
  const size_t cap = staging_bytes(p);
  if (on_device) {
    p->ops->init_phi(p, phi0, 0, N, st);
    LSB_HIP(hipGetLastError());
  } else {
    const int chunk_phi = (int)std::min<size_t>(N, cap / sizeof(double));
    for (int c0 = 0; c0 < N; c0 += chunk_phi) {
      const int c1 = std::min(N, c0 + chunk_phi);
      LSB_HIP(hipMemcpyAsync(stg, phi0 + c0, (size_t)(c1 - c0) * sizeof(double), hipMemcpyHostToDevice, st));
      p->ops->init_phi(p, reinterpret_cast<double*>(stg), c0, c1, st);
      LSB_HIP(hipStreamSynchronize(st));
    }
  }
  p->ops->init_band(p, st);
  LSB_HIP(hipGetLastError());
  auto init_populations = [&]() -> int {
    if (on_device) {
      p->ops->init_pop(p, rho0, u0, 0, N, st);
      LSB_HIP(hipGetLastError());
      return LSB_OK;
    }
    const int chunk = (int)std::min<size_t>(N, cap / (4 * sizeof(double)));
    for (int c0 = 0; c0 < N; c0 += chunk) {
      const int c1 = std::min(N, c0 + chunk);
      double* r = reinterpret_cast<double*>(stg);
      double* u = r + (c1 - c0);
      if (rho0) LSB_HIP(hipMemcpyAsync(r, rho0 + c0, (size_t)(c1 - c0) * sizeof(double), hipMemcpyHostToDevice, st));
      if (u0) LSB_HIP(hipMemcpyAsync(u, u0 + 3 * (size_t)c0, 3 * (size_t)(c1 - c0) * sizeof(double), hipMemcpyHostToDevice, st));
      p->ops->init_pop(p, rho0 ? r : nullptr, u0 ? u : nullptr, c0, c1, st);
      LSB_HIP(hipStreamSynchronize(st));
    }
    return LSB_OK;
  };
  p->rho_ref[0] = p->rho_ref[1] = 1.0;
  if (int r = init_populations()) return r;
  if (p->P.storage == LSB_F16DEV || p->P.storage == LSB_BF16DEV) {
    // The codec's reference density of each phase: its mean initial LB
    // density (fixed reduction grid, so the value is deterministic); the
    // populations are initialised again in that frame.
    p->ops->integrals_partial(p, nullptr, st);
    LSB_HIP(hipGetLastError());
    std::vector<double> part((size_t)p->red_blocks * 16);
    LSB_HIP(hipMemcpyAsync(part.data(), p->ws + p->off_partial, part.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    LSB_HIP(hipStreamSynchronize(st));
    double mass[2] = {0, 0}, cnt[2] = {0, 0};
    for (int b = 0; b < p->red_blocks; ++b)
      for (int k = 0; k < 2; ++k) {
        mass[k] += part[16 * (size_t)b + k];
        cnt[k] += part[16 * (size_t)b + 11 + k];
      }
    for (int k = 0; k < 2; ++k) {
      // rounded to the FP32 arithmetic of the 16-bit storage modes, so that a
      // phase at density 1 keeps the frame of the rest state exactly
      const double m = cnt[k] > 0 ? (double)(float)(mass[k] / cnt[k]) : 1.0;
      p->rho_ref[k] = (std::isfinite(m) && m > 0) ? m : 1.0;
    }
    if (p->rho_ref[0] != 1.0 || p->rho_ref[1] != 1.0)
      if (int r = init_populations()) return r;
  }
  // the reference densities travel with the state image (scalar slots)
  LSB_HIP(hipMemcpyAsync(p->ws + p->off_scal + lsb::SC_RREF * sizeof(double), p->rho_ref, 2 * sizeof(double),
                         hipMemcpyHostToDevice, st));
  p->ops->pack(p, st);
  LSB_HIP(hipGetLastError());
  LSB_HIP(hipStreamSynchronize(st));
  LSB_HIP(hipEventRecord(p->ev_pop_done, st));
  LSB_HIP(hipEventRecord(p->ev_bulk_done, st));
  p->inited = true;
  return LSB_OK;
}

int lsb_get_integrals(lsb_plan* p, lsb_integrals* out, void* stream);

int lsb_step(lsb_plan* p, int nsteps, int check_every, void* stream) {
  if (!p) return fail(LSB_EINVAL, "null plan");
  if (!p->inited) return fail(LSB_ESTATE, "lsb_step before lsb_init");
  if (nsteps < 0) return fail(LSB_EINVAL, "negative step count");
  hipStream_t st = as_stream(stream);
  for (int s = 0; s < nsteps; ++s) {
    p->ops->step(p, st);
    // the caller's stream sees the whole step (bulk part included)
    if (p->schedule == LSB_SCHED_OVERLAP) LSB_HIP(hipStreamWaitEvent(st, p->ev_bulk_done, 0));
    if (int r = check_launch()) return r;
    if (check_every > 0 && (p->nstep % check_every) == 0) {
      lsb_integrals I;
      if (int r = lsb_get_integrals(p, &I, stream)) return r;
      double bad = 0;
      std::vector<double> part((size_t)p->red_blocks * 16);
      LSB_HIP(hipMemcpy(part.data(), p->ws + p->off_partial, part.size() * sizeof(double), hipMemcpyDeviceToHost));
      for (int b = 0; b < p->red_blocks; ++b) bad += part[16 * (size_t)b + 10];
      if (bad > 0 || !std::isfinite(I.mass[0]) || !std::isfinite(I.mass[1]))
        return fail(LSB_EUNSTABLE, "unstable state at step " + std::to_string(p->nstep));
    }
  }
  return LSB_OK;
}

int lsb_get_fields(lsb_plan* p, double* rho, double* u, double* pr, uint8_t* phase, int on_device, void* stream) {
  if (!p) return fail(LSB_EINVAL, "null plan");
  if (!p->inited) return fail(LSB_ESTATE, "no state");
  hipStream_t st = as_stream(stream);
  const int N = p->N;
  if (on_device) {
    p->ops->fields(p, rho, u, pr, phase, 0, N, st);
    return check_launch();
  }
  char* stg = staging(p);
  const size_t cap = staging_bytes(p);
  const int D = p->D;
  struct Part { int kind; void* host; size_t per_cell; };
  const Part parts[4] = {{0, rho, sizeof(double)}, {1, u, D * sizeof(double)}, {2, pr, sizeof(double)}, {3, phase, 1}};
  for (const Part& pt : parts) {
    if (!pt.host) continue;
    const int chunk = (int)std::min<size_t>(N, cap / pt.per_cell);
    for (int c0 = 0; c0 < N; c0 += chunk) {
      const int c1 = std::min(N, c0 + chunk);
      double* d = reinterpret_cast<double*>(stg);
      p->ops->fields(p, pt.kind == 0 ? d : nullptr, pt.kind == 1 ? d : nullptr, pt.kind == 2 ? d : nullptr,
                     pt.kind == 3 ? reinterpret_cast<uint8_t*>(stg) : nullptr, c0, c1, st);
      LSB_HIP(hipGetLastError());
      LSB_HIP(hipMemcpyAsync(static_cast<char*>(pt.host) + (size_t)c0 * pt.per_cell, stg, (size_t)(c1 - c0) * pt.per_cell,
                             hipMemcpyDeviceToHost, st));
      LSB_HIP(hipStreamSynchronize(st));
    }
  }
  return LSB_OK;
}

int lsb_get_interface(lsb_plan* p, double* phi, double* nrm, double* kap, uint8_t* tags, int on_device, void* stream) {
  if (!p) return fail(LSB_EINVAL, "null plan");
  if (!p->inited) return fail(LSB_ESTATE, "no state");
  hipStream_t st = as_stream(stream);
  const int N = p->N;
  if (on_device) {
    p->ops->interface(p, phi, nrm, kap, tags, 0, N, st);
    return check_launch();
  }
  char* stg = staging(p);
  const size_t cap = staging_bytes(p);
  const int D = p->D;
  struct Part { int kind; void* host; size_t per_cell; };
  const Part parts[4] = {{0, phi, sizeof(double)}, {1, nrm, D * sizeof(double)}, {2, kap, sizeof(double)}, {3, tags, 1}};
  for (const Part& pt : parts) {
    if (!pt.host) continue;
    const int chunk = (int)std::min<size_t>(N, cap / pt.per_cell);
    for (int c0 = 0; c0 < N; c0 += chunk) {
      const int c1 = std::min(N, c0 + chunk);
      double* d = reinterpret_cast<double*>(stg);
      p->ops->interface(p, pt.kind == 0 ? d : nullptr, pt.kind == 1 ? d : nullptr, pt.kind == 2 ? d : nullptr,
                        pt.kind == 3 ? reinterpret_cast<uint8_t*>(stg) : nullptr, c0, c1, st);
      LSB_HIP(hipGetLastError());
      LSB_HIP(hipMemcpyAsync(static_cast<char*>(pt.host) + (size_t)c0 * pt.per_cell, stg, (size_t)(c1 - c0) * pt.per_cell,
                             hipMemcpyDeviceToHost, st));
      LSB_HIP(hipStreamSynchronize(st));
    }
  }
  return LSB_OK;
}

int lsb_get_bubbles(lsb_plan* p, int max, int* count, double* out, int32_t* labels, int on_device, void* stream) {
  if (!p || !count) return fail(LSB_EINVAL, "null argument");
  if (!p->inited) return fail(LSB_ESTATE, "no state");
  if (p->P.use_pb != 2) return fail(LSB_EINVAL, "lsb_get_bubbles needs use_pb = 2");
  hipStream_t st = as_stream(stream);
  double nb = 0.0;
  LSB_HIP(hipMemcpyAsync(&nb, p->ws + p->off_scal + lsb::SC_NBUB * sizeof(double), sizeof(double),
                         hipMemcpyDeviceToHost, st));
  LSB_HIP(hipStreamSynchronize(st));
  const int n = (int)nb;
  *count = n;
  if (n > lsb::kMaxBubbles) return fail(LSB_EUNSTABLE, "more than LSB_MAX_BUBBLES bubbles");
  if (out && max > 0 && n > 0)
    LSB_HIP(hipMemcpyAsync(out, p->ws + p->off_bres, (size_t)std::min(n, max) * 5 * sizeof(double),
                           hipMemcpyDeviceToHost, st));
  if (labels)
    LSB_HIP(hipMemcpyAsync(labels, p->ws + p->off_blab, (size_t)p->N * sizeof(int32_t),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  LSB_HIP(hipStreamSynchronize(st));
  return LSB_OK;
}

int lsb_get_populations(lsb_plan* p, double* out, int on_device, void* stream) {
  if (!p || !out) return fail(LSB_EINVAL, "null argument");
  if (!p->inited) return fail(LSB_ESTATE, "no state");
  hipStream_t st = as_stream(stream);
  const int N = p->N;
  if (on_device) {
    p->ops->populations(p, out, 0, p->Q, 0, N, st);
    return check_launch();
  }
  char* stg = staging(p);
  const int chunk = (int)std::min<size_t>(N, staging_bytes(p) / sizeof(double));
  for (int i = 0; i < p->Q; ++i)
    for (int c0 = 0; c0 < N; c0 += chunk) {
      const int c1 = std::min(N, c0 + chunk);
      p->ops->populations(p, reinterpret_cast<double*>(stg), i, i + 1, c0, c1, st);
      LSB_HIP(hipGetLastError());
      LSB_HIP(hipMemcpyAsync(out + (size_t)i * N + c0, stg, (size_t)(c1 - c0) * sizeof(double), hipMemcpyDeviceToHost, st));
      LSB_HIP(hipStreamSynchronize(st));
    }
  return LSB_OK;
}

int lsb_get_moments(lsb_plan* p, double* out, int on_device, void* stream) {
  if (!p || !out) return fail(LSB_EINVAL, "null argument");
  if (!p->inited) return fail(LSB_ESTATE, "no state");
  hipStream_t st = as_stream(stream);
  const int N = p->N;
  if (on_device) {
    p->ops->moments(p, out, 0, N, st);
    return check_launch();
  }
  char* stg = staging(p);
  const int chunk = (int)std::min<size_t>(N, staging_bytes(p) / (10 * sizeof(double)));
  for (int c0 = 0; c0 < N; c0 += chunk) {
    const int c1 = std::min(N, c0 + chunk);
    p->ops->moments(p, reinterpret_cast<double*>(stg), c0, c1, st);
    LSB_HIP(hipGetLastError());
    LSB_HIP(hipMemcpyAsync(out + 10 * (size_t)c0, stg, 10 * (size_t)(c1 - c0) * sizeof(double), hipMemcpyDeviceToHost, st));
    LSB_HIP(hipStreamSynchronize(st));
  }
  return LSB_OK;
}

int lsb_get_integrals(lsb_plan* p, lsb_integrals* out, void* stream) {
  if (!p || !out) return fail(LSB_EINVAL, "null argument");
  if (!p->inited) return fail(LSB_ESTATE, "no state");
  hipStream_t st = as_stream(stream);
  p->ops->integrals_partial(p, nullptr, st);
  LSB_HIP(hipGetLastError());
  std::vector<double> part((size_t)p->red_blocks * 16);
  LSB_HIP(hipMemcpyAsync(part.data(), p->ws + p->off_partial, part.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  double pb = 0;
  LSB_HIP(hipMemcpyAsync(&pb, p->ws + p->off_scal + lsb::SC_PB * sizeof(double), sizeof(double), hipMemcpyDeviceToHost, st));
  LSB_HIP(hipStreamSynchronize(st));
  double v[11] = {0};
  double umax = 0;
  for (int b = 0; b < p->red_blocks; ++b) {
    for (int m = 0; m < 11; ++m)
      if (m != 9) v[m] += part[16 * (size_t)b + m];
    umax = std::max(umax, part[16 * (size_t)b + 9]);
  }
  out->mass[0] = v[0];
  out->mass[1] = v[1];
  out->volume_gas = v[2];
  for (int a = 0; a < 3; ++a) {
    out->centroid[a] = v[2] > 0 ? v[3 + a] / v[2] : 0.0;
    out->vel_b[a] = v[2] > 0 ? v[6 + a] / v[2] : 0.0;
  }
  out->pb = pb;
  out->umax = umax;
  out->step = p->nstep;
  return LSB_OK;
}

// ---------------------------------------------------------------------------
// Integrals without allocation (lsb_get_integrals_static).  The reduction's
// partial sums go to this file-scope device array instead of the plan's
// workspace: LSB_INTEGRALS_STATIC_BLOCKS blocks of 16 doubles, then 16 for
// the result.  Each GPU holds its own copy until the process ends; in host
// code `scratch` is only a symbol, its device address on the current device
// comes from hipGetSymbolAddress (kept per device).  Every block of the
// partial kernel writes all the slots that the final kernel reads, so nothing
// needs clearing between calls.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[LSB_INTEGRALS_STATIC_BLOCKS * 16 + 16];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up once per device)
int scratch_address(double** out) {
  int dev = 0;
  LSB_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LSB_EDEVICE, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    LSB_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(LSB_EDEVICE, "hipGetSymbolAddress returned no address for the static scratch");
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return LSB_OK;
}

// The host reduction of lsb_get_integrals on the device: one thread per
// slot adds the blocks' partial sums in block order (slot 9: maximum), so
// the result has the same bits; then the derived quantities.
__global__ void k_integrals_static_final(const double* part, int nblocks, const double* pb, double* res,
                                         double* out) {
  const int m = threadIdx.x;
  if (m < 11) {
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) {
      const double x = part[16 * (size_t)b + m];
      v = (m == 9) ? (v < x ? x : v) : v + x;  // the host side's std::max(v, x)
    }
    res[m] = v;
  }
  __syncthreads();
  if (m == 0) {
    const double V = res[2];
    out[0] = res[0];
    out[1] = res[1];
    out[2] = V;
    for (int a = 0; a < 3; ++a) {
      out[3 + a] = V > 0 ? res[3 + a] / V : 0.0;
      out[6 + a] = V > 0 ? res[6 + a] / V : 0.0;
    }
    out[9] = *pb;
    out[10] = res[9];
    out[11] = res[10];
    for (int k = 12; k < 16; ++k) out[k] = 0.0;
  }
}
}  // namespace

int lsb_get_integrals_static(lsb_plan* p, double* out, void* stream) {
  if (!p || !out) return fail(LSB_EINVAL, "null argument");
  if (p->red_blocks > LSB_INTEGRALS_STATIC_BLOCKS)
    return fail(LSB_EINVAL, "the plan's reduction grid exceeds LSB_INTEGRALS_STATIC_BLOCKS");
  if (!p->inited) return fail(LSB_ESTATE, "no state");
  double* s = nullptr;
  if (int r = scratch_address(&s)) return r;
  hipStream_t st = as_stream(stream);
  double* part = s;
  double* res = s + (size_t)LSB_INTEGRALS_STATIC_BLOCKS * 16;
  p->ops->integrals_partial(p, part, st);
  const double* pb = reinterpret_cast<const double*>(p->ws + p->off_scal + lsb::SC_PB * sizeof(double));
  k_integrals_static_final<<<1, 64, 0, st>>>(part, p->red_blocks, pb, res, out);
  return check_launch();
}

// State image: populations, phi, moments, scalars (device) plus a small
// host header with the step count.
static size_t state_layout(const lsb_plan* p, size_t* o_pop, size_t* o_phi, size_t* o_M, size_t* o_scal, size_t* o_hdr) {
  const size_t N = (size_t)p->N;
  size_t o = 0;
  *o_hdr = o; o = align256(o + 64);
  *o_pop = o; o = align256(o + p->pop_bytes);
  *o_phi = o; o = align256(o + N * p->bytes_real);
  *o_M = o; o = align256(o + 10 * N * p->bytes_real);
  *o_scal = o; o = align256(o + lsb::SC_COUNT * sizeof(double));
  return o;
}

int lsb_state_bytes(const lsb_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(LSB_EINVAL, "null argument");
  size_t a, b, c, d, e;
  *bytes = state_layout(p, &a, &b, &c, &d, &e);
  return LSB_OK;
}

int lsb_save_state(lsb_plan* p, void* dst, void* stream) {
  if (!p || !dst) return fail(LSB_EINVAL, "null argument");
  if (!p->inited) return fail(LSB_ESTATE, "no state");
  hipStream_t st = as_stream(stream);
  size_t o_pop, o_phi, o_M, o_scal, o_hdr;
  state_layout(p, &o_pop, &o_phi, &o_M, &o_scal, &o_hdr);
  char* d = static_cast<char*>(dst);
  const size_t N = (size_t)p->N;
  long hdr[8] = {0x4c5342, p->nstep, p->N, p->Q, (long)p->bytes_pop, 0, 0, 0};
  LSB_HIP(hipMemcpyAsync(d + o_hdr, hdr, sizeof(hdr), hipMemcpyHostToDevice, st));
  LSB_HIP(hipMemcpyAsync(d + o_pop, p->ws + p->off_A[p->cur], p->pop_bytes, hipMemcpyDeviceToDevice, st));
  LSB_HIP(hipMemcpyAsync(d + o_phi, p->ws + p->off_phi, N * p->bytes_real, hipMemcpyDeviceToDevice, st));
  LSB_HIP(hipMemcpyAsync(d + o_M, p->ws + p->off_M[p->cur], 10 * N * p->bytes_real, hipMemcpyDeviceToDevice, st));
  LSB_HIP(hipMemcpyAsync(d + o_scal, p->ws + p->off_scal, lsb::SC_COUNT * sizeof(double), hipMemcpyDeviceToDevice, st));
  LSB_HIP(hipStreamSynchronize(st));
  return LSB_OK;
}

int lsb_load_state(lsb_plan* p, const void* src, void* stream) {
  if (!p || !src) return fail(LSB_EINVAL, "null argument");
  if (!p->bound) return fail(LSB_ESTATE, "lsb_load_state before lsb_bind");
  hipStream_t st = as_stream(stream);
  size_t o_pop, o_phi, o_M, o_scal, o_hdr;
  state_layout(p, &o_pop, &o_phi, &o_M, &o_scal, &o_hdr);
  const char* s = static_cast<const char*>(src);
  long hdr[8];
  LSB_HIP(hipMemcpyAsync(hdr, s + o_hdr, sizeof(hdr), hipMemcpyDeviceToHost, st));
  LSB_HIP(hipStreamSynchronize(st));
  if (hdr[0] != 0x4c5342 || hdr[2] != p->N || hdr[3] != p->Q || hdr[4] != (long)p->bytes_pop)
    return fail(LSB_EINVAL, "state image does not match this plan");
  const size_t N = (size_t)p->N;
  LSB_HIP(hipStreamSynchronize(p->side));
  p->cur = 0;
  p->tcur = 0;
  LSB_HIP(hipMemcpyAsync(p->ws + p->off_A[0], s + o_pop, p->pop_bytes, hipMemcpyDeviceToDevice, st));
  LSB_HIP(hipMemcpyAsync(p->ws + p->off_phi, s + o_phi, N * p->bytes_real, hipMemcpyDeviceToDevice, st));
  LSB_HIP(hipMemcpyAsync(p->ws + p->off_s1, s + o_phi, N * p->bytes_real, hipMemcpyDeviceToDevice, st));
  LSB_HIP(hipMemcpyAsync(p->ws + p->off_s2, s + o_phi, N * p->bytes_real, hipMemcpyDeviceToDevice, st));
  LSB_HIP(hipMemcpyAsync(p->ws + p->off_p0, s + o_phi, N * p->bytes_real, hipMemcpyDeviceToDevice, st));
  LSB_HIP(hipMemcpyAsync(p->ws + p->off_M[0], s + o_M, 10 * N * p->bytes_real, hipMemcpyDeviceToDevice, st));
  LSB_HIP(hipMemcpyAsync(p->ws + p->off_scal, s + o_scal, lsb::SC_COUNT * sizeof(double), hipMemcpyDeviceToDevice, st));
  double rr[2] = {1.0, 1.0};
  LSB_HIP(hipMemcpyAsync(rr, s + o_scal + lsb::SC_RREF * sizeof(double), sizeof(rr), hipMemcpyDeviceToHost, st));
  LSB_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < 2; ++k) p->rho_ref[k] = (std::isfinite(rr[k]) && rr[k] > 0) ? rr[k] : 1.0;
  p->nstep = hdr[1];  // before the rebuild: the candidate flags are kept by step parity
  p->ops->rebuild(p, st);
  p->ops->pack(p, st);
  LSB_HIP(hipGetLastError());
  LSB_HIP(hipStreamSynchronize(st));
  LSB_HIP(hipEventRecord(p->ev_pop_done, st));
  LSB_HIP(hipEventRecord(p->ev_bulk_done, st));
  p->inited = true;
  return LSB_OK;
}

long lsb_step_count(const lsb_plan* p) { return p ? p->nstep : -1; }

int lsb_set_schedule(lsb_plan* p, int schedule) {
  if (!p) return fail(LSB_EINVAL, "null plan");
  if (schedule != LSB_SCHED_SERIAL && schedule != LSB_SCHED_OVERLAP) return fail(LSB_EINVAL, "unknown schedule");
  p->schedule = schedule;
  return LSB_OK;
}

int lsb_set_kernel_timing(lsb_plan* p, int enable) {
  if (!p) return fail(LSB_EINVAL, "null plan");
  if (enable && p->ev.empty()) {
    p->ev.resize(2 * lsb::kEventPairs);
    for (auto& e : p->ev) LSB_HIP(hipEventCreate(&e));
  }
  if (p->timing) lsb::timing_flush(p);
  p->timing = enable != 0;
  p->ev_used = 0;
  if (enable) {
    p->timing_ms = 0.0;
    p->timing_launches = 0;
  }
  return LSB_OK;
}

int lsb_get_kernel_timing(lsb_plan* p, double* total_ms, long* launches) {
  if (!p || !total_ms || !launches) return fail(LSB_EINVAL, "null argument");
  lsb::timing_flush(p);
  *total_ms = p->timing_ms;
  *launches = p->timing_launches;
  return LSB_OK;
}

int lsb_get_counts(lsb_plan* p, int* counts, void* stream) {
  if (!p || !counts) return fail(LSB_EINVAL, "null argument");
  if (!p->inited) return fail(LSB_ESTATE, "no state");
  hipStream_t st = as_stream(stream);
  int c[lsb::CNT_NUM];
  LSB_HIP(hipMemcpyAsync(c, p->ws + p->off_cnt, sizeof(c), hipMemcpyDeviceToHost, st));
  LSB_HIP(hipStreamSynchronize(st));
  counts[0] = c[lsb::CNT_SPEC];
  counts[1] = c[lsb::CNT_TILES];
  counts[2] = c[lsb::CNT_FLIP];
  counts[3] = c[lsb::CNT_WALL];
  return LSB_OK;
}

// ---------------------------------------------------------------------------
// Reverse mode
// ---------------------------------------------------------------------------
static void adj_layout(const lsb_plan* p, int max_steps, lsb::AdjState& s, size_t* total) {
  const size_t N = (size_t)p->N, rb = p->bytes_real;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  s.s_A = take(p->pop_bytes);
  s.s_M = take(10 * N * rb);
  s.s_phi = take(N * rb);
  s.s_G = take(4 * N * rb);
  s.s_tag = take(N);
  s.s_scal = take(lsb::SC_COUNT * sizeof(double));
  s.s_Mn = take(10 * N * rb);
  s.s_ut = take((size_t)(p->P.n_ext + 1) * 3 * N * rb);
  s.s_s1 = take(N * rb);
  s.s_s2 = take(N * rb);
  const bool rein = p->P.reinit_every > 0 && p->P.n_reinit > 0;
  s.s_p0 = take(rein ? N * rb : 0);
  s.s_rein = take(rein ? (size_t)3 * p->P.n_reinit * N * rb : 0);
  s.stride = o;
  o = 0;
  s.o_snap = take((size_t)(max_steps + 1) * s.stride);
  for (int r = 0; r < 2; ++r) {
    s.o_Abar[r] = take(9 * N * sizeof(double));
    s.o_Mbar[r] = take(10 * N * sizeof(double));
    s.o_phibar[r] = take(N * sizeof(double));
    s.o_Gbar[r] = take(4 * N * sizeof(double));
    s.o_utbar[r] = take(3 * N * sizeof(double));
  }
  s.o_s1bar = take(N * sizeof(double));
  s.o_s2bar = take(N * sizeof(double));
  for (int r = 0; r < 2; ++r) s.o_rphibar[r] = take(rein ? N * sizeof(double) : 0);
  s.o_rs1bar = take(rein ? N * sizeof(double) : 0);
  s.o_rs2bar = take(rein ? N * sizeof(double) : 0);
  s.o_p0bar = take(rein ? N * sizeof(double) : 0);
  s.o_ytmp = take(19 * N * sizeof(double));
  s.o_scal = take(lsb::AdjState::SC_NUM * sizeof(double));
  s.o_partial = take(2 * lsb::AdjState::kInitBlocks * sizeof(double));
  *total = o;
}

static int adj_check(const lsb_plan* p) {
  if (!p) return fail(LSB_EINVAL, "null plan");
  if (!p->adj_ops)
    return fail(LSB_EINVAL, "the reverse mode needs the D2Q9 lattice with LSB_F64 or LSB_F32 storage");
  if (p->P.use_pb == 2) return fail(LSB_EINVAL, "the reverse mode takes one gas baseline (use_pb 0 or 1)");
  return LSB_OK;
}

int lsb_adjoint_workspace_bytes(const lsb_plan* p, int max_segment_steps, size_t* bytes) {
  if (int r = adj_check(p)) return r;
  if (!bytes || max_segment_steps < 1) return fail(LSB_EINVAL, "bad argument");
  lsb::AdjState s;
  adj_layout(p, max_segment_steps, s, bytes);
  return LSB_OK;
}

int lsb_adjoint_bind(lsb_plan* p, void* ws, size_t bytes, int max_segment_steps) {
  if (int r = adj_check(p)) return r;
  if (!ws || max_segment_steps < 1) return fail(LSB_EINVAL, "bad argument");
  size_t need = 0;
  lsb::AdjState s;
  adj_layout(p, max_segment_steps, s, &need);
  if (bytes < need) return fail(LSB_ENOMEM, "adjoint workspace too small: need " + std::to_string(need) + " bytes");
  s.ws = static_cast<char*>(ws);
  s.bytes = bytes;
  s.max_steps = max_segment_steps;
  p->adj = s;
  return LSB_OK;
}

int lsb_adjoint_record(lsb_plan* p, int nsteps, void* stream) {
  if (int r = adj_check(p)) return r;
  if (!p->adj.ws) return fail(LSB_ESTATE, "lsb_adjoint_record before lsb_adjoint_bind");
  if (!p->inited) return fail(LSB_ESTATE, "lsb_adjoint_record before lsb_init");
  if (nsteps < 1 || nsteps > p->adj.max_steps) return fail(LSB_EINVAL, "segment length out of range");
  hipStream_t st = as_stream(stream);
  LSB_HIP(hipStreamWaitEvent(st, p->ev_bulk_done, 0));
  p->adj_ops->record(p, nsteps, st);
  if (int r = check_launch()) return r;
  return LSB_OK;
}

int lsb_adjoint_seed_centroid(lsb_plan* p, int axis, void* stream) {
  if (int r = adj_check(p)) return r;
  if (!p->adj.ws || p->adj.nrec < 1) return fail(LSB_ESTATE, "no recorded segment");
  if (axis < 0 || axis > 1) return fail(LSB_EINVAL, "axis must be 0 or 1");
  p->adj_ops->seed_centroid(p, axis, as_stream(stream));
  if (int r = check_launch()) return r;
  p->adj.seeded = true;
  return LSB_OK;
}

int lsb_adjoint_reverse(lsb_plan* p, void* stream) {
  if (int r = adj_check(p)) return r;
  if (!p->adj.seeded || p->adj.nrec < 1) return fail(LSB_ESTATE, "lsb_adjoint_reverse before a seed and a record");
  hipStream_t st = as_stream(stream);
  p->adj_ops->reverse(p, st);
  if (int r = check_launch()) return r;
  int flag = 0;
  LSB_HIP(hipMemcpyAsync(&flag, p->adj.ws + p->adj.o_scal + lsb::AdjState::SC_FLAG * sizeof(double), sizeof(int),
                         hipMemcpyDeviceToHost, st));
  LSB_HIP(hipStreamSynchronize(st));
  if (flag) return fail(LSB_EDEVICE, "internal: reverse-mode input list overflow");
  return LSB_OK;
}

int lsb_adjoint_initial(lsb_plan* p, const double* phi0, const double* u0, int rho0_given, double* dL_dphi0,
                        double* dL_dsigma, void* stream) {
  if (int r = adj_check(p)) return r;
  if (!p->adj.seeded || p->adj.nrec < 1) return fail(LSB_ESTATE, "no reversed segment");
  if (!phi0 || !dL_dphi0 || !dL_dsigma) return fail(LSB_EINVAL, "null argument");
  hipStream_t st = as_stream(stream);
  const int hydro = (p->P.init_hydrostatic && !rho0_given) ? 1 : 0;
  p->adj_ops->initial(p, phi0, u0, hydro, dL_dphi0, st);
  if (int r = check_launch()) return r;
  LSB_HIP(hipMemcpyAsync(dL_dsigma, p->adj.ws + p->adj.o_scal + lsb::AdjState::SC_SIGBAR * sizeof(double),
                         sizeof(double), hipMemcpyDeviceToHost, st));
  LSB_HIP(hipStreamSynchronize(st));
  return LSB_OK;
}

}  // extern "C"
