// plan.h -- host-side plan: validated parameters, workspace layout and the
// per-(velocity set, storage) launch table.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lsb.h"

struct lsb_plan;

namespace lsb {

// Cell-range launchers [c0, c1) write their outputs at offset c - c0, so
// host-pointer calls can stage chunks through the workspace.
struct Ops {
  void (*init_phi)(lsb_plan*, const double* phi0, int c0, int c1, hipStream_t);
  void (*init_band)(lsb_plan*, hipStream_t);
  void (*init_pop)(lsb_plan*, const double* rho0, const double* u0, int c0, int c1, hipStream_t);
  void (*step)(lsb_plan*, hipStream_t);
  void (*fields)(lsb_plan*, double* rho, double* u, double* p, uint8_t* phase, int c0, int c1, hipStream_t);
  void (*populations)(lsb_plan*, double* out, int i0, int i1, int c0, int c1, hipStream_t);
  void (*interface)(lsb_plan*, double* phi, double* nrm, double* kap, uint8_t* tags, int c0, int c1, hipStream_t);
  void (*moments)(lsb_plan*, double* out, int c0, int c1, hipStream_t);
  // partial: 16 doubles per reduction block; nullptr = the workspace's region
  void (*integrals_partial)(lsb_plan*, double* partial, hipStream_t);
  void (*rebuild)(lsb_plan*, hipStream_t);
  void (*pack)(lsb_plan*, hipStream_t);  // interface records of the current state
};

// reverse mode (D2Q9, FP64 / FP32 state)
struct AdjOps {
  void (*record)(lsb_plan*, int nsteps, hipStream_t);
  void (*seed_centroid)(lsb_plan*, int axis, hipStream_t);
  void (*reverse)(lsb_plan*, hipStream_t);
  void (*initial)(lsb_plan*, const double* phi0, const double* u0, int hydro, double* dphi0, hipStream_t);
};
const AdjOps* adj_ops_d2q9(int storage);

// Reverse-mode workspace: snapshots of a recorded checkpoint segment (state
// before each step plus the step's intermediates) and the FP64 adjoints.
struct AdjState {
  // slots of the FP64 scalar block
  enum { SC_PBBAR = 0, SC_SIGBAR = 2, SC_XC0BAR = 3, SC_W = 6, SC_XC = 8, SC_V = 10, SC_SIGMA = 11, SC_FLAG = 12,
         SC_NUM = 16 };
  static constexpr int kInitBlocks = 256;
  char* ws = nullptr;
  size_t bytes = 0;
  int max_steps = 0;
  size_t stride = 0, o_snap = 0;  // snapshot slot size and offset of slot 0
  size_t s_A = 0, s_M = 0, s_phi = 0, s_G = 0, s_tag = 0, s_scal = 0, s_Mn = 0, s_ut = 0, s_s1 = 0, s_s2 = 0;
  size_t s_p0 = 0, s_rein = 0;  // reinitialisation: level set before it, stage inputs of every pseudo step
  size_t o_Abar[2] = {0, 0}, o_Mbar[2] = {0, 0}, o_phibar[2] = {0, 0}, o_Gbar[2] = {0, 0}, o_utbar[2] = {0, 0};
  size_t o_s1bar = 0, o_s2bar = 0, o_ytmp = 0, o_scal = 0, o_partial = 0;
  size_t o_rphibar[2] = {0, 0}, o_rs1bar = 0, o_rs2bar = 0, o_p0bar = 0;
  std::vector<unsigned char> reinit_at;  // per recorded step: the step reinitialised
  int role = 0;       // adjoint buffers holding the adjoint of the latest state
  int nrec = 0;       // steps of the recorded segment
  int rec_slot = -1;  // slot written by the step being recorded
  bool seeded = false;
};

const Ops* ops_d2q9(int storage);
const Ops* ops_d3q19(int storage);
const Ops* ops_d3q27(int storage);

void set_error(const std::string& msg);
// lsb_create, also accepting kFaceInject faces (a refined box's level)
int create_plan(const lsb_params* P, bool allow_inject, lsb_plan** out);
// events around the dominant kernel (no-ops unless timing is enabled)
void timing_begin(lsb_plan* p, hipStream_t st);
void timing_end(lsb_plan* p, hipStream_t st);

}  // namespace lsb

struct lsb_plan {
  lsb_params P;
  int D = 0, Q = 0;
  int N = 0;
  size_t bytes_pop = 0;  // bytes per stored population value
  size_t pop_bytes = 0;  // bytes of one population buffer (the 3D layout pads N to a multiple of 256)
  size_t bytes_real = 0; // bytes per level-set / moment value
  int tdim[3] = {1, 1, 1};
  int ntile[3] = {1, 1, 1};
  int ntiles = 0;
  int red_blocks = 512;  // fixed reduction grid (deterministic sums)
  double rho_ref[2] = {1.0, 1.0};  // the codec's reference density per phase (see KArgs::rho_ref)
  // workspace regions (byte offsets)
  size_t off_A[2], off_phi, off_s1, off_s2, off_p0, off_tag, off_aux, off_M[2], off_G, off_ut[2];
  size_t off_scal, off_cnt, off_tile_act, off_tile_list, off_cand_list, off_spec_list, off_flip_list, off_partial;
  size_t off_wall_list;
  size_t off_ghost = 0;    // injected-face populations [Q][N] (a refined box's level only)
  size_t off_ext_k;        // extension coefficients of the current step
  size_t off_irec;         // packed interface records [N][16]
  size_t off_blab = 0, off_broots = 0, off_bpart = 0, off_bres = 0, off_pbc = 0;  // several bubbles
  size_t off_tile_act2;    // second tile-activity buffer
  size_t off_cflag[2];     // candidate-tile flags, by step parity
  int tcur = 0;            // which tile-activity buffer holds this step's flags
  int schedule = 0;        // LSB_SCHED_*
  hipStream_t side = nullptr;        // library-owned stream of the bulk collide-stream
  hipEvent_t ev_pop_done = nullptr;  // band, interface and wall collide-stream of the last step finished
  hipEvent_t ev_bulk_done = nullptr; // bulk collide-stream of the last step finished
  long n_wall_cells = 0;   // bound on wall-adjacent cells (static)
  int grid_walls = 1;
  size_t total = 0;
  char* ws = nullptr;
  int cur = 0;           // index of the current population / moment buffer
  bool bound = false;
  bool inited = false;
  long nstep = 0;
  const lsb::Ops* ops = nullptr;
  const lsb::AdjOps* adj_ops = nullptr;  // null where the reverse mode is not available
  lsb::AdjState adj;
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev;  // start/stop pairs
  int ev_used = 0;
  double timing_ms = 0.0;
  long timing_launches = 0;
  // grid sizes of list-driven kernels
  int grid_tiles = 1024;
  int grid_cells = 1024;
};
