/*
 * lsb.h -- C ABI of the coupled level-set lattice Boltzmann hot path on
 * AMD MI355X (gfx950).
 *
 * Method: Vorspohl, Peng, Meinke, Krug, Schroeder, "Coupled Level-Set Lattice
 * Boltzmann Method on Adaptive Cartesian Grids".  Each fluid phase runs its
 * own lattice Boltzmann solver (Sec. 2.1); the phases are coupled at the
 * sharp interface phi = 0 by interpolated bounce-back carrying the stress
 * jump (Sec. 2.3); the level set is advected, extended and reinitialised on
 * a narrow band (Sec. 2.2); cells swept by the interface are refilled
 * (Sec. 2.4).
 *
 * Conventions
 *   - Grids are dense, uniform, cell centred (x = i + 1/2), row-major
 *     [nz][ny][nx]; nz = 1 with D2Q9 is two-dimensional.
 *   - Phase 0 is the liquid (phi < 0), phase 1 the gas (phi >= 0).
 *   - Faces are ordered -x, +x, -y, +y, -z, +z.  Paired faces are either both
 *     periodic or both walls.
 *   - Lattice units: dx = dt = 1, cs^2 = 1/3.
 *   - Every function returns LSB_OK (0) or a negative error code;
 *     lsb_last_error() gives a thread-local message.
 *   - Device memory belongs to the caller: the library computes the size of
 *     one workspace (lsb_workspace_bytes), the caller allocates it and binds
 *     it (lsb_bind).  The library never allocates or frees device memory.
 *   - `stream` is a hipStream_t (may be NULL for the default stream).  Calls
 *     enqueue work on it; calls that take host pointers (on_device = 0)
 *     synchronise the stream before returning.
 */
#ifndef LSB_H
#define LSB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes.  LSB_EBAND: a refined box no longer holds the level-set
 * band with its margin (lsb_refine2.h). */
enum { LSB_OK = 0, LSB_EINVAL = -1, LSB_ENOMEM = -2, LSB_EDEVICE = -3, LSB_ESTATE = -4, LSB_EUNSTABLE = -5,
       LSB_EBAND = -6 };

/* Velocity sets (Sec. 2.1 velocity-set figure; D3Q19 is the textbook subset
 * made of the D3Q27 directions 0..17 plus rest). */
enum { LSB_D2Q9 = 0, LSB_D3Q19 = 1, LSB_D3Q27 = 2 };

/* Population storage.  F64: FP64 deviations f - w, FP64 arithmetic.
 * F32: FP32 deviations, FP32 arithmetic.  F16DEV / BF16DEV: scaled deviations
 * s (f - w) / w stored in FP16 (s = 2^fp16_scale_log2) or BF16 (s = 1), FP32
 * arithmetic.  Level set, geometry and moments are FP64 on the F64 path and
 * FP32 otherwise; reductions accumulate in FP64. */
enum { LSB_F64 = 0, LSB_F32 = 1, LSB_F16DEV = 2, LSB_BF16DEV = 3 };

/* Face conditions: periodic; no-slip wall on the face (halfway bounce-back,
 * moving with wall_u, Sec. 2.1 eq:bb); free-slip wall (specular reflection). */
enum { LSB_PERIODIC = 0, LSB_NOSLIP = 1, LSB_FREESLIP = 2 };

/* Collision operator of a phase (Sec. 2.1): BGK with the equilibrium eq:feq,
 * or the cumulant operator (cumulants of the populations relaxed towards
 * their Maxwell values: shear cumulants at omega = 1/tau, every other
 * cumulant at rate one; D3Q27 only).  Both add the same body-force term. */
enum { LSB_BGK = 0, LSB_CUMULANT = 1 };

/* Most bubbles tracked with use_pb = 2. */
enum { LSB_MAX_BUBBLES = 64 };

/* Problem statement (Sec. 2 and the setups of Sec. 3). */
typedef struct lsb_params {
  int lattice, storage, nx, ny, nz;
  int bc[6];
  double wall_u[6][3];      /* velocity of each no-slip face */
  double rho_phys[2];       /* physical densities [liquid, gas] */
  double tau[2];            /* BGK relaxation times, tau = 1/2 + nu / cs^2 (eq:omega) */
  double accel[2][3];       /* body acceleration of each phase (gravity, or force density / rho_phys) */
  double sigma;             /* surface tension */
  double band;              /* narrow-band half width B in cells (level set clamped to +-B) */
  int n_ext;                /* velocity-extension sweeps per step (eq:hyperbolicExtension) */
  double ext_dtau;          /* pseudo time step of the extension */
  int reinit_every;         /* reinitialise every k steps (0 = never) */
  int n_reinit;             /* pseudo steps per reinitialisation */
  double reinit_dtau;       /* pseudo time step of the reinitialisation */
  double heaviside_eps;     /* half width of the smoothed Heaviside (Sec. 3.2 integrals) */
  int use_pb;               /* gas pressure baseline under gravity: 0 off (pb0 throughout),
                               1 one baseline from the gas centroid, 2 one per bubble (the
                               connected components of the smoothed Heaviside's support, each
                               with the baseline at its own centroid; at most LSB_MAX_BUBBLES) */
  double pb0;               /* initial gas pressure baseline */
  int init_hydrostatic;     /* default initial LB density is hydrostatic about the gas centroid */
  int fp16_scale_log2;      /* s = 2^k for LSB_F16DEV (typically 12) */
  int collision[2];         /* collision operator of each phase [liquid, gas]: LSB_BGK, or
                               LSB_CUMULANT (Sec. 2.1: cumulants relaxed towards the Maxwell
                               values, shear rate 1/tau, every other rate one; D3Q27 only) */
} lsb_params;

typedef struct lsb_plan lsb_plan; /* opaque; owned by the library */

/* Integral quantities (Sec. 3.2): per-phase mass, Heaviside-weighted gas
 * volume, centroid and bubble velocity of all gas, gas pressure baseline
 * (use_pb = 1: the one baseline; use_pb = 0 or 2: pb0, the per-bubble
 * baselines are in lsb_get_bubbles), max |u|. */
typedef struct lsb_integrals {
  double mass[2];
  double volume_gas;
  double centroid[3];
  double vel_b[3];
  double pb;
  double umax;
  long step;
} lsb_integrals;

/* Validate a parameter block and create a plan (host memory only).
 * Errors: LSB_EINVAL for an unknown lattice/storage, a grid smaller than
 * 4 cells per used axis, nz != 1 with D2Q9, unpaired periodic faces,
 * tau <= 1/2, band < 2, negative counts, an unknown collision operator or
 * LSB_CUMULANT with a lattice other than D3Q27. */
int lsb_create(const lsb_params* params, lsb_plan** out);
void lsb_destroy(lsb_plan* plan);

/* Bytes of device workspace the plan needs (256-byte aligned regions). */
int lsb_workspace_bytes(const lsb_plan* plan, size_t* bytes);

/* Bind a caller-owned device buffer of at least lsb_workspace_bytes bytes.
 * LSB_ENOMEM if it is too small; LSB_EINVAL for a NULL pointer. */
int lsb_bind(lsb_plan* plan, void* device_workspace, size_t bytes);

/* Initial state (Sec. 2.1 equilibrium; Sec. 2.2 signed distance):
 * phi0 [N] signed distance (clamped to +-band); rho0 [N] LB density or NULL
 * (1, or hydrostatic when init_hydrostatic); u0 [N*3] velocity (x,y,z
 * interleaved per cell) or NULL (rest).  Populations start at the
 * equilibrium.  Arrays are device pointers when on_device != 0, otherwise
 * host pointers staged through the workspace.  LSB_ESTATE before lsb_bind. */
int lsb_init(lsb_plan* plan, const double* phi0, const double* rho0, const double* u0, int on_device,
             void* stream);

/* Advance nsteps time steps (Sec. 2: the collide-stream of each phase,
 * Eq. 1 with the BGK or cumulant operator and the body force, with wall
 * bounce-back, eq:bb, and interface bounce-back, eq:bb_cc with the stress
 * jump eq:Sdecomp; Sec. 2.2: velocity extension, eq:hyperbolicExtension,
 * transport of the level set and periodic reinitialisation; Sec. 2.4:
 * classification and refill of cells whose phase changed; Sec. 3.2: gas
 * centroid and pressure baseline).
 * If check_every > 0, every check_every steps the stream is synchronised and
 * LSB_EUNSTABLE returned on a non-finite or non-positive density or
 * |u| > 0.3.  LSB_ESTATE before lsb_init. */
int lsb_step(lsb_plan* plan, int nsteps, int check_every, void* stream);

/* Macroscopic fields (Sec. 2.1, eq:macro): rho [N] (sum of populations), u [N*d] (d = 2 or 3,
 * interleaved per cell; time-centred velocity sum(c f)/rho - a/2), p [N]
 * (phase pressure rho_phys cs^2 (rho - 1), plus the baseline in the gas),
 * phase [N] (0 liquid, 1 gas).  Any pointer may be NULL. */
int lsb_get_fields(lsb_plan* plan, double* rho, double* u, double* p, uint8_t* phase, int on_device,
                   void* stream);

/* Interface description (Sec. 2.2: the level set, its normal and its
 * curvature kappa = div n): phi [N], normal [N*d], kappa [N] (valid on
 * LS-active cells), tags [N] (bit0 gas, bit1 LS-active, bit2 has a lattice
 * link to the other phase).  Any pointer may be NULL. */
int lsb_get_interface(lsb_plan* plan, double* phi, double* normal, double* kappa, uint8_t* tags,
                      int on_device, void* stream);

/* Bubbles (use_pb = 2; Sec. 3.2 integrals per bubble): *count bubbles,
 * numbered by their smallest cell; out [max][5] (host) per bubble: volume
 * (sum of the smoothed Heaviside), centroid[3], gas pressure baseline
 * pb0 + rho_l a_l . (x_c - x_c0); labels [N] (int32, host or device as
 * on_device): the bubble of each cell, -1 outside the Heaviside support.
 * out and labels may be NULL.  Synchronises the stream.  LSB_EINVAL unless
 * use_pb = 2; LSB_EUNSTABLE when more than LSB_MAX_BUBBLES bubbles were
 * found (the baselines of the rest are missing; *count holds the number). */
int lsb_get_bubbles(lsb_plan* plan, int max, int* count, double* out, int32_t* labels, int on_device, void* stream);

/* Decoded populations A[i*N + cell] (post-collision, FP64; Eq. 1, the
 * paper's direction order with the rest direction last). */
int lsb_get_populations(lsb_plan* plan, double* out, int on_device, void* stream);

/* Moments of the last collision per cell (the inputs of the interface
 * coupling, Sec. 2.3), [N][10] = (rho, u[3], S[6] with
 * S = xx, yy, zz, xy, xz, yz); valid on LS-active cells. */
int lsb_get_moments(lsb_plan* plan, double* out, int on_device, void* stream);

/* Integral quantities (Sec. 3.2: per-phase mass, gas volume, centroid and
 * bubble velocity with the smoothed Heaviside, the gas pressure baseline,
 * max |u|), FP64, synchronises the stream. */
int lsb_get_integrals(lsb_plan* plan, lsb_integrals* out, void* stream);

/* lsb_get_integrals without allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * it): no device or host allocation and no synchronisation; the work is
 * queued on the stream.  The reduction's partial sums use a static device
 * array of the library (LSB_INTEGRALS_STATIC_BLOCKS x 16 + 16 doubles,
 * 64.1 KiB, held on each GPU the library runs on until the process ends)
 * instead of the workspace, added in the same fixed order, so the values
 * equal lsb_get_integrals' bit for bit.  out (device, 16 doubles, caller
 * owned): mass[2], volume_gas, centroid[3], vel_b[3], pb, umax, the number
 * of cells failing the stability test, 4 zeros.  All calls on one GPU
 * share the array: calls that overlap on one GPU (concurrent streams or
 * threads) race.  LSB_EINVAL for a NULL argument or a plan whose reduction
 * grid exceeds LSB_INTEGRALS_STATIC_BLOCKS (checked before any device
 * access); LSB_ESTATE before lsb_init; LSB_EDEVICE if the array's device
 * address cannot be obtained. */
#define LSB_INTEGRALS_STATIC_BLOCKS 512
int lsb_get_integrals_static(lsb_plan* plan, double* out, void* stream);

/* Checkpoint / resume: device-to-device copy of the full state into or out
 * of a caller buffer of lsb_state_bytes bytes. */
int lsb_state_bytes(const lsb_plan* plan, size_t* bytes);
int lsb_save_state(lsb_plan* plan, void* device_dst, void* stream);
int lsb_load_state(lsb_plan* plan, const void* device_src, void* stream);

/* Steps taken since lsb_init. */
long lsb_step_count(const lsb_plan* plan);

/* Cell and tile counts after the last step (synchronises the stream);
 * counts has 4 entries: counts[0] interface-adjacent cells, counts[1]
 * LS-active tiles, counts[2] cells refilled in the last step, counts[3]
 * wall-adjacent cells (cells with a lattice link through a wall face). */
int lsb_get_counts(lsb_plan* plan, int* counts, void* stream);

/* Kernel timing: while enabled, every step records a pair of HIP events
 * around the bulk collide-stream kernel (the dominant kernel; one launch
 * per step), on the stream that kernel runs on.  Enabling clears the accumulator.
 * lsb_get_kernel_timing waits for the recorded events and returns the summed
 * kernel duration in milliseconds and the number of launches timed. */
int lsb_set_kernel_timing(lsb_plan* plan, int enable);
int lsb_get_kernel_timing(lsb_plan* plan, double* total_ms, long* launches);

/* ---------------------------------------------------------------------------
 * Reverse mode (differentiation pattern; not in the paper).  Gradient of the
 * gas centroid after n steps with respect to the surface tension sigma and
 * the initial level set phi0, under the decisions the forward steps took
 * (phase and band tags, cut and wall links, Bouzidi branch, upwind
 * directions, the clamp at +-B, refill events, the Godunov branches and
 * subcell-fix set of the reinitialisation).  D2Q9 with LSB_F64 or LSB_F32
 * storage only.  Adjoints are FP64.
 *
 * Use with time checkpoints (lsb_save_state every K steps of the forward
 * run).  Then, for each segment from the last to the first:
 * lsb_load_state(checkpoint), lsb_adjoint_record(K), for the last segment
 * lsb_adjoint_seed_centroid, then lsb_adjoint_reverse.  Finally
 * lsb_adjoint_initial.  Recording re-runs the forward kernels, which are
 * deterministic, so the recomputed decisions are the forward run's.
 *
 * lsb_adjoint_workspace_bytes: device bytes for segments of up to
 *   max_segment_steps steps (snapshots of every step's state and
 *   intermediates, and the adjoint arrays); the caller allocates them.
 * lsb_adjoint_bind: hands over that workspace (LSB_ENOMEM if too small).
 * lsb_adjoint_record: runs nsteps forward steps from the current state
 *   (serial schedule), recording them; the plan's state advances.
 * lsb_adjoint_seed_centroid: loss L = gas centroid coordinate `axis` (0 = x,
 *   1 = y) of the last recorded state, with the smoothed Heaviside of the
 *   integrals; clears all adjoints and seeds dL/dphi.
 * lsb_adjoint_reverse: reverses the recorded segment (synchronises the
 *   stream); the adjoint of its first state is kept for the previous segment.
 * lsb_adjoint_initial: after the segment that starts at step 0, reverses the
 *   initialisation (clamp of phi0 to +-B, initial geometry, hydrostatic
 *   initial density about the initial centroid unless rho0 was given) and
 *   writes dL/dphi0 (device array of N doubles; phi0 and u0 are the device
 *   arrays passed to lsb_init, u0 may be NULL) and dL/dsigma (host double).
 * LSB_EINVAL for an unsupported lattice, storage or parameter, LSB_ESTATE
 * for a wrong call order. */
int lsb_adjoint_workspace_bytes(const lsb_plan* plan, int max_segment_steps, size_t* bytes);
int lsb_adjoint_bind(lsb_plan* plan, void* device_workspace, size_t bytes, int max_segment_steps);
int lsb_adjoint_record(lsb_plan* plan, int nsteps, void* stream);
int lsb_adjoint_seed_centroid(lsb_plan* plan, int axis, void* stream);
int lsb_adjoint_reverse(lsb_plan* plan, void* stream);
int lsb_adjoint_initial(lsb_plan* plan, const double* phi0, const double* u0, int rho0_given, double* dL_dphi0,
                        double* dL_dsigma, void* stream);

/* Step schedule.  SERIAL: every kernel of a step runs on the caller's
 * stream.  OVERLAP: the collide-stream of the cells outside the LS-active
 * tiles runs on a library-owned stream (default priority), concurrently
 * with the collide-stream of the band, interface and wall cells and the
 * level-set chain on the caller's stream; each lsb_step call returns with
 * the caller's stream ordered after all of its work.  Both give bit-identical
 * results.  Call between steps (the default is SERIAL); LSB_EINVAL for an
 * unknown schedule. */
enum { LSB_SCHED_SERIAL = 0, LSB_SCHED_OVERLAP = 1 };
int lsb_set_schedule(lsb_plan* plan, int schedule);

const char* lsb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LSB_H */
