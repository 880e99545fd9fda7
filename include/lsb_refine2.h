/* The two-phase step on a two-level grid (C ABI).
 *
 * The paper keeps the interface on its finest refinement level, with the
 * same level on both sides of it (Sec. 3.2), and couples its levels after
 * Dupuis and Chopard: populations missing at a refinement jump come from
 * the other level by interpolation in space and time, with the relaxation
 * time of eq. (omega) taken per level for one viscosity (Sec. 2.1).  This
 * module runs that arrangement with one refined box, ratio 2:
 *
 *   coarse grid  nx x ny (x nz) nodes, periodic on every face, each node in
 *                one phase (gas where phi >= 0 at initialisation); every
 *                uncovered node runs the plain BGK step of its phase with
 *                that phase's body force (Sec. 2.1), FP64.
 *   fine level   the box [ia, ib] x [ja, jb] (x [ka, kb]) of coarse nodes
 *                at half spacing, (2 (ib - ia) + 1) (2 (jb - ja) + 1)
 *                (2 (kb - ka) + 1) nodes, fine node (i, j, k) at coarse
 *                coordinates (ia + i/2, ja + j/2, ka + k/2).  It runs the
 *                whole two-phase step of lsb.h (interface bounce-back with
 *                the stress jump, level set, reinitialisation, refill) in
 *                its own lattice units: tau_f = 2 tau_c - 1/2 per phase,
 *                sigma_f = 2 sigma_c, a_f = a_c / 2, band, pseudo-time steps
 *                and heaviside_eps in fine cells, the storage of params.
 *
 * One coarse step: the coarse nodes step, the box perimeter keeping its
 * pre-collision sets; then two fine steps.  A fine surface node takes each
 * population whose source lies outside the box from the perimeter sets,
 * linear in time (the mean of the two coarse time levels, then the new
 * one), the mean of the 2 (or 4) coarse nodes beside an odd fine coordinate,
 * the non-equilibrium part about the equilibrium of the interpolated moments
 * scaled by tau_f,k / (2 tau_c,k) of the node's phase k, plus one fine step
 * of body force (a pre-collision set lags the physical time by one step of
 * its own level).  After the second fine step the covered coarse nodes next
 * to the perimeter take f_eq + 2 (tau_c,k - 1) / tau_f,k (f - f_eq) plus
 * the coarse body force, from the coincident fine node's pre-collision
 * populations f less one fine step of force.
 *
 * The interface and its level-set band must stay inside the box: the fine
 * level's LS-active cells (the band dilated by one cell) keep 3 fine cells
 * from every box face; lsb_ref2_sensor and lsb_ref2_remesh move the box
 * with the interface.
 *
 * Conventions as in lsb.h: every function returns LSB_OK (0) or a negative
 * code (message from lsb_last_error); calls that take a stream enqueue work
 * on it; the library allocates no device memory (the caller binds a
 * workspace and keeps ownership of it and of every array it passes).
 */
#ifndef LSB_REFINE2_H
#define LSB_REFINE2_H

#include <stddef.h>
#include <stdint.h>

#include "lsb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lsb_ref2 lsb_ref2;

/* params: the coarse grid and both phases in coarse lattice units; every
 * face LSB_PERIODIC (coarse walls are not available on this path), both
 * phases LSB_BGK; init_hydrostatic is not read (the initial state is the
 * caller's).  box: ia, ib, ja, jb, ka, kb (ka, kb
 * ignored for D2Q9), inclusive coarse nodes, 1 <= ia, ib <= nx - 2 and
 * ib - ia >= 4, the same for j and (3D) k.  Host memory only.
 * LSB_EINVAL for a NULL pointer or anything outside these ranges or those of
 * lsb_create. */
int lsb_ref2_create(const lsb_params* params, const int* box, lsb_ref2** out);
void lsb_ref2_destroy(lsb_ref2* ref);

/* Device workspace: the coarse populations twice (FP64, [Q][node]), the
 * coarse phases, the perimeter sets at two time levels and the fine level's
 * lsb_plan workspace (with its ghost populations).  The caller keeps
 * ownership and keeps it alive while the handle is used; 256-byte aligned.
 * LSB_ENOMEM if too small. */
int lsb_ref2_workspace_bytes(const lsb_ref2* ref, size_t* bytes);
int lsb_ref2_bind(lsb_ref2* ref, void* device_workspace, size_t bytes);

/* Fine nodes per axis: shape[0] = x, shape[1] = y, shape[2] = z. */
int lsb_ref2_fine_shape(const lsb_ref2* ref, int* shape);

/* The fine level as an lsb_plan owned by the handle, for the queries of
 * lsb.h (lsb_get_fields, lsb_get_interface, lsb_get_populations,
 * lsb_get_integrals, ...; fine lattice units and cell coordinates).  It
 * must not be stepped, re-initialised, bound or destroyed by the caller. */
int lsb_ref2_fine(lsb_ref2* ref, lsb_plan** fine);

/* Initial state from device arrays: phi_c, rho_c [nx ny nz] and u_c
 * [nx ny nz][3] on the coarse nodes (x fastest; equilibria, the phase from
 * the sign of phi_c), phi_f (signed distance in fine cells), rho_f and u_f
 * [.][3] on the fine nodes (lsb_init of the fine level).
 * LSB_ESTATE before lsb_ref2_bind. */
int lsb_ref2_init(lsb_ref2* ref, const double* phi_c, const double* rho_c, const double* u_c, const double* phi_f,
                  const double* rho_f, const double* u_f, void* stream);

/* nsteps coarse steps (2 nsteps fine steps), then one synchronisation of
 * the stream to read the band check.  LSB_EBAND if the fine level's
 * LS-active cells came within 3 fine cells of a box face in any step so far
 * (the steps still ran; the result is no longer that of the method);
 * LSB_ESTATE before lsb_ref2_init. */
int lsb_ref2_step(lsb_ref2* ref, int nsteps, void* stream);
long lsb_ref2_step_count(const lsb_ref2* ref);

/* Coarse post-collision populations pop [Q][nx ny nz] (FP64) and phases
 * phase [nx ny nz] (0 liquid, 1 gas) into device arrays (either may be
 * NULL).  Covered nodes hold the fine state restricted to the coarse level
 * (f_eq + 2 (tau_c - 1) / tau_f (f - f_eq) plus the coarse force, from the
 * coincident fine node's pre-collision populations less one fine step of
 * force), restricted every step. */
int lsb_ref2_get_coarse(lsb_ref2* ref, double* pop, uint8_t* phase, void* stream);

/* The current box (6 ints; ka = kb = 0 in 2D). */
int lsb_ref2_get_box(const lsb_ref2* ref, int* box);

/* Re-meshing: the box keeps its extents and follows the interface (the
 * paper's level-set sensor, Sec. 3.2, refines the gas and a band around
 * it; its tree refines cell by cell, here one box moves).
 *
 * lsb_ref2_sensor: the fine cells with phi >= -d_ref (fine cells; the gas
 * and a band of width d_ref around it) are tagged, and box (host, 6 ints)
 * receives the current box moved so that the centre of their bounding box
 * falls on its centre, rounded half up to whole coarse nodes, clamped one
 * node inside the grid faces; the current box when nothing is tagged.
 * Synchronises the stream.
 *
 * lsb_ref2_remesh: between coarse steps, onto box (host, 6 ints) of the
 * same extents.  Fine nodes inside the old box keep their state; the others
 * take the coarse post-collision populations H interpolated as at the
 * perimeter, with u = m/rho: f_eq(rho, u - a_f) + (tau_f - 1) / (2 (tau_c -
 * 1)) (H - F_c - f_eq(rho, u - a_c)) + F_f (F the levels' body forces; no
 * non-equilibrium part at tau_c = 1), and the level set +-band by the
 * coarse phase.  The fine level's tags, band, geometry and bubbles are
 * built again, its initial gas centroid moves with its coordinates (the
 * gas pressure baseline is unchanged), and the new perimeter's pre-collision
 * sets are inverted from the coarse state, f_eq(rho, u - a_c) + tau_c /
 * (tau_c - 1) (f - F_c - f_eq(rho, u - a_c)).  Synchronises the stream.
 * LSB_EINVAL for other extents or a box without a node to spare at a grid
 * face; LSB_EBAND if the band does not fit the new box (the re-mesh is
 * done; move the box again); LSB_ESTATE before lsb_ref2_init. */
int lsb_ref2_sensor(lsb_ref2* ref, double d_ref, int* box, void* stream);
int lsb_ref2_remesh(lsb_ref2* ref, const int* box, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LSB_REFINE2_H */
