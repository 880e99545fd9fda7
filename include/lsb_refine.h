/* Static grid refinement of the lattice Boltzmann solver, two to four
 * nested levels (C ABI).
 *
 * The paper refines its lattice Boltzmann grid after Dupuis and Chopard:
 * distributions missing at a refinement jump are obtained by spatial and
 * temporal interpolation between the known neighbouring distributions, and
 * the collision frequency of eq. (omega) is taken with each level's time
 * step so that the viscosity is the same on all levels (Sec. 2, lattice
 * Boltzmann method).  This module runs that coupling for one static fine
 * patch, refinement ratio 2, D2Q9, D3Q19 or D3Q27, BGK collision (eq. (feq)
 * equilibrium), FP64, in a coarse grid periodic on every axis.  The fine
 * level sub-cycles: two fine steps per coarse step, with
 * tau_f = 2 tau_c - 1/2.
 *
 * Geometry (cell-vertex): coarse node (I, J, K), I in [0, nx), J in
 * [0, ny), K in [0, nz); the patch covers the coarse nodes [ia, ib] x
 * [ja, jb] (x [ka, kb]) at half spacing, fine node (i, j, k) at coarse
 * coordinates (ia + i/2, ja + j/2, ka + k/2), i in [0, 2 (ib - ia)], and
 * so on.  Coarse nodes strictly inside the box are covered (their
 * populations are restricted from the coincident fine nodes); those on its
 * boundary are perimeter nodes.
 *
 * One coarse step: every uncovered coarse node pulls and collides with
 * tau_c, the perimeter nodes keeping their pre-collision populations; then
 * two fine steps, where a fine perimeter node takes each population whose
 * source lies outside the patch from the coarse perimeter: linear in time
 * (the mean of the two coarse time levels, then the new one), along each
 * odd fine coordinate the mean of the two coarse nodes beside it (2, or 4
 * at a face centre), and the non-equilibrium part about the equilibrium of
 * the interpolated moments scaled by tau_f / (2 tau_c); the second fine
 * step writes each covered
 * coarse node f_eq + 2 (tau_c - 1) / tau_f (f - f_eq) from the coincident
 * fine node's pre-collision populations f.
 *
 * Nested levels: level 1 may hold a patch of level 2 (and level 2 one of
 * level 3), a box of its own nodes with one node to spare at every side;
 * each pair of adjacent levels is coupled as above, tau doubles minus 1/2
 * from level to level, and every sub-step of a level is followed by its
 * child's two sub-steps, the second of which restricts into the level's new
 * populations.  A level restricts into its parent from its own
 * pre-collision populations (at nodes its child covers, those come from the
 * child's restriction).
 *
 * Conventions as in lsb.h: every function returns LSB_OK (0) or a negative
 * code of lsb.h (message from lsb_last_error); calls that take a stream
 * enqueue work on it and return without waiting; the library allocates no
 * device memory (the caller binds a workspace).
 */
#ifndef LSB_REFINE_H
#define LSB_REFINE_H

#include <stddef.h>

#include "lsb.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LSB_REF_MAX_LEVELS 4
#define LSB_REF_MAX_BOXES 15

typedef struct lsb_ref_params {
  int lattice;      /* LSB_D2Q9, LSB_D3Q19 or LSB_D3Q27 */
  int nx, ny, nz;   /* coarse nodes, >= 4 per axis; nz = 1 for D2Q9 */
  int patch[6];     /* ia, ib, ja, jb, ka, kb: coarse node box of the fine patch, inclusive;
                       1 <= ia, ib <= nx - 2, ib - ia >= 2, the same for j and (3D) k;
                       ka, kb ignored for D2Q9 */
  double tau_c;     /* coarse relaxation time, > 1/2 */
  int max_extent[3]; /* largest patch extents (coarse cells per axis) that lsb_ref_remesh may
                        choose; 0 or anything below the initial patch's extent keeps that
                        extent; at most n - 3 */
  int levels;       /* 2 .. LSB_REF_MAX_LEVELS (0 is read as 2) */
  int inner[LSB_REF_MAX_LEVELS - 2][6]; /* inner[l - 2]: box of level l in level l - 1's node
                        coordinates (nodes 0 .. m per axis, m = twice the parent box's
                        extent): 1 <= a, b <= m - 1, b - a >= 2 per axis; ka, kb ignored in
                        2D; unused entries ignored */
  int max_inner_extent[LSB_REF_MAX_LEVELS - 2][3]; /* largest extents (parent cells per axis) that
                        lsb_ref_remesh_levels may choose for level l (entry l - 2); 0 or
                        anything below the initial box's extent keeps that extent; at most
                        twice the parent's largest extent minus 2 */
} lsb_ref_params;

typedef struct lsb_ref lsb_ref;

/* Validates the parameters and creates a handle (host memory only).
 * LSB_EINVAL for a NULL pointer, an unknown lattice, parameters outside
 * the ranges above, or a level of more than 2^31 nodes (with the ghost
 * shell). */
int lsb_ref_create(const lsb_ref_params* params, lsb_ref** out);

/* A tree of boxes instead of a chain: box b (1 .. nbox) refines grid
 * parents[b - 1] (0: the coarse grid, else an earlier box; parents[0] = 0)
 * over boxes[6 (b - 1) ...] = (ia, ib, ja, jb, ka, kb) of that grid's nodes,
 * with one node to spare at every side, at least two cells per axis, and
 * the boxes refining one grid at least one of its nodes apart (each pair of grids is coupled as above; a grid's
 * sub-step is followed by each of its boxes' two sub-steps in turn).
 * params gives the lattice, the coarse grid, tau_c and box 1's max_extent;
 * its patch, levels, inner and max_inner_extent are not read.  Grid b's
 * arrays in lsb_ref_init_levels and lsb_ref_get_level are box b's;
 * lsb_ref_remesh_levels re-meshes a tree (box 1 up to max_extent, every
 * other box up to its initial extents), the sensor takes chains only
 * (LSB_EINVAL for a tree).
 * LSB_EINVAL for anything outside these ranges. */
int lsb_ref_create_tree(const lsb_ref_params* params, int nbox, const int* parents, const int* boxes,
                        lsb_ref** out);
void lsb_ref_destroy(lsb_ref* ref);

/* Device workspace the caller provides: every level's populations twice
 * (double buffers, level 1 sized for the largest patch) and each refined
 * level's perimeter sets from its parent at two time levels.  The library
 * keeps the pointer; the caller keeps ownership and must keep it alive
 * while the handle is used.  LSB_ENOMEM if it is too small. */
int lsb_ref_workspace_bytes(const lsb_ref* ref, size_t* bytes);
int lsb_ref_bind(lsb_ref* ref, void* device_workspace, size_t bytes);

/* Equilibrium initial state of a two-level hierarchy from device arrays:
 * rho_c [nx*ny*nz], u_c [nx*ny*nz*D] (D components per node, x fastest over
 * the nodes), rho_f and u_f the same over the fine nodes ((2(ib-ia)+1)
 * (2(jb-ja)+1) (2(kb-ka)+1) in 3D, i fastest).  The coarse perimeter's
 * pre-collision sets start at those equilibria.
 * LSB_ESTATE before lsb_ref_bind; LSB_EINVAL with more than two levels. */
int lsb_ref_init(lsb_ref* ref, const double* rho_c, const double* u_c, const double* rho_f, const double* u_f,
                 void* stream);

/* The same for any number of levels: rho[l] and u[l] (host arrays of
 * `levels` device pointers) over level l's nodes, laid out as above.
 * LSB_ESTATE before lsb_ref_bind. */
int lsb_ref_init_levels(lsb_ref* ref, const double* const* rho, const double* const* u, void* stream);

/* nsteps coarse steps (2^l nsteps steps of level l).  A coarse step is
 * launched as a HIP graph (two graphs, one per parity of the double
 * buffers, captured on the first call after lsb_ref_bind, lsb_ref_init or
 * a re-mesh; the graphs are runtime objects, not device memory of the
 * library).  LSB_ESTATE before lsb_ref_init; LSB_EDEVICE if a capture or a
 * launch fails. */
int lsb_ref_step(lsb_ref* ref, int nsteps, void* stream);

/* Graph launches on (on != 0, the default) or plain kernel launches; both
 * give the same results bit for bit. */
int lsb_ref_set_graphs(lsb_ref* ref, int on);

/* Level-set refinement sensor (Sec. 3, adaptive mesh refinement): from a
 * level set on the coarse nodes (device array [nx*ny*nz], negative in the
 * liquid, >= 0 in the gas: the opposite of the sign the paper's sensor is
 * written with), the coarse nodes with phi >= -d_ref (the gas and a band of
 * width d_ref around it) are tagged, and patch (host, 6 ints: ia, ib, ja,
 * jb, ka, kb; ka = kb = 0 in 2D) receives their bounding box grown by margin
 * nodes, clamped to keep one node at each grid face and widened to two
 * cells per axis; the current patch when no node is tagged.  Synchronises
 * the stream.  LSB_EINVAL for a NULL pointer or a negative margin. */
int lsb_ref_sensor(lsb_ref* ref, const double* phi, double d_ref, int margin, int* patch, void* stream);

/* Re-meshing onto a new patch (host, 6 ints as above) between coarse steps:
 * fine nodes inside the old patch keep their populations; the others take
 * the coarse post-collision populations interpolated like the perimeter's
 * (the mean of the 2, 4 or 8 coarse nodes around an off-grid node), the
 * non-equilibrium part scaled by (tau_f - 1) / (2 (tau_c - 1)) about the
 * equilibrium of the interpolated moments (the equilibrium alone at
 * tau_c = 1); the new perimeter's pre-collision sets come from inverting
 * the coarse BGK step.  LSB_EINVAL for a patch outside the grid or larger
 * than max_extent, or a hierarchy of more than two levels; LSB_ESTATE
 * before lsb_ref_init. */
int lsb_ref_remesh(lsb_ref* ref, const int* patch, void* stream);

/* The sensor for every refined level: the tagged coarse nodes' bounding box
 * (as lsb_ref_sensor, tagging phi >= -d_ref) grown by margins[l - 1] coarse
 * nodes for level l, written in the parent's node coordinates (coarse node
 * X is node 2^(l-1) X - o of the parent, o its first node's index in its
 * own spacing counted from coarse node 0), clamped to keep one parent node
 * at each side and widened to two cells per axis; levels in order, each
 * inside the one computed before it.  boxes (host) receives 6 ints per
 * refined level, ka = kb = 0 in 2D; the current boxes when no node is
 * tagged.  Synchronises the stream.  LSB_EINVAL for a NULL pointer or a
 * negative margin. */
int lsb_ref_sensor_levels(lsb_ref* ref, const double* phi, double d_ref, const int* margins, int* boxes,
                          void* stream);

/* The sensor for a tree of boxes refining the coarse grid: every tagged
 * coarse node (phi >= -d_ref, as lsb_ref_sensor) belongs to its nearest
 * seed (seeds: host, nseeds coarse nodes of 3 ints, z ignored in 2D, for
 * example the rounded centroids of bubbles; squared distances compared as
 * integers, ties to the lower index); each seed with tagged nodes gives
 * their bounding box grown by margin, clamped one node inside the grid and
 * widened to two cells per axis; boxes closer than one node apart merge
 * into their union (in the earlier box's place) until every pair is apart.
 * boxes (host, 6 ints per box, room for nseeds) and *nboxes receive the
 * result, the input of lsb_ref_create_tree (parents all 0) or of
 * lsb_ref_remesh_levels on a tree of that many root boxes.  Synchronises
 * the stream.  LSB_EINVAL for a NULL pointer, a negative margin or nseeds
 * outside [1, LSB_REF_MAX_BOXES]; LSB_ESTATE before lsb_ref_bind. */
int lsb_ref_sensor_seeded(lsb_ref* ref, const double* phi, double d_ref, int margin, int nseeds, const int* seeds,
                          int* boxes, int* nboxes, void* stream);

/* Re-meshing of every box of a chain or a tree (boxes: host, 6 ints per
 * box, each in its new parent's node coordinates; the tree's shape stays),
 * box 1 first, each inside its re-meshed parent and, in a tree, at least
 * one parent node from its siblings, with the rules of lsb_ref_remesh per
 * pair of grids: a new node at a position the old level covered keeps its
 * populations, the others are interpolated from the parent's post-collision
 * populations with the non-equilibrium part scaled by
 * (tau_l - 1) / (2 (tau_{l-1} - 1)), and each level's perimeter sets come
 * from inverting the parent's BGK step.  nboxes is the number of boxes
 * given and must equal the hierarchy's refined grids (levels - 1; the
 * seeded sensor may return fewer boxes than a tree has when boxes merge:
 * such a result needs a new tree, lsb_ref_create_tree).  LSB_EINVAL for
 * nboxes != levels - 1 (checked first, before any other access), a box
 * outside its parent (one node to spare, two cells per axis) or beyond the
 * workspace's extents; LSB_ESTATE before lsb_ref_init. */
int lsb_ref_remesh_levels(lsb_ref* ref, const int* boxes, int nboxes, void* stream);

/* Post-collision populations of both levels into device arrays, [Q][nodes]
 * in the paper's direction ordering (rest direction last): coarse
 * [Q][nz][ny][nx] (covered nodes hold the restricted values), fine
 * [Q][2(kb-ka)+1][2(jb-ja)+1][2(ib-ia)+1] (one z layer in 2D).
 * Either pointer may be NULL.  LSB_ESTATE before lsb_ref_init. */
int lsb_ref_get_populations(lsb_ref* ref, double* coarse, double* fine, void* stream);

/* Post-collision populations of one level (0 = coarse) into a device array,
 * [Q][nodes of that level] as above.  LSB_EINVAL for a level outside
 * [0, levels); LSB_ESTATE before lsb_ref_init. */
int lsb_ref_get_level(lsb_ref* ref, int level, double* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LSB_REFINE_H */
