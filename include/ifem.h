/*
 * ifem.h -- C ABI of the MI355X (gfx950) IFEM coupling-step library.
 *
 * One coupling step of the immersed-finite-element method of Saadat, Guido,
 * Iaccarino & Shaqfeh (arXiv 1807.08219), Sec. III.A, steps 1, 2 and 4:
 *
 *   ifem_element_forces  internal nodal forces of every Lagrangian particle
 *                        (Sec. II.B: eq. FEM for tetrahedral solids, eq.
 *                        FEM_Membrane for membranes, the Helfrich bending
 *                        force) plus FP64 per-particle volume, area and
 *                        centroid (Sec. II.E volume formula);
 *   ifem_spread          F_J = sum_k phi_J(x_J - x_k) F_k onto the staggered
 *                        Eulerian lattices (Sec. II.C spreading operator);
 *   ifem_interp          v_k = sum_J phi_J(x_J - x_k) v_J back to the nodes
 *                        (Sec. II.C interpolation operator);
 *
 * for viscoelastic suspensions, the interpolation of the conformation tensor
 * to the nodes (ifem_interp_cells, Sec. III.A step 4) and the fluid-stress
 * forces on solids (ifem_fluid_forces, Sec. II.B eq. FEM, Sec. III.A step 1);
 * and the end of a time step (Sec. III.A, last step; Sec. III.B): the second-order
 * Adams-Bashforth update of the positions (ifem_advance) and the membrane
 * volume correction of Sec. II.E (ifem_volume_correct) and the node-face
 * anti-sticking of Sec. III.B (ifem_antistick),
 *
 * with phi the linear moving-least-squares weights of Sec. II.C (27-node
 * stencil around the nearest lattice node, cubic-spline weight, support
 * sqrt(3) h).
 *
 * Conventions
 * -----------
 * Every array passed to the step calls is DEVICE memory owned by the
 * caller; the library never frees or reallocates it.  Inputs are not
 * modified; outputs are overwritten (never accumulated, except the
 * documented in-out forces of ifem_fluid_forces).  An output may not alias an
 * input (except in place where a call says so): that is rejected with
 * IFEM_ERR_INVALID_ARG.
 *
 * Layouts (structure of arrays, 32-bit indices):
 *   positions, forces, velocities   [3][n_nodes]  (component-major)
 *   grid fields                     [3][total_cells], component d of box b at
 *                                   d * total_cells + cell_offset[b] + (k*ny + j)*nx + i
 *   tri / tet connectivity          [3][n_tris] / [4][n_tets], global node ids,
 *                                   triangles counter-clockwise seen from outside,
 *                                   tetrahedra with positive reference volume.
 * Nodes, triangles and tetrahedra are contiguous per particle.
 *
 * Precisions (`dtype`):
 *   IFEM_F64  positions are absolute float64; forces, grids, velocities float64;
 *             `anchor` must be NULL.
 *   IFEM_F32  positions are float32 offsets from a per-particle float64 anchor
 *             (`anchor` [n_particles][3], device, required): the node position
 *             is anchor[p] + (double)offset.  Forces, grids, velocities float32.
 *             Strain invariants are formed without cancellation (membranes:
 *             the metric difference g - G error-free in float-float;
 *             tetrahedra: exact edges, the deformation gradient in float64).
 *   Per-particle reductions are float64 in both precisions.
 *
 * Lattices: box b has n = (nx, ny, nz) cells of spacing h, periodic on every
 * axis.  Component d of the velocity/force lives at origin + (i + s_d) h with
 * s_d = 1/2 on the two axes other than d and 0 on axis d (MAC staggering).
 * The nearest-node rule is bit-specified: q = p - origin, t = fma(q, 1/h, -s),
 * base = floor(t + 1/2), computed in float64 in both precisions.
 *
 * Streams: `stream` is a hipStream_t passed as void*; NULL is the default
 * stream.  The step calls are asynchronous, allocate nothing and do not
 * synchronise, so a caller may capture them in a hipGraph.  A plan owns the
 * workspaces its calls use (spread lists and halos, contact cells and keys,
 * status counters): calls on one plan must be ordered (one stream, or streams
 * the caller synchronises); calls that overlap on one plan race on that
 * workspace.  Different plans are independent.
 *
 * Errors: every call returns IFEM_OK or a negative code; argument errors are
 * reported before anything is launched and ifem_last_error() (thread local)
 * describes the last failure.  Conditions found on the device do not fail
 * the call: they increment the plan's status counters (ifem_plan_status)
 *   counts[0]  degenerate or inverted elements (tet det F <= 0, triangle
 *              I2 <= 0); such an element contributes zero force;
 *   counts[1]  non-finite nodal force components written;
 *   counts[2]  points whose MLS moment matrix was singular (weights zero);
 *   counts[3]  nodes a tiled spread skipped because their nearest lattice
 *              node moved between binning and accumulation, or nodes the
 *              anti-sticking pass left unmoved because its second pass could
 *              not reproduce their least distance (in both cases: positions
 *              written concurrently with the call); 0 in normal use;
 *   counts[4]  membranes whose volume-correction multiplier did not converge
 *              (ifem_volume_correct; their nodes are moved by the last iterate).
 */
#ifndef IFEM_H
#define IFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ifem_status;
enum {
  IFEM_OK = 0,
  IFEM_ERR_INVALID_ARG = -1, /* bad pointer, count, layout or aliasing          */
  IFEM_ERR_UNSUPPORTED = -2, /* valid input outside what this build handles     */
  IFEM_ERR_DEVICE = -3,      /* a HIP runtime call failed                       */
  IFEM_ERR_DEGENERATE = -4,  /* reference element with non-positive area/volume */
  IFEM_ERR_NOMEM = -5        /* device allocation failed at plan creation       */
};

enum { IFEM_F32 = 0, IFEM_F64 = 1 };

/* Constitutive laws (Sec. II.A): neo-Hookean membrane, Skalak membrane,
 * slightly compressible neo-Hookean solid. */
enum { IFEM_LAW_TRI_NEOHOOKE = 0, IFEM_LAW_TRI_SKALAK = 1, IFEM_LAW_TET_NEOHOOKE = 2 };

/* Spreading algorithms: deterministic tile-owned LDS reduction (default), or
 * one global atomic add per (point, stencil node) -- the plain baseline. */
enum { IFEM_SPREAD_TILED = 0, IFEM_SPREAD_ATOMIC = 1 };

/* Plan options for ifem_plan_set.
 *   IFEM_OPT_SPREAD_MODE    IFEM_SPREAD_TILED or IFEM_SPREAD_ATOMIC.
 *   IFEM_OPT_KERNEL_TIMING  0 switches the per-kernel event timer off; n > 0
 *                           switches it on with room for n kernel launches
 *                           (2n HIP events created now, none per call).  While
 *                           on, every kernel a step call launches is bracketed
 *                           by events on the launch stream; read them with
 *                           ifem_plan_kernel_times.  Synchronises the device. */
enum { IFEM_OPT_SPREAD_MODE = 1, IFEM_OPT_KERNEL_TIMING = 2 };

/* Kernel slots reported by ifem_plan_kernel_times. */
enum {
  IFEM_KERNEL_FORCES = 0,        /* per-particle element, bending and reduction kernel */
  IFEM_KERNEL_BIN_COUNT = 1,     /* spread: home-tile list lengths (per node)           */
  IFEM_KERNEL_SCAN = 2,          /* spread: offsets of the home-tile lists              */
  IFEM_KERNEL_BIN_FILL = 3,      /* spread: fill of the home-tile lists                 */
  IFEM_KERNEL_SPREAD_HOME = 4,   /* spread: per-tile LDS accumulation and grid write    */
  IFEM_KERNEL_SPREAD_MERGE = 8,  /* spread: neighbour halos added to tile border cells  */
  IFEM_KERNEL_SPREAD_ATOMIC = 5, /* spread: plain global-atomic baseline                */
  IFEM_KERNEL_INTERP = 6,        /* interpolation                                       */
  IFEM_KERNEL_FILL = 7,          /* zero fills                                          */
  IFEM_KERNEL_VOLUME = 9,        /* membrane volume correction                          */
  IFEM_KERNEL_ADVANCE = 10,      /* Adams-Bashforth position update                     */
  IFEM_KERNEL_INTERP_CELLS = 11, /* interpolation of cell-centred fields                */
  IFEM_KERNEL_FLUID = 12,        /* fluid-stress forces on solids                       */
  IFEM_KERNEL_CONTACT = 13       /* node-face anti-sticking (all of its kernels)        */
};

/* Mesh description, HOST memory, read once by ifem_plan_create. */
typedef struct {
  int32_t n_particles, n_nodes, n_tris, n_tets;
  const int32_t* tri;        /* [3][n_tris] global node ids                                   */
  const int32_t* tet;        /* [4][n_tets] global node ids                                   */
  const int32_t* node_start; /* [n_particles + 1], node_start[0] = 0                         */
  const int32_t* tri_start;  /* [n_particles + 1]                                            */
  const int32_t* tet_start;  /* [n_particles + 1]                                            */
  const int32_t* law;        /* [n_particles] IFEM_LAW_*                                     */
  const double* mu;          /* [n_particles] shear modulus (membrane: per length)           */
  const double* mu2;         /* [n_particles] Skalak dilatation modulus / solid bulk modulus */
  const double* kb;          /* [n_particles] bending modulus (membranes; 0 = no bending)    */
  const double* c0;          /* [n_particles] spontaneous curvature                          */
  const int32_t* box;        /* [n_particles] index of the periodic box holding the particle */
  const double* X_ref;       /* [3][n_nodes] reference (stress-free) configuration           */
} ifem_mesh_desc;

/* One periodic Eulerian box, HOST memory.  Boxes are laid out one after the
 * other in the grid arrays, in the order given. */
typedef struct {
  int32_t n[3];
  double h;
  double origin[3];
} ifem_box;

/* Launch shape.  Pass NULL to ifem_plan_create for the shape that
 * ifem_plan_autotune last chose for plans of the same sizes on the same kind of
 * device, else the defaults {tile 32 x 16 x 8, block_forces 512, block_points
 * 256}, the fastest measured on dense red-cell suspensions and on sparse
 * boxes of mixed particles.  The spread region
 * of a tile, (tile_x + 5)(tile_y + 2)(tile_z + 2) cells, must not exceed 13568
 * (12 bytes of LDS per cell in float64). */
typedef struct {
  int32_t tile[3];      /* spread tile, cells per axis (powers of two, 4..64) */
  int32_t block_forces; /* threads per particle workgroup (power of two, 64..512) */
  int32_t block_points; /* threads per workgroup of the point kernels  */
} ifem_tuning;

typedef struct ifem_plan_s* ifem_plan;

/* Launch-shape autotuning.  Times the tiled spread on the caller's inputs for
 * each candidate tile shape that fits LDS (32x16x8, 16x16x16, 64x8x8,
 * 32x32x4, 16x32x8, 32x8x8, 16x16x8, 64x16x4, 32x16x16; the plan's spread
 * workspace is rebuilt for each, so the call allocates and frees device memory),
 * then the interpolation for block_points 64, 128 and 256 (median of five
 * calls after two untimed ones, each timed call after an untimed call of the
 * other transfer, as in a coupling step; HIP events on `stream`; 30 untimed
 * spread + interpolation pairs first bring the device's clocks up, and the
 * candidates are timed in order and again in reverse order, each keeping its
 * better median, so that a drift favours none), and leaves the plan
 * with the fastest: every later call of the plan uses it, and gives the same
 * results bit for bit as a plan created with that tuning.  The choice is
 * recorded for (current device, the plan's sizes: particle, node and element
 * counts, bending membranes, box lattices): a later ifem_plan_create with
 * tuning == NULL for the same sizes on the same kind of device takes it.  The
 * record lasts for the process; when the environment variable IFEM_TUNE_CACHE
 * names a file, it is also appended there and read back by later processes.
 * block_forces is not tuned (it shapes the element colouring made at plan
 * creation).
 *   x, anchor, F  positions and forces as for ifem_spread (dtype as there: the
 *                 tuning is for that precision), device
 *   grid          [3][total_cells] scratch output of the timed spreads
 *   grid_u        [3][total_cells] velocity for the timed interpolations
 *   v_out         [3][n_nodes] scratch output of the timed interpolations
 *   chosen        the tuning now in force, or NULL.
 * Synchronises the device; not for graph capture.  Outputs may not alias
 * inputs or each other. */
ifem_status ifem_plan_autotune(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, const void* F,
                               void* grid, const void* grid_u, void* v_out, void* stream, ifem_tuning* chosen);

/* Build a plan for one set of meshes and boxes (Sec. II.B reference
 * configuration): copies connectivity and materials to the device, computes
 * the float64 reference data of every element on the device (triangles their
 * metric and area, tetrahedra the inverse edge matrix and volume), colours the
 * elements of each particle for conflict-free accumulation, builds the
 * one-ring of every bending node and sizes the spreading workspace.  A
 * particle whose float64 nodal accumulators fit one workgroup's LDS (up to
 * 6741 nodes, 5056 when any particle bends) is handled by one workgroup; a
 * larger one by the global-memory path (element forces into a scratch slot
 * per corner, then a fixed-order gather per node), with the same results to
 * rounding and the same run-to-run bits; there is no size limit beyond the
 * 32-bit counts.  Returns IFEM_ERR_DEGENERATE if a reference element has
 * non-positive area or volume, IFEM_ERR_UNSUPPORTED for a non-manifold
 * bending surface.  Synchronises `stream`.
 * tuning == NULL selects the default launch shape (see ifem_tuning). */
ifem_status ifem_plan_create(const ifem_mesh_desc* mesh, const ifem_box* boxes, int32_t n_boxes,
                             const ifem_tuning* tuning, void* stream, ifem_plan* out);
ifem_status ifem_plan_destroy(ifem_plan plan);

/* Set an option (IFEM_OPT_SPREAD_MODE: IFEM_SPREAD_TILED or IFEM_SPREAD_ATOMIC). */
ifem_status ifem_plan_set(ifem_plan plan, int32_t option, int64_t value);

/* Read back the plan's geometry: info[0] total_cells, info[1] n_nodes,
 * info[2] n_particles, info[3..5] tile, info[6] block_forces,
 * info[7] block_points, info[8] workspace bytes, info[9] spread mode. */
ifem_status ifem_plan_info(ifem_plan plan, int64_t info[10]);

/* Step 1 of the algorithm (Sec. III.A): internal nodal forces.
 *   x        [3][n_nodes] positions (see dtype), device
 *   anchor   [n_particles][3] float64 anchors (IFEM_F32) or NULL (IFEM_F64)
 *   f_out    [3][n_nodes] nodal forces: elastic (eq. FEM / FEM_Membrane) plus
 *            Helfrich bending for membranes with kb != 0
 *   red_out  [n_particles][5] float64 {volume, area, centroid x, y, z} or NULL.
 *            Membranes: enclosed volume and surface area; solids: volume and 0.
 */
ifem_status ifem_element_forces(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, void* f_out,
                                double* red_out, void* stream);

/* Step 2 (Sec. III.A): spread nodal forces F [3][n_nodes] to grid [3][total_cells].
 * The grid holds forces (its sum equals the Lagrangian total), not densities.
 * IFEM_SPREAD_TILED (default) sums in 64-bit fixed point per lattice tile:
 * bitwise reproducible, no global float atomics; every finite force of
 * either precision is held (the fixed-point scale of a tile's list follows a
 * power-of-two bound on its largest |F|).  A non-finite force component, or a
 * node whose position is not finite (its MLS system has no solution: counted
 * in counts[2]), cannot be held in fixed point: it turns the tiles that take
 * its stencil (its home tile and at most one x-neighbour; a non-finite
 * position is binned at lattice index 0), plus their one-cell y/z halos, into
 * NaN for that component (the plain IFEM_SPREAD_ATOMIC mode spreads it to the
 * 27 stencil cells only).  The plan keeps each call's list lengths to lay out
 * the next call's lists, so that the node lists are written in one pass over
 * the nodes while positions move by less than the room left in each list (a
 * second pass fills the lists that outgrew theirs, and every list on the
 * plan's first call); the grid does not depend on it. */
ifem_status ifem_spread(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, const void* F,
                        void* grid, void* stream);

/* For callers that cannot allocate device memory while they step (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * ifem_spread in the tiled mode (whatever IFEM_OPT_SPREAD_MODE says), with the
 * same kernels and the same result bit for bit, whose workspace (list counts,
 * offsets, cursors, flags, force bounds, placement totals, node lists and
 * halo rows) lives in a static device array of the library, 64 MiB per GPU,
 * held from the library's first use of a device until the process ends,
 * instead of the plan's.  The call allocates nothing, synchronises nothing and
 * is graph-capturable; the array's address on each device is looked up once,
 * on the first call there.  Returns IFEM_ERR_UNSUPPORTED, before launching
 * anything, when the plan's workspace does not fit: 5 (3 n_tiles) int32 + 2
 * int32 + the node lists (6 or 9 int32 per node) + 3 n_tiles tile_x (2
 * (tile_y + tile_z) + 4) values of the call's precision, each part rounded up
 * to 256 bytes (a 128^3 grid with 32 x 16 x 8 tiles takes 21 MB in float64).
 * Every call on one GPU uses that GPU's one array, whatever the plan: calls
 * that overlap on a GPU (on different streams or host threads, with any
 * plans) race on it and must be ordered by the caller.  The array keeps the
 * last call's contents; each call clears what it needs cleared.  Arguments and
 * errors as ifem_spread. */
ifem_status ifem_spread_noalloc(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, const void* F,
                                void* grid, void* stream);

/* Step 4 (Sec. III.A): interpolate grid velocity grid_u [3][total_cells] to the nodes, v_out [3][n_nodes]. */
ifem_status ifem_interp(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, const void* grid_u,
                        void* v_out, void* stream);

/* Membrane volume conservation (Sec. II.E, conservation of volume for
 * membranes), applied to positions after they have been advanced.  For every
 * membrane the nodes move by dx_I = L alpha_I: alpha_I = -(1/2) dV/dx_I is the
 * stationary direction of the section's cost function (sum of squared nodal
 * displacements plus a multiplier times the volume error), and L is the real
 * root of smallest magnitude of the cubic A L^3 + B L^2 + C L + D = 0 with the
 * section's coefficients, D = V(x) - V0, so that the enclosed volume after the
 * move equals V0.  L is found by Newton's iteration from 0 (counts[4] of
 * ifem_plan_status counts membranes where it did not converge).  Everything is
 * computed in float64.  Solids (tetrahedral particles) are copied unchanged.
 *   x           [3][n_nodes] positions (see dtype), device.  IFEM_F32: float32
 *               offsets from the caller's per-particle anchors; the correction
 *               does not depend on the anchors (volume and alpha are unchanged by
 *               a translation of a closed surface), so none is passed, and x_out
 *               holds offsets from the same anchors.
 *   V0          [n_particles] float64 target volumes, device, or NULL for the
 *               volumes of the reference configuration X_ref (computed by
 *               ifem_plan_create); entries of solids are ignored.
 *   x_out       [3][n_nodes] corrected positions, same dtype.  x_out == x
 *               corrects in place; any other overlap with an input is rejected.
 *   lambda_out  [n_particles] float64 multipliers L (0 for solids), or NULL.
 * Returns IFEM_ERR_UNSUPPORTED if a membrane's triangles do not form a closed,
 * consistently oriented surface (its enclosed volume is then undefined).
 * Membranes above the one-workgroup size take a global-memory path of four
 * launches (alpha, beta, the multiplier, the move). */
ifem_status ifem_volume_correct(ifem_plan plan, int32_t dtype, const void* x, const double* V0, void* x_out,
                                double* lambda_out, void* stream);

/* Interpolation of cell-centred fields to the nodes (Sec. III.A step 4: the
 * conformation tensor C_k = sum_J phi_J(x_J - x_k) C_J).  The fields live at
 * the cell centres origin + (i + 1/2, j + 1/2, k + 1/2) h of every box (the
 * fourth lattice beside the three velocity lattices), with the same MLS
 * weights and stencil rule.
 *   grid  [ncomp][total_cells] (same dtype), device; for the conformation
 *         ncomp = 6 in the order xx, yy, zz, xy, xz, yz.
 *   out   [ncomp][n_nodes], overwritten.
 *   ncomp 1..64.  Singular MLS systems are counted in counts[2]. */
ifem_status ifem_interp_cells(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, const void* grid,
                              int32_t ncomp, void* out, void* stream);

/* Fluid-stress forces on solids (Sec. II.B: the Newtonian and polymer parts of
 * eq. FEM, F_k = -V0 (P^s - P^fN - P^fP) grad N_k; Sec. III.A step 1), ADDED
 * to f_inout for the nodes of every tetrahedral particle (membrane nodes are
 * left as they are).  Per element, with L the velocity gradient of the
 * interpolated nodal velocities:
 *   P^fN = eta J (L + L^T) F^-T,  P^fP = J G (C_avg - I) F^-T,
 * C_avg the mean of the element's four nodal conformation tensors.  eta is the
 * Newtonian viscosity, G the polymer modulus eta_p / lambda (eta (1 - beta) /
 * lambda in the paper's notation, with eta the total viscosity there).  The
 * kernel uses the equal current-configuration form V sigma grad_x N_k; float64
 * arithmetic.  Inverted or flat elements contribute nothing (ifem_element_forces
 * counts them).
 *   x        [3][n_nodes] positions (see dtype; float32 offsets need no anchor:
 *            the forces do not change under a translation), device.
 *   v        [3][n_nodes] nodal velocities, same dtype.
 *   C        [6][n_nodes] nodal conformation (xx, yy, zz, xy, xz, yz), same
 *            dtype, or NULL for a Newtonian fluid (G is then unused).
 *   eta, G   finite.
 *   f_inout  [3][n_nodes] nodal forces, same dtype, read and written; it may
 *            not overlap an input. */
ifem_status ifem_fluid_forces(ifem_plan plan, int32_t dtype, const void* x, const void* v, const void* C, double eta,
                              double G, void* f_inout, void* stream);

/* Lagrangian update (Sec. III.A, last step of the algorithm): second-order
 * Adams-Bashforth with the interpolated velocities of this step and the last,
 *   x_out = x + dt (3/2 v - 1/2 v_prev),
 * or the forward Euler step x + dt v when v_prev is NULL (the first step).
 * Arithmetic is float64 in the order written, without fused multiply-add.
 *   x, x_out     [3][n_nodes] positions (see dtype), device.  IFEM_F32: float32
 *                offsets from the caller's anchors; x_out holds offsets from the
 *                same anchors (the displacement is added in float64 and the
 *                offset rounded once).  x_out == x updates in place.
 *   v, v_prev    [3][n_nodes] velocities in the same dtype, device (v_prev may
 *                be NULL); neither may overlap x_out.
 *   dt           time step (finite). */
ifem_status ifem_advance(ifem_plan plan, int32_t dtype, const void* x, const void* v, const void* v_prev, double dt,
                         void* x_out, void* stream);

/* Node-face anti-sticking (Sec. III.B, resolving numerical sticking): every
 * node closer than d_min to a face of another particle of its periodic box is
 * moved away from the closest point c of that face to c + d_min (x - c)/|x - c|
 * (along the face normal when x lies on the face).  Faces are the membrane
 * triangles (face id = triangle index) and the boundary faces of the solids'
 * tetrahedral meshes (ids n_tris + k, listed by tetrahedron and local face
 * opposite node j = 0..3, oriented outward in X_ref).  The closest face is the
 * one of least float64 distance, exact ties (faces sharing the closest edge or
 * vertex) to the lower id; a node moves when that distance is below d_min.
 * Distances use the periodic minimum image; every node is tested against the positions
 * before the call (no node sees another's move).  Exact search: a uniform grid
 * of contact cells about two lattice cells wide per box replaces the paper's
 * bounding-box broad phase.  A face that is not finite or spans more than half
 * a box is skipped.  One pass; a node pushed out of one particle's range into
 * another's is not checked again.
 *   x, anchor  positions (see dtype), device.
 *   d_min      separation, 0 < d_min <= the contact-cell width (box length /
 *              max(1, floor(n / 2)) per axis) and <= a quarter box; the paper
 *              uses one lattice spacing h.
 *   x_out      [3][n_nodes] moved positions, same dtype (float32: offsets from
 *              the same anchors); must not overlap x.
 *   face_out   [n_nodes] int64, device, or NULL: the face that moved each node,
 *              -1 for nodes that stay. */
ifem_status ifem_antistick(ifem_plan plan, int32_t dtype, const void* x, const double* anchor, double d_min,
                           void* x_out, int64_t* face_out, void* stream);

/* Synchronise `stream` and the timer's events; total_ms[i] and launches[i]
 * receive the summed duration and number of launches of kernel slot i
 * (IFEM_KERNEL_*) recorded since the last reset; launches[15] counts launches
 * not recorded because the event pool was full.  reset != 0 empties the pool. */
ifem_status ifem_plan_kernel_times(ifem_plan plan, void* stream, double total_ms[16], int64_t launches[16],
                                   int32_t reset);

/* Synchronise `stream`, copy the device status counters into counts[5] and,
 * if reset != 0, clear them. */
ifem_status ifem_plan_status(ifem_plan plan, void* stream, int64_t counts[5], int32_t reset);

/* Thread-local description of the last non-OK return ("" if none). */
const char* ifem_last_error(void);

/* Library version, e.g. 10400 for 1.4.0. */
int32_t ifem_version(void);

#ifdef __cplusplus
}
#endif
#endif /* IFEM_H */
