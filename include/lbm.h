/*
 * lbm.h -- C ABI of the MI355X (gfx950) D3Q19 lattice Boltzmann library with
 * the on-site velocity boundary condition of M. Hecht and J. Harting,
 * "Implementation of on-site velocity boundary conditions for D3Q19 lattice
 * Boltzmann" (arXiv:0811.4593).
 *
 * What one time step computes (lbm_step):
 *   1. streaming: every population moves one link along its lattice vector
 *      c_i (Sec. II, the alternating stream/collide scheme); on a periodic
 *      axis populations leaving one end enter at the other (Sec. III);
 *   2. boundary rules at nodes on a non-periodic plane, using only the
 *      node's own populations (Sec. IV, Sec. V, Appendix):
 *        - face nodes: the prescribed velocity v is imposed exactly; the
 *          density follows from the known populations (eq_uin and its
 *          Appendix forms); the unknown populations are rebuilt by
 *          non-equilibrium bounce-back plus the transverse momentum
 *          corrections N (eq_f5, eq_f9-eq_f17, eq_Nx, eq_Ny, eq_bbshort);
 *          v = 0 is the on-site no-slip wall (Sec. V);
 *        - edge nodes (two planes meet): no-slip bounce-back, the momentum
 *          correction along the edge (eq_Nxzy, eq_edge) and the buried links
 *          (eq_buried);
 *        - corner nodes (three planes meet): no-slip bounce-back and the six
 *          buried links (eq_corner);
 *      Edge and corner nodes are always no-slip, also where they border a
 *      velocity plane: the paper requires the inflow to decay to zero at the
 *      edges (end of Sec. IV; Sec. V);
 *   3. BGK collision f <- f - (f - f^eq(rho, u))/tau with the second-order
 *      equilibrium (eq_bgk, eq_feq, eq_weights).
 * The stored state is the post-collision population set.
 *
 * Conventions
 *   node index   n = x + nx*(y + ny*z)
 *   population   k = i - 1, where i = 1..19 numbers the lattice vectors as the
 *                columns of the matrix M (Sec. II, eq_deffs); k = 18 is the
 *                rest population.  Host population arrays are structure-of-
 *                arrays, f[k*N + n] with N = nx*ny*nz.  Device buffers use
 *                one of two layouts (lbm_set_layout): row-major, element
 *                k*R + 19*R*r + x for the x-row r = y + ny*z, R = nx rounded
 *                up to a multiple of 128 bytes (the start of lbm_create), or
 *                population-major, element k*P + n with
 *                P = lbm_population_pitch(N) (the start of
 *                lbm_create_on_buffers); lbm_buffer_elements gives a
 *                buffer's size.
 *   axes         every axis is periodic until a face of it gets a velocity
 *                or pressure BC; lbm_step then requires both faces of that
 *                axis to be set.
 *                A non-periodic axis needs at least 3 nodes.
 *
 * Storage forms (lbm_storage).  The device buffers hold the deviation of
 * each population from its rest value, d_k = f_k - w_k (w_k: lattice weight,
 * eq_weights); every rule is evaluated in these variables, which keeps the
 * narrow forms accurate.  The populations themselves are f_k = w_k + d_k.
 *   LBM_STORE_F64      d_k in double, arithmetic in double
 *   LBM_STORE_F32      d_k in float,  arithmetic in double
 *   LBM_STORE_F16_DEV  d_k as half-precision scaled deviations
 *                      h_k = RNE(d_k * 2^8), decoded d_k = h_k * 2^-8,
 *                      arithmetic in float.  Limit: near a steady state
 *                      round-to-nearest rounds every node the same way at
 *                      every step, which acts as a constant forcing; on the
 *                      512 x 256 x 256 duct after 20000 steps the velocity
 *                      field is 1.95e-3 (relative L2) from the FP64 form,
 *                      over a 1e-3 bound.  Use LBM_STORE_F16_DEV_SR for
 *                      long runs to steady state.
 *   LBM_STORE_F16_DEV_SR  as LBM_STORE_F16_DEV, but each step rounds
 *                      d_k * 2^8 stochastically to one of its two neighbouring
 *                      half values, unbiased; the random bits are a hash of
 *                      (step index, node, population), so results are
 *                      reproducible and the same alone or in a batch.  The
 *                      16-bit form for steady states: 2.2e-4 relative L2 on
 *                      the same run
 *
 * Errors: every call returns an lbm_status and never aborts.  On failure
 * lbm_last_error() returns a message for the calling thread.  Calls on one
 * handle are not thread-safe.
 *
 * Ownership: lbm_create allocates the two population buffers on the current
 * HIP device; lbm_create_on_buffers adopts caller-owned device buffers that
 * must outlive the handle.  The caller owns every other pointer it passes.
 * All device work of a handle runs on the stream given at creation (NULL: the
 * null stream).  lbm_step only enqueues; the calls that return data
 * synchronize that stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_lattice lbm_lattice;

typedef enum {
  LBM_OK = 0,
  LBM_ERR_ARG = -1,       /* invalid argument (sizes, tau, velocity, pointer) */
  LBM_ERR_OOM = -2,       /* device allocation failed */
  LBM_ERR_HIP = -3,       /* a HIP runtime call failed */
  LBM_ERR_STATE = -4,     /* handle not in a state that allows the call */
  LBM_ERR_NONFINITE = -5  /* a reduction found NaN or Inf in the state */
} lbm_status;

typedef enum { LBM_STORE_F64 = 0, LBM_STORE_F32 = 1, LBM_STORE_F16_DEV = 2, LBM_STORE_F16_DEV_SR = 3 } lbm_storage;

/* Faces: x = 0 (paper: left), x = nx-1 (right), y = 0 (front),
 * y = ny-1 (back), z = 0 (bottom), z = nz-1 (top). */
typedef enum { LBM_X0 = 0, LBM_X1 = 1, LBM_Y0 = 2, LBM_Y1 = 3, LBM_Z0 = 4, LBM_Z1 = 5 } lbm_face;

/* Create a lattice of nx*ny*nz nodes (each >= 1, N < 2^31) with relaxation
 * time tau > 1/2, all axes periodic, every node at f^eq(rho0, u0)
 * (eq_feq).  rho0 > 0; u0 may be NULL (rest).  hip_stream is a hipStream_t
 * or NULL.  On success *out receives the handle.  The library allocates two
 * buffers that hold either layout and starts row-major (lbm_set_layout).
 * Errors: LBM_ERR_ARG (sizes, tau, rho0, storage, out == NULL),
 * LBM_ERR_OOM, LBM_ERR_HIP. */
lbm_status lbm_create(int nx, int ny, int nz, double tau, double rho0, const double u0[3],
                      lbm_storage storage, void *hip_stream, lbm_lattice **out);

/* As lbm_create, on two caller-owned device buffers of buf_bytes bytes each
 * (at least 19*P*element size with P = lbm_population_pitch(N), 256-byte
 * aligned), starting population-major; lbm_set_layout to the row-major
 * layout needs lbm_buffer_elements(..., LBM_LAYOUT_ROW_MAJOR) elements per
 * buffer.  The library never frees them.  Errors as lbm_create; LBM_ERR_ARG
 * if a buffer is NULL, too small or misaligned. */
lbm_status lbm_create_on_buffers(int nx, int ny, int nz, double tau, double rho0, const double u0[3],
                                 lbm_storage storage, void *hip_stream, void *buf_a, void *buf_b,
                                 size_t buf_bytes, lbm_lattice **out);

/* Prescribe the velocity u[3] (lattice units) on a face (Sec. IV, eq_uin;
 * u = 0: on-site no-slip, Sec. V).  The face's axis becomes non-periodic.
 * May be called between steps (moving walls).
 * Errors: LBM_ERR_ARG if L or u is NULL, the face is invalid, the axis has
 * fewer than 3 nodes, |u . n| >= 1 (the density of eq_uin diverges) or
 * |u| >= 1/sqrt(3) (the lattice speed of sound). */
lbm_status lbm_set_velocity_bc(lbm_lattice *L, lbm_face face, const double u[3]);

/* Prescribe the density rho0 on a face (pressure boundary; Sec. IV eq_rhoin,
 * Appendix) with the tangential velocity u_t (only its components parallel
 * to the face are used; NULL: zero).  Each step the normal velocity follows
 * from rho0 and the known populations, and the unknowns from the same closure
 * as a velocity face.  Edges and corners of a pressure face take the no-slip
 * rules with the buried links and rest population set from rho0 (Sec. V,
 * eq_buried_rho), so every edge and corner node of that face has density
 * rho0.  Pressure faces must lie on one axis (edges between two pressure
 * faces are not defined): lbm_step returns LBM_ERR_STATE otherwise.  A face
 * set with lbm_set_velocity_bc afterwards is a velocity face again.
 * Errors: LBM_ERR_ARG if L is NULL, the face is invalid, the axis has fewer
 * than 3 nodes, rho0 is not a positive finite number, or |u_t| >= 1/sqrt(3). */
lbm_status lbm_set_pressure_bc(lbm_lattice *L, lbm_face face, double rho0, const double u_t[3]);

/* Per-node velocities of a velocity face: v[3 * i + d] is component d at face
 * node i, where i = y + ny*z on the x faces, x + nx*z on the y faces and
 * x + nx*y on the z faces (host memory, copied before return; the caller
 * keeps ownership).  The face becomes a velocity face; each entry obeys the
 * limits of lbm_set_velocity_bc.  Used for inflow profiles such as the
 * parabolic Poiseuille velocity of the tilted channel (Sec. VI, eq_pois).
 * v = NULL removes the field (the face keeps its uniform velocity).
 * lbm_set_velocity_bc, lbm_set_pressure_bc and lbm_clear_bc on the face also
 * remove it.  Errors: LBM_ERR_ARG, LBM_ERR_OOM, LBM_ERR_HIP. */
lbm_status lbm_set_velocity_field(lbm_lattice *L, lbm_face face, const double *v);

/* Solid nodes: solid[n] != 0 marks node n (n = x + nx*(y + ny*z), host
 * memory, N bytes, copied before return) as solid.  A fluid node whose
 * streaming source is solid receives its own opposite population of the
 * previous step (mid-grid bounce-back, Sec. III; the wall lies half-way
 * between the two nodes); solid nodes keep their populations unchanged.  A
 * solid node on a bounded face takes no boundary rule.  solid = NULL removes
 * the mask.  Lattices with a mask or a face velocity field are advanced by
 * the extended sweep (one node per thread; the mask is turned on the host
 * into one 4-byte word per node holding the node's own flag and those of its
 * 18 sources, read once per node).  Errors: LBM_ERR_ARG, LBM_ERR_OOM,
 * LBM_ERR_HIP. */
lbm_status lbm_set_solid_mask(lbm_lattice *L, const unsigned char *solid);

/* Complex geometry (Sec. V): cell[n] (host, N bytes, copied before return)
 * is 0 for a fluid node, 1 for a wall node (the on-site no-slip wall lies on
 * it) and 2 for a solid-interior node (no populations; what would stream
 * from it is unknown at the receiving wall node).  Each wall node's rule
 * follows from its unknown populations, classified once here (the paper's
 * per-node normal index): the unknowns of one plane -> the plane rule with
 * v = 0; of two planes on different axes -> the concave-edge rule; of three
 * -> the corner rule; a single unknown diagonal n1 + n2 -> the convex-edge
 * rule (eq_edge2: bounce back, then remove the momentum along the edge from
 * the four populations with c.e != 0 that travel into the bulk); any other
 * set (an edge meeting a plane, thin features) -> bounce back every unknown
 * whose opposite is known and give the buried links and the rest population
 * the others' mass in the ratio of the lattice weights.  All axes are
 * periodic (the geometry carries every wall): lbm_step returns
 * LBM_ERR_STATE if a face BC or a solid mask is also set.  cell = NULL
 * removes the geometry.  Errors: LBM_ERR_ARG (a type other than 0, 1, 2),
 * LBM_ERR_OOM, LBM_ERR_HIP. */
lbm_status lbm_set_geometry(lbm_lattice *L, const unsigned char *cell);

/* Host only (no GPU needed): the classification lbm_set_geometry uses.
 * code[n] (N unsigned, caller-owned): bits 0-17 the unknown populations,
 * bits 18-23 the wall planes as a face mask (bit f: a wall with the inward
 * normal of face f), bits 24-26 the kind: 0 fluid, 1 solid interior,
 * 2 plane / concave edge / corner, 3 convex edge, 4 general.  counts (NULL
 * or 5 entries) receives the number of nodes of each kind.  Errors:
 * LBM_ERR_ARG. */
lbm_status lbm_classify_geometry(int nx, int ny, int nz, const unsigned char *cell, unsigned *code,
                                 long long counts[5]);

/* Rule options (bit mask): LBM_RULE_NO_TRANSVERSE applies the face rule
 * without the transverse corrections N (non-equilibrium bounce-back of every
 * unknown, Sec. IV eq_f9NoNs-eq_f17NoNs): the comparison variant of the
 * paper's tilted-channel test, not a recommended setting.  0 (default): the
 * paper's rule.  Errors: LBM_ERR_ARG (NULL, unknown bits). */
#define LBM_RULE_NO_TRANSVERSE 1u
lbm_status lbm_set_rule_options(lbm_lattice *L, unsigned flags);

/* Body force F (lattice units) acting on every node: the velocity inside
 * f^eq is shifted by tau F / rho (eq_gravity).  F = 0 (the default) is the
 * plain method.  With a force, the stored (post-collision) state carries
 * momentum rho u + F, where u is the post-boundary, pre-collision velocity;
 * lbm_moments reports the stored state.  Errors: LBM_ERR_ARG (NULL, not
 * finite). */
lbm_status lbm_set_body_force(lbm_lattice *L, const double F[3]);

/* Remove the velocity or pressure BC of a face.  When both faces of an axis
 * are cleared the axis is periodic again.  Errors: LBM_ERR_ARG. */
lbm_status lbm_clear_bc(lbm_lattice *L, lbm_face face);

/* Enqueue nsteps >= 0 time steps on the handle's stream; returns without
 * waiting.  Errors: LBM_ERR_ARG (L NULL, nsteps < 0), LBM_ERR_STATE (an axis
 * with a BC on one face only, pressure faces on more than one axis),
 * LBM_ERR_HIP (launch failure). */
lbm_status lbm_step(lbm_lattice *L, int nsteps);

/* Density rho[n] and velocity u[a*N + n] of the stored state (eq_rho,
 * eq_vel), in double.  Either pointer may be NULL.  dst_on_device != 0: the
 * pointers are device pointers; otherwise host pointers.  Synchronizes the
 * handle's stream.  Errors: LBM_ERR_ARG, LBM_ERR_OOM, LBM_ERR_HIP. */
lbm_status lbm_moments(lbm_lattice *L, double *rho, double *u, int dst_on_device);

/* Total mass sum_n rho and momentum sum_n rho u of the stored state, reduced
 * in double in a fixed order (results do not depend on scheduling).
 * Synchronizes.  Errors: LBM_ERR_ARG, LBM_ERR_HIP, LBM_ERR_NONFINITE (NaN or
 * Inf in the totals; the values are still written). */
lbm_status lbm_totals(lbm_lattice *L, double *mass, double momentum[3]);

/* For callers that cannot allocate device memory (work under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * totals of lbm_totals -- mass sum_n rho, then momentum sum_n rho u -- of a
 * population buffer f in device memory (storage form `storage`, layout
 * `layout` of an nx*ny*nz lattice, as lbm_state_buffer gives it), written to
 * out_device[4] (device memory) by kernels enqueued on hip_stream (NULL: the
 * null stream); returns without waiting.  Nothing is allocated: the partial
 * sums of the fixed-order reduction (1024 blocks, the same order as
 * lbm_totals, so the results are the same bits) live in a static device
 * array of 32 KiB that each GPU the library runs on holds until the process
 * ends, and that every call on that GPU shares: calls that overlap on one
 * GPU (on different streams or threads) race and may return wrong totals.
 * The caller owns f and out_device.  Errors: LBM_ERR_ARG (NULL pointer,
 * sizes < 1, 2^31 nodes or more, unknown storage or layout), LBM_ERR_HIP
 * (symbol lookup or launch failure). */
lbm_status lbm_totals_static(const void *f, int nx, int ny, int nz, lbm_storage storage, int layout,
                             void *hip_stream, double *out_device);

/* Copy the stored state to / from a host array f[19*N] of populations f_k
 * in double (same layout as the device state).  get returns w_k + d_k; set
 * stores d_k = f_k - w_k evaluated in double, rounded to nearest even for
 * LBM_STORE_F32 and both FP16 forms (the stochastic rounding of
 * LBM_STORE_F16_DEV_SR applies to steps only).  Synchronizes.
 * Errors: LBM_ERR_ARG, LBM_ERR_OOM, LBM_ERR_HIP. */
lbm_status lbm_get_populations(lbm_lattice *L, double *f);
lbm_status lbm_set_populations(lbm_lattice *L, const double *f);

/* Device pointer of the buffer that holds the stored state, in the storage
 * form's encoding of d_k = f_k - w_k and the lattice's layout (it alternates
 * between the two buffers every step).  Errors: LBM_ERR_ARG. */
lbm_status lbm_state_buffer(const lbm_lattice *L, void **dev_ptr);

/* Layout of the populations in the device buffers (the host-side arrays of
 * lbm_get_populations / lbm_set_populations and every result are the same
 * in both):
 *   LBM_LAYOUT_POPULATION_MAJOR  element k*P + n, P = lbm_population_pitch(N):
 *                                19 arrays of N nodes (the start of a
 *                                lattice on caller-owned buffers);
 *   LBM_LAYOUT_ROW_MAJOR         element k*R + 19*R*r + x, r = y + ny*z, with
 *                                the row pitch R = nx rounded up to a
 *                                multiple of 128 bytes (32 FP32, 16 FP64 or
 *                                64 FP16 elements): the 19 populations of
 *                                each x-row stored next to each other, every
 *                                row on a cache-line boundary.  A sweep then
 *                                streams through a few neighbouring regions
 *                                of HBM instead of 38 regions P elements
 *                                apart; on the MI355X this moves more bytes
 *                                per second (the start of lbm_create).
 * Every layout gives bitwise the same results.  lbm_set_layout moves the
 * state into the other buffer in the new layout (enqueued on the stream, so
 * lbm_state_buffer changes).  The library's buffers hold either layout;
 * caller-owned buffers smaller than the row-major layout needs (padded rows,
 * lbm_buffer_elements) give LBM_ERR_STATE and the lattice keeps its layout.
 * Errors: LBM_ERR_ARG (unknown layout, NULL), LBM_ERR_STATE, LBM_ERR_HIP. */
enum { LBM_LAYOUT_POPULATION_MAJOR = 0, LBM_LAYOUT_ROW_MAJOR = 1 };
lbm_status lbm_set_layout(lbm_lattice *L, int layout);
lbm_status lbm_get_layout(const lbm_lattice *L, int *layout);

/* Elements one population buffer needs for an nx*ny*nz lattice in a layout:
 * 19*P population-major, 19*R*ny*nz row-major (R as above); multiply by
 * lbm_element_bytes for bytes.  0 for invalid sizes, storage or layout. */
size_t lbm_buffer_elements(int nx, int ny, int nz, lbm_storage storage, int layout);

/* Bytes of one population element for a storage form (8, 4 or 2); 0 if the
 * storage value is invalid. */
size_t lbm_element_bytes(lbm_storage storage);

/* Population stride P of the device buffers, in elements, for a lattice of
 * `nodes` nodes: nodes rounded up to a multiple of 64, so that every
 * population starts on a cache-line boundary.  In the population-major
 * layout population k of node n is element k*P + n of a buffer; a buffer
 * holds 19*P elements in either layout. */
size_t lbm_population_pitch(size_t nodes);

/* Placement of the sweep's blocks on the 8 XCDs (each with its own L2) of
 * the MI355X, which deals workgroups to the XCDs in turn:
 *   LBM_XCD_NONE   dispatch order;
 *   LBM_XCD_SLABS  each XCD sweeps one contiguous eighth of the lattice;
 *   LBM_XCD_ROWS   the blocks of one x-row run on one XCD, rows dealt to the
 *                  XCDs in turn (the same as NONE with one block per row). */
enum { LBM_XCD_NONE = 0, LBM_XCD_SLABS = 1, LBM_XCD_ROWS = 2 };

/* Launch shape of the sweep kernel: block_x threads along x (64, 128, 256 or
 * 512), nodes_per_thread along x (1, 2 or 4), xcd_remap one of LBM_XCD_*.
 * Any shape gives the same results.  Errors: LBM_ERR_ARG for an unsupported
 * shape. */
lbm_status lbm_set_launch(lbm_lattice *L, int block_x, int nodes_per_thread, int xcd_remap);
lbm_status lbm_get_launch(const lbm_lattice *L, int *block_x, int *nodes_per_thread, int *xcd_remap);

/* Steps per pass over HBM.  steps_per_pass = 2 (temporal blocking): lbm_step
 * advances pairs of steps with one kernel in which a workgroup streams a
 * tile of 64 x BY nodes (by default BY = 13 for FP32 and FP16, 5 for FP64) through
 * ranges of z_planes planes, computes the first step on the tile plus a
 * one-node halo into LDS and the second from LDS into HBM.  Per pair of
 * steps every node's populations are read about once (the halo rows are
 * shared with neighbouring tiles through L2) and written once, against
 * twice each with two single sweeps; the first step's arithmetic on the
 * halo nodes is done twice (about 1.2 times the updates).  Every node's
 * arithmetic, rounding and random words are the single sweep's, so the state
 * after a pair equals the state after two single sweeps bit for bit.  The
 * pass applies to lattices in the row-major layout without a solid mask,
 * face velocity field or geometry; for others, and for the last step of an
 * odd count, lbm_step runs the single sweep.  z_planes >= 1 (0: 64) sets the
 * planes per workgroup; the first step on the two planes beyond a range is
 * done by both neighbouring ranges.  tile_rows picks the tile height: 0,
 * the form's default; 5, five-row tiles (two workgroups per compute unit);
 * 12, twelve-row tiles (15 waves, three of step 2's 12 on each SIMD;
 * measured faster than 13 rows on 512 x 256 x 256 FP32, slower on
 * 1024 x 512 x 512); FP64 tiles have five rows either way.  Every variant
 * gives the same bits.  steps_per_pass = 1: one single sweep per step (the
 * default).  Errors: LBM_ERR_ARG (NULL, steps_per_pass not 1 or 2,
 * z_planes < 0, tile_rows not 0, 5 or 12). */
lbm_status lbm_set_steps_per_pass(lbm_lattice *L, int steps_per_pass, int z_planes, int tile_rows);
lbm_status lbm_get_steps_per_pass(const lbm_lattice *L, int *steps_per_pass, int *z_planes, int *tile_rows);

/* Number of steps the lattice has taken since creation (lbm_step,
 * lbm_autotune; lbm_set_populations does not reset it).  It also keys the
 * random numbers of the stochastic-rounding form.  Errors: LBM_ERR_ARG. */
lbm_status lbm_get_step(const lbm_lattice *L, unsigned long long *steps);

/* Pick the fastest launch shape for this lattice by timing real steps: for
 * each candidate of the single sweep (blocks of 64..512 threads no wider
 * than the row rounded up to a power of two, 1, 2 or 4 nodes per thread; one
 * node per thread with a solid mask, face field or geometry; each XCD
 * placement) one untimed and trial_steps >= 1 timed steps, and, in the
 * row-major layout without those options, for each two-step pass
 * (lbm_set_steps_per_pass: z ranges of 16, 32 or 64 planes, tiles of the
 * form's default rows, 5 or 12 rows (FP64: its 5 only), slab or
 * dispatch-order placement) one
 * untimed and trial_steps timed pairs, on the lattice's stream (HIP events,
 * compared per step).  The steps are part of the run (results do not depend
 * on the choice).  Sets the winner -- launch shape, steps per pass, z range
 * and tile rows -- and returns the launch shape through the non-NULL
 * pointers (lbm_get_steps_per_pass gives the rest).  Synchronizes.  Errors:
 * LBM_ERR_ARG, LBM_ERR_STATE (as lbm_step), LBM_ERR_HIP; on error the
 * previous settings are restored. */
lbm_status lbm_autotune(lbm_lattice *L, int trial_steps, int *block_x, int *nodes_per_thread, int *xcd_remap);

/* Pick the physical placement of the two population buffers by timing real
 * steps.  The sweep's speed depends on where its source and destination
 * buffers lie in device memory, as a fixed property of each pair of
 * allocations (measured on the 1024 x 512 x 512 FP32 duct: 5.3 to 6.0 TB/s
 * for different pairs, each steady to 0.2%).  The call keeps the lattice's
 * two buffers, allocates up to max_buffers - 2 more (2 <= max_buffers <= 8;
 * fewer when the device would keep less than 1/8 of its memory, and at
 * least 1 GiB, free), and times every pair: with the state in the pair's
 * first buffer, two untimed and 2 * trial_steps timed steps (trial_steps >=
 * 1; HIP events on the lattice's stream).  The lattice keeps the fastest
 * pair, with the state copied into it, and every other buffer is freed.  The
 * steps are part of the run: the lattice advances by 2 + 2 * trial_steps
 * steps per pair (at most 28 pairs), and results do not depend on placement.
 * Out (each may be NULL): buffers_tried, and the milliseconds per step of
 * the lattice's own pair (ms_before) and of the chosen one (ms_after).
 * Synchronizes; lbm_state_buffer changes.  Errors: LBM_ERR_ARG,
 * LBM_ERR_STATE (as lbm_step, or a lattice on caller-owned buffers),
 * LBM_ERR_HIP; on error the lattice keeps a valid pair holding its state. */
lbm_status lbm_tune_placement(lbm_lattice *L, int max_buffers, int trial_steps, int *buffers_tried,
                              double *ms_before, double *ms_after);

/* Bandwidth probes on the handle's buffers (measurement only; they overwrite
 * the non-current buffer and leave the stored state intact):
 *   kind 0: plain contiguous copy of the 19*N elements;
 *   kind 1: the sweep's streaming access pattern (19 pulled loads, 19
 *           stores per node) with no boundary rule and no arithmetic.
 * Enqueues nrep launches.  Errors: LBM_ERR_ARG, LBM_ERR_HIP. */
lbm_status lbm_probe(lbm_lattice *L, int kind, int nrep);

/* Lattice size as given at creation.  Errors: LBM_ERR_ARG (NULL). */
lbm_status lbm_get_size(const lbm_lattice *L, int *nx, int *ny, int *nz);

/* Release the handle and the buffers it allocated.  NULL is a no-op. */
void lbm_destroy(lbm_lattice *L);

/* Message of the last failed call on this thread ("" if none). */
const char *lbm_last_error(void);

/* ------------------------------------------------------------------------
 * Batch runtime: many independent lattices resident on one GPU, advanced
 * together by a persistent multi-lattice sweep (the same per-node update as
 * lbm_step, so a lattice's result does not depend on what else runs).
 * Lattices ("jobs") are admitted from a queue when a slot and memory in the
 * HBM budget are free; steps run in chunks captured as HIP graphs; after each
 * chunk the convergence measure
 *     delta = max_nodes,components |u(t) - u(t - chunk)| / u_ref
 * decides retirement (delta < tol, or steps >= max_steps).  Retired jobs'
 * moments are copied to host memory (page-locked when the runtime grants it,
 * held until lbm_batch_result or lbm_batch_destroy) and their device memory
 * is returned to the pool at once.  The paper runs a fixed number of steps (Sec. VI); the
 * convergence measure and its use for stopping are this library's.
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch;

typedef struct {
  int nx, ny, nz;            /* lattice size; N = nx*ny*nz < 2^31 */
  double tau;                /* > 1/2 */
  double rho0;               /* initial density (> 0); initial velocity 0 */
  lbm_storage storage;
  unsigned bc_mask;          /* bit f: face f is bounded; both faces of an axis or none */
  double bc_velocity[6][3];  /* as lbm_set_velocity_bc, same limits (pressure faces: see pressure_mask) */
  double force[3];           /* body force, as lbm_set_body_force (0: none) */
  double u_ref;              /* velocity scale of delta (> 0), e.g. |inflow velocity| */
  double tol;                /* stop when delta < tol (tol <= 0: never) */
  int max_steps;             /* stop once steps >= max_steps */
  unsigned pressure_mask;    /* bit f: face f (also in bc_mask) is a pressure face with density
                                bc_rho[f] and tangential velocity bc_velocity[f], as
                                lbm_set_pressure_bc; pressure faces on one axis only */
  double bc_rho[6];
} lbm_job;

typedef enum { LBM_JOB_QUEUED = 0, LBM_JOB_RUNNING = 1, LBM_JOB_DONE = 2 } lbm_job_state;

typedef struct {
  int state;        /* lbm_job_state */
  int steps;        /* steps taken (a multiple of 2; chunks and autotune trials) */
  double delta;     /* convergence measure at the last check (inf before the first) */
  int converged;    /* 1 if it stopped on delta < tol */
  long long nodes;  /* nx*ny*nz: the length of the rho array of lbm_batch_result */
} lbm_job_status;

/* Device bytes a job occupies while resident: two population buffers and a
 * float velocity snapshot, each rounded up to 256 bytes -- the larger of the
 * two layouts a batch may give it.  Errors: LBM_ERR_ARG. */
lbm_status lbm_job_bytes(const lbm_job *job, size_t *bytes);

/* Create a batch with a device pool of hbm_budget_bytes (one allocation, made
 * here), chunks of chunk_steps (even, >= 2) steps and at most max_jobs
 * resident jobs.  hip_stream NULL: the batch creates its own stream (graph
 * capture needs a stream other than the null stream).
 * Errors: LBM_ERR_ARG, LBM_ERR_OOM (pool), LBM_ERR_HIP. */
lbm_status lbm_batch_create(size_t hbm_budget_bytes, int chunk_steps, int max_jobs, void *hip_stream,
                            lbm_batch **out);

/* Queue a job; *job_id receives its id.  Errors: LBM_ERR_ARG (invalid job),
 * LBM_ERR_OOM (the job alone exceeds the budget). */
lbm_status lbm_batch_submit(lbm_batch *B, const lbm_job *job, int *job_id);

/* Admit queued jobs that fit; on every idle lane (lbm_batch_set_lanes) start
 * a chunk of chunk_steps steps of the resident jobs the policy gives it (jobs
 * in flight on another lane are not eligible); block until at least one
 * lane's chunk has completed; for each completed chunk evaluate delta and
 * retire the finished jobs (their moments are on the host when the call
 * returns).  Chunks of other lanes may still be running on the device when
 * the call returns: the next call starts new chunks beside them.  With one
 * lane (the default) a call runs exactly one chunk.  n_active / n_queued (may
 * be NULL) receive the resident and queued counts at return.
 * Errors: LBM_ERR_ARG, LBM_ERR_HIP, LBM_ERR_OOM (host memory for results,
 * tile tables). */
lbm_status lbm_batch_run_chunk(lbm_batch *B, int *n_active, int *n_queued);

/* Status of a job.  Errors: LBM_ERR_ARG (unknown id). */
lbm_status lbm_batch_poll(lbm_batch *B, int job_id, lbm_job_status *st);

/* Moments of a finished job, rho[N] and u[3*N] (host arrays; either may be
 * NULL), then forget the job and free its host copy.  Errors: LBM_ERR_ARG
 * (unknown id), LBM_ERR_STATE (not finished). */
lbm_status lbm_batch_result(lbm_batch *B, int job_id, double *rho, double *u);

/* Launch shape of the multi-lattice sweep: block_x threads (128 or 256),
 * tile_nodes nodes per tile (>= 256), grid_blocks 0 for one workgroup per
 * tile (the default, with tiles of 256 nodes), or that many persistent
 * workgroups walking the tile list.  Any shape gives the same results. */
lbm_status lbm_batch_set_shape(lbm_batch *B, int block_x, int tile_nodes, int grid_blocks);

/* Which resident jobs a chunk steps (with one lane; lbm_batch_set_lanes
 * gives the rule for several):
 *   LBM_BATCH_LOCKSTEP        all of them (the default): every resident job
 *                             advances chunk_steps steps per chunk;
 *   LBM_BATCH_SHORTEST_FIRST  the job with the least remaining work (nodes
 *                             times the steps left to max_steps) and, if it
 *                             has fewer than fill_nodes nodes, the next ones
 *                             below fill_nodes until at least fill_nodes
 *                             nodes are chosen; every job left out for 50
 *                             scheduling rounds in a row is added.  Small
 *                             jobs then step at their own pace instead of a
 *                             large co-resident job's; the others wait,
 *                             resident.
 * A job's results do not depend on the policy (only when its steps run).
 *   LBM_BATCH_LARGE_IN_ORDER  meant for several lanes: jobs of at least
 *                             fill_nodes nodes are large and run one at a
 *                             time in submission order (a later large job
 *                             never slows an earlier one down); small jobs
 *                             run one per remaining lane, shortest remaining
 *                             work first, beside the large one.
 * Set the policy before submitting: with LBM_BATCH_SHORTEST_FIRST, jobs of
 * at least fill_nodes nodes submitted afterwards are stored row-major with
 * padded rows, with LBM_BATCH_LARGE_IN_ORDER every job (and with two steps
 * per pass, lbm_batch_set_steps_per_pass(B, 2, ...), every job whatever the
 * policy); a chunk that steps a single row-major job runs the single-lattice
 * sweep (or two-step pass) on it.
 * lbm_batch_autotune steps every resident job whatever the policy.
 * Errors: LBM_ERR_ARG (NULL, unknown policy). */
enum { LBM_BATCH_LOCKSTEP = 0, LBM_BATCH_SHORTEST_FIRST = 1, LBM_BATCH_LARGE_IN_ORDER = 2 };
lbm_status lbm_batch_set_policy(lbm_batch *B, int policy, size_t fill_nodes);
lbm_status lbm_batch_get_shape(const lbm_batch *B, int *block_x, int *tile_nodes, int *grid_blocks);

/* Steps per pass over HBM for the batch's chunks (Sec. II's update, two steps
 * at a time as lbm_set_steps_per_pass does for one lattice):
 *   1 (the default)  one step per launch;
 *   2                every chunk by passes of two steps: one launch per
 *                    storage form over the 64 x 13 (FP64: 64 x 5) tiles and
 *                    z ranges of z_planes planes (0: 32) of all its jobs, or
 *                    the single-lattice two-step kernel for a chunk of one
 *                    job; every job is then stored row-major with padded
 *                    rows.
 * Single steps close a chunk whose step count needs them (chunk_steps 2 mod
 * 4: two).  Results are the same bits in either mode.  Two steps per pass
 * pay for batches of large FP32 and FP64 lattices (eight 256^3 cubes: FP32
 * 37.1 -> 40.4 GLUPS, FP64 17.8 -> 23.8), not for small or narrow ones: on
 * 64 uneven ducts of 32-256 x 16-128 x 16-128 nodes they ran 1.3x slower
 * than one step per launch (a quarter of the tiles' lanes fall outside such
 * lattices), and a chunk of one cube of up to 320^3 nodes has too few tiles
 * to fill the chip (FP32 no faster, FP16 1.6x slower).
 * Errors: LBM_ERR_ARG (steps not 1 or 2, z_planes outside [0, 4096]),
 * LBM_ERR_STATE (a chunk in flight; 2 while a population-major job is queued
 * or resident -- set the mode before submitting). */
lbm_status lbm_batch_set_steps_per_pass(lbm_batch *B, int steps_per_pass, int z_planes);
lbm_status lbm_batch_get_steps_per_pass(const lbm_batch *B, int *steps_per_pass, int *z_planes);

/* Admit what fits, then time trial_steps (even) steps of the resident jobs
 * for each candidate shape (one workgroup per tile: 256 threads and tiles of
 * 256, 512 or 1024 nodes, 128 threads and 256 nodes; persistent: 256 threads,
 * 1024-node tiles, 16 workgroups per compute unit, and 128 threads, 1024
 * nodes, 8 per compute unit) and keep the fastest; with two steps per pass,
 * z ranges of 16, 32 or 64 planes in two box orders (each XCD a contiguous
 * share of the box list, or dispatch order), timed over trial_steps rounded
 * up to a multiple of 4 (at least 4) after 4 warm-up steps.  The trial steps are
 * real steps of every resident job (their step counts advance).  Results are
 * cached per process by storage mix and node-count class; a cached class is
 * not re-timed.  Outputs may be NULL.  Errors: LBM_ERR_ARG, LBM_ERR_STATE (no
 * resident job), LBM_ERR_HIP. */
lbm_status lbm_batch_autotune(lbm_batch *B, int trial_steps, int *block_x, int *tile_nodes, int *grid_blocks);

/* Bytes of the pool in use and in total.  Errors: LBM_ERR_ARG. */
lbm_status lbm_batch_memory(const lbm_batch *B, size_t *used, size_t *capacity);

/* Lanes: independent streams of one batch that run chunks at the same time
 * on the device, all sharing the batch's HBM pool.  A lane's chunk steps its
 * group of jobs (one launch sequence: the multi-lattice sweep, or the
 * single-lattice sweep for one row-major job); groups are formed from the
 * jobs not in flight whenever a lane is idle:
 *   LBM_BATCH_LOCKSTEP        every such job, spread over the idle lanes
 *                             (largest first, each to the lane with the
 *                             fewest nodes so far);
 *   LBM_BATCH_SHORTEST_FIRST  in order of remaining work, one job per idle
 *                             lane; a job below fill_nodes nodes takes
 *                             further jobs below fill_nodes into its lane's
 *                             launch until it holds fill_nodes nodes;
 *   LBM_BATCH_LARGE_IN_ORDER  the earliest submitted large job (at least
 *                             fill_nodes nodes) on one lane while no large
 *                             job is in flight, small jobs one per other
 *                             idle lane, shortest remaining work first.
 * So a request that arrives while others are on the GPU starts at once on
 * an idle lane, and its steps overlap theirs on the device, instead of
 * waiting for them.  1 <= lanes <= 8 (1: the default, one chunk at a time;
 * lane 0 runs on the batch's stream, the others on streams the batch
 * creates, all at the default priority).  Each lane holds a small
 * descriptor table and page-locked staging.  Results do not depend on the
 * lanes.  Errors: LBM_ERR_ARG (NULL, out of range), LBM_ERR_STATE (a chunk
 * in flight), LBM_ERR_OOM, LBM_ERR_HIP. */
lbm_status lbm_batch_set_lanes(lbm_batch *B, int lanes);

/* What the batch has run so far (counts since creation). */
typedef struct {
  int lanes;                   /* lanes configured now */
  long long chunks;            /* chunks started (on any lane) */
  long long job_chunks;        /* sum over chunks of the jobs each stepped */
  long long multi_job_chunks;  /* chunks whose launches stepped two or more jobs */
  int max_jobs_in_chunk;       /* most jobs one chunk stepped */
  long long overlapped_chunks; /* chunks started while another lane's chunk was still running on the device */
  int max_lanes_running;       /* most lanes with a chunk running on the device at one chunk start */
} lbm_batch_stats;

/* Copy the counts into *stats.  Errors: LBM_ERR_ARG (NULL). */
lbm_status lbm_batch_get_stats(const lbm_batch *B, lbm_batch_stats *stats);

/* Release the batch, its pool and every job.  NULL is a no-op. */
void lbm_batch_destroy(lbm_batch *B);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
