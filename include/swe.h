/*
 * swe.h -- C ABI of the MI355X (gfx950) shallow-water library.
 *
 * The library advances the depth-averaged shallow-water equations in
 * surface-elevation form (paper: section "Mathematical formulation",
 * subsection Hydrodynamics, eq. Hyd_gov_equations) with the explicit,
 * first-order, cell-centred finite-volume update of eq.
 * hydrodynamicupdateformula on a conforming triangulation (section "Domain
 * discretization").  One step does, for every cell: hydrostatic
 * reconstruction of modified states with wet/dry handling, an HLLC edge flux
 * (section "Numerical solution", Hydrodynamics paragraph on HLLC), the
 * conservative update, the Manning friction split (eq. friction_closure and
 * the Manning row of Table friction_closure), and the next global CFL step
 * (eq. CFL_condition).  All of it runs in hand-written HIP kernels; the host
 * code only prepares the mesh, moves memory and launches.
 *
 * Conventions
 *  - Every pointer argument named *_host / plain arrays is HOST memory and is
 *    copied; the caller keeps ownership.  Device memory is obtained through
 *    the swe_device callbacks (or hipMalloc when none are given) and is owned
 *    by the handle until its *_destroy.
 *  - Cell arrays are in the caller's ORIGINAL cell order on input and output;
 *    the library renumbers cells internally (Hilbert order of centroids).
 *  - Status codes: SWE_OK (0) or a negative SWE_E* value; swe_last_error()
 *    returns a thread-local message for the last failure on this thread.
 *  - A handle may be used by one host thread at a time.  A mesh must outlive
 *    the states created on it; a state must outlive the batches holding it.
 */
#ifndef SWE_H
#define SWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct swe_mesh swe_mesh;
typedef struct swe_state swe_state;
typedef struct swe_batch swe_batch;
typedef int32_t swe_status;

enum {
    SWE_OK = 0,
    SWE_EINVAL = -1,     /* invalid argument or mesh */
    SWE_ENOMEM = -2,     /* allocation failed */
    SWE_EDEVICE = -3,    /* a HIP call failed */
    SWE_ENONFINITE = -4, /* the state became non-finite */
    SWE_ENEGDEPTH = -5,  /* negative depth under SWE_NEG_ERROR */
    SWE_EBUDGET = -6,    /* batch footprint budget exceeded */
    SWE_ENODT = -7,      /* no finite positive time step (dry domain, no cap) */
    SWE_ESINK = -8       /* an exact sink asked for more water than a cell held */
};

/* Device memory and stream bridge.  alloc(bytes, ctx) returns device memory
 * (NULL on failure) aligned to at least 256 bytes; free(ptr, ctx) releases it.
 * hip_stream is a hipStream_t on which every kernel and copy of the handle is
 * issued (NULL = the default stream).  A NULL swe_device, or NULL alloc/free,
 * means hipMalloc/hipFree. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
    void *hip_stream;
} swe_device;

/* Boundary kinds (section "Boundary conditions", Hydrodynamic BCs, and the
 * standard inflows and outflows of the supplementary feature table).  Series
 * are linear in time (or in the surface elevation for an h-Q table), constant
 * past their ends, and taken at the step's start time.
 *  - WALL: reflective, impermeable (the default on every external boundary:
 *    edges whose tag has no entry, and untagged edges, are walls).
 *  - INFLOW_UNIFORM (Q(t), slope S): q = Q / (boundary length) enters at
 *    the Manning normal depth (n q / sqrt(S))^(3/5) of the edge's cell.
 *  - OUTFLOW_ZEROGRAD: the ghost repeats the interior state.
 *  - ZHYDROGRAPH (surface elevation series): still water at that surface
 *    over the cell's bed; water flows in or out as the levels differ.
 *  - INFLOW_FROUDE (Q(t), slope = Froude number Fr > 0): q enters at the
 *    depth (q / (Fr sqrt(g)))^(2/3) where the flow has that Froude number.
 *  - OUTFLOW_UNIFORM (slope S): the ghost has the normal depth of the cell's
 *    outflowing unit discharge, with the cell's velocity.
 *  - OUTFLOW_WEIR (slope = crest elevation z_w, par = Poleni factor mu > 0):
 *    the edge carries q = (2/3) mu sqrt(2g) d^(3/2) out, d = H - max(z_w, z)
 *    of its cell, with the cell's state: flux (q, q^2/h + g h^2/2, q u_t).
 *  - OUTFLOW_HQ (t = surface elevations H, Q = discharges >= 0): q =
 *    Q(H) / (boundary length) leaves like over a weir.
 *  - DYNAMIC_WALL (slope = collapse time, par = collapse depth >= 0, 0 for
 *    none): a wall before its collapse time and, with a collapse depth,
 *    until the end of the first step that starts with its cell at that
 *    depth or deeper (h = H - z); zero gradient from then on.  A state
 *    created from another one's read-out starts with its walls standing.
 * On tagged interior edges (internal conditions, section "Hydrodynamic
 * BCs"): WALL makes each side a wall of its own state; DYNAMIC_WALL does so
 * until it collapses (by time, or by the depth of a cell on either side),
 * after which the edge is an ordinary one; OUTFLOW_HQ
 * is a rating curve: q = Q(H) / (the curve's length) at the surface H of the
 * cell left of each segment (walking from its first node to its second)
 * crosses to the cell on the right, leaving with the left cell's state,
 * while the right cell's momentum sees a wall (one-way flow; species cross
 * with the left cell's concentrations, sediment and diffusion do not cross;
 * not with the draining-time limiter).
 * Uniform inflow and outflow need the Manning or Strickler closure and a
 * positive friction parameter in their cells.  Inflows carry their inflow
 * concentrations of passive species; outflows the interior's. */
enum {
    SWE_BC_WALL = 0,
    SWE_BC_INFLOW_UNIFORM = 1,
    SWE_BC_OUTFLOW_ZEROGRAD = 2,
    SWE_BC_ZHYDROGRAPH = 3,
    SWE_BC_INFLOW_FROUDE = 4,
    SWE_BC_OUTFLOW_UNIFORM = 5,
    SWE_BC_OUTFLOW_WEIR = 6,
    SWE_BC_OUTFLOW_HQ = 7,
    SWE_BC_DYNAMIC_WALL = 8
};

typedef struct {
    int32_t tag;      /* boundary tag given to swe_mesh_create */
    int32_t kind;     /* SWE_BC_* */
    double slope;     /* energy slope (uniform), Froude number, crest elevation (weir) or collapse time [s] */
    const double *t;  /* series times [s] or the surface elevations of an h-Q table, strictly increasing (host) */
    const double *Q;  /* discharge [m^3/s], or surface elevation [m] for a zhydrograph (host) */
    int32_t n_pts;    /* number of series points (>= 1 where a series is needed) */
    double par;       /* Poleni factor of a weir, collapse depth [m] of a dynamic wall */
} swe_bc;

/* Precision (section "Parallelization Strategy and Computational Backends":
 * double by default, single optional).  FP32 states store the discharges
 * and the bed in FP32 and the water surface as an FP32 high part plus a
 * 16-bit low part (about 40 significant bits, so that small increments are
 * not rounded away); depth tests, time, the time step and the tallies stay
 * in FP64. */
enum { SWE_FP64 = 0, SWE_FP32 = 1 };
/* Friction closures (eq. friction_closure, Table friction_closure): the
 * per-cell parameter given to swe_state_init is Manning n [s m^-1/3],
 * Strickler k_str [m^1/3 s^-1], Chezy K_s [m] or Bezzola y_R [m]; 0 means no
 * friction in that cell. */
enum { SWE_FRICTION_MANNING = 0, SWE_FRICTION_STRICKLER = 1, SWE_FRICTION_CHEZY = 2, SWE_FRICTION_BEZZOLA = 3 };
enum { SWE_NEG_CLIP = 0, SWE_NEG_ERROR = 1 }; /* negative-depth policy */
enum { SWE_LIMIT_NONE = 0, SWE_LIMIT_DRAIN = 1 }; /* positivity limiter */

/* Parameters (supplementary feature table, hydrodynamics parameters: CFL,
 * minimum water depth, upper limit of the time step; eq. CFL_condition for
 * the CFL range (0, 1] and its default 0.9). */
typedef struct {
    double g;               /* gravity [m/s^2], default 9.81 */
    double cfl;             /* CFL number in (0, 1], default 0.9 */
    double h_min;           /* minimum water depth [m] > 0, default 1e-4 */
    double dt_max;          /* upper limit of the time step [s] > 0, default +inf */
    int32_t precision;      /* SWE_FP64 (default) or SWE_FP32 */
    int32_t neg_depth_policy; /* SWE_NEG_CLIP (default) or SWE_NEG_ERROR */
    int32_t block_size;     /* cells per tile = threads per block: 128, 256 or 512; 0 = default (256).
                               One thread per cell; a tile's edges (about 1.7 per cell) are spread
                               over its threads, so this also sets the edges per thread */
    int32_t steps_per_graph;  /* steps captured per hipGraph in swe_run_until; 0 = default (32) */
    int32_t renumber;       /* 1 = Hilbert order of cell centroids (default), 0 = input order */
    int32_t friction;       /* SWE_FRICTION_* closure (default Manning) */
    int32_t limiter;        /* SWE_LIMIT_NONE (default: negative depths are clipped and tallied) or
                               SWE_LIMIT_DRAIN: every flux leaving a cell acts only for that cell's
                               draining time h |Omega| / (its outgoing mass flux), so depths stay
                               >= 0 without the clip (up to rounding); costs a second edge pass per
                               step; not with passive species, morphodynamics or batches */
} swe_params;

/* Fills *p with the defaults listed above. */
void swe_params_default(swe_params *p);

/* Builds a mesh from node coordinates and elevations (node_xyz: n_nodes x 3
 * doubles x, y, z, host) and triangles (tri: n_tri x 3 node ids, host, any
 * winding -- fixed to counter-clockwise).  bnd_seg (n_seg x 2 node ids) with
 * bnd_tag (n_seg ints) tags edges: boundary edges, and interior edges that
 * carry an internal condition (at most 31 such tags; the segment's node
 * order gives its direction, see the boundary kinds); every segment must be
 * an edge of the mesh.  The cell bed elevation is the mean of its three node
 * elevations.  Rejects non-finite coordinates, degenerate triangles, edges
 * shared by three or more triangles and inconsistently oriented neighbours
 * (SWE_EINVAL).  params may be NULL (defaults); only params->renumber is read.
 * dev may be NULL.  On success *out owns the mesh. */
swe_status swe_mesh_create(const double *node_xyz, int64_t n_nodes, const int32_t *tri, int64_t n_tri,
                           const int32_t *bnd_seg, const int32_t *bnd_tag, int64_t n_seg,
                           const swe_params *params, const swe_device *dev, swe_mesh **out);
void swe_mesh_destroy(swe_mesh *m);
/* counts: cells, edges, boundary edges (any pointer may be NULL) */
void swe_mesh_info(const swe_mesh *m, int64_t *n_cells, int64_t *n_edges, int64_t *n_boundary_edges);
/* Device bytes one solve of this precision needs: the state plus the mesh
 * data its kernels read (tile edge lists, areas). */
int64_t swe_state_footprint(const swe_mesh *m, int32_t precision);
/* Host-side consistency check of the mesh's tile edge lists for a block
 * size (128, 256 or 512): every cell edge covered exactly once, indices,
 * orientation flags and normals consistent.  SWE_OK or SWE_EINVAL with the
 * first problem in swe_last_error().  Diagnostic; no device work. */
swe_status swe_mesh_check(const swe_mesh *m, int32_t tile);

/* Creates a device-resident state (section "Initial and boundary
 * conditions": region-defined initial values or dry).  Exactly one of
 * H0 (surface elevation; values below the cell bed mean a dry cell) and h0
 * (depth >= 0) may be non-NULL; both NULL means dry.  qx0, qy0 (discharge per
 * unit width) may be NULL (zero); manning (the friction parameter >= 0 per
 * cell of the closure params->friction selects: Manning n by default) may be
 * NULL (frictionless).  All arrays are host arrays of n_cells doubles in
 * original cell order.  bcs[n_bc] maps tags to kinds; inflow edges need the
 * Manning or Strickler closure (their normal depth has a closed form) and a
 * positive parameter in their cell.  t0 is the start time (restart = re-init
 * from a read state).  params may be NULL.  Computes the first time step on
 * the device. */
swe_status swe_state_init(const swe_mesh *m, const swe_params *params, const double *H0,
                          const double *h0, const double *qx0, const double *qy0,
                          const double *manning, const swe_bc *bcs, int32_t n_bc, double t0,
                          swe_state **out);
void swe_state_destroy(swe_state *s);

/* One step of eq. hydrodynamicupdateformula with dt = min(dt_max,
 * CFL * min rho/lambda) (no end-time cap).  Blocks until done; *dt_taken may
 * be NULL.  Returns SWE_ENODT when no finite step exists, SWE_ENONFINITE /
 * SWE_ENEGDEPTH when the state broke.  A step that raises such an error is
 * not completed consistently: the tiles that ran before the flag was raised
 * wrote the new level, the later ones skip theirs, so the state read
 * afterwards mixes two time levels and only tells where the failure began;
 * a run continues from a state saved before the failing step. */
swe_status swe_step(swe_state *s, double *dt_taken);

/* Steps until t = t_end (the last step is shortened to land on t_end), with
 * steps_per_graph steps per hipGraph launch and one 64-byte status read per
 * launch.  *n_steps (may be NULL) receives the number of steps taken. */
swe_status swe_run_until(swe_state *s, double t_end, int64_t *n_steps);

/* Issues k steps capped at t_end on the state's stream WITHOUT waiting
 * (graph launches); swe_sync waits and reports errors.  For timing. */
swe_status swe_launch_steps(swe_state *s, double t_end, int64_t k);
swe_status swe_sync(swe_state *s);
/* Captures and instantiates the hipGraphs that swe_run_until and
 * swe_launch_steps replay -- steps_per_graph step launches each, one graph
 * per starting launch phase (the step count mod 3) -- WITHOUT launching
 * anything, so that a timed region that follows replays graphs only.
 * steps_per_graph in 1..4096 also replaces the state's setting; 0 keeps it.
 * SWE_EINVAL out of range, SWE_EDEVICE when capture fails. */
swe_status swe_prepare_graphs(swe_state *s, int32_t steps_per_graph);

/* Copies the state to the host in original cell order as doubles; any
 * pointer may be NULL.  H surface elevation, h depth, qx, qy discharges,
 * *t the current time. */
swe_status swe_state_read(const swe_state *s, double *H, double *h, double *qx, double *qy, double *t);

/* Diagnostics computed on the device: volume sum (H - z)|Omega| (compensated
 * FP64, fixed order), the time integral of the mass flux leaving through open
 * boundaries, the volume added by positivity clips, and the step count.
 * The scheme is conservative: mass(t) = mass(0) - bnd_flux + clipped. */
swe_status swe_mass(const swe_state *s, double *mass, double *bnd_flux, double *clipped, int64_t *steps);
/* The part of bnd_flux that crossed the boundary edges carrying `tag`
 * (positive: water left the domain; an inflow's is minus the volume it
 * delivered), summed over those edges' accumulators in a fixed order.
 * 0 for a tag with no open edges. */
swe_status swe_boundary_flux(const swe_state *s, int32_t tag, double *volume);

/* ---- passive species (section "Scalar advection-diffusion": eq.
 * scalar_goveq without the diffusion tensor, updated by eq.
 * scl:updateformula with the advective fluxes only).  Per species c the
 * specific mass q_c = h phi_c is carried by the HLLC mass flux of each edge
 * times the concentration of the cell the water leaves (phi = q/h in cells
 * with water, 0 in dry ones).  Walls carry nothing; zero-gradient and
 * prescribed-surface edges repeat the interior concentration; active inflow
 * edges carry their condition's inflow concentration.  A cell the step leaves
 * without water keeps no species mass; the mass so removed is tallied.
 *
 * swe_state_set_scalars: ns in 0..5 species (0 removes them).  phi0 (host,
 * ns x n_cells doubles, original cell order; NULL = 0) gives initial
 * concentrations: q = h phi0 of the state's current depth.  phi_in (host,
 * n_bc x ns doubles in the order of the bcs given to swe_state_init; NULL =
 * 0) gives the inflow concentrations.  Allocates 2 ns n_cells values of the
 * state's precision; switches the state to 256-cell tiles (the only tile size
 * of the species-carrying step; swe_autotune then keeps it).  States with
 * species cannot join a batch.  SWE_EINVAL for ns out of range or non-finite
 * values, SWE_ENOMEM when the device allocation fails (species removed). */
swe_status swe_state_set_scalars(swe_state *s, int32_t ns, const double *phi0, const double *phi_in);
/* Copies the specific masses q (ns x n_cells doubles, original cell order) to
 * host memory; nothing is written when the state has no species. */
swe_status swe_state_read_scalars(const swe_state *s, double *q);
/* Per species (arrays of ns doubles, any may be NULL): mass sum q |Omega|
 * (compensated FP64, fixed order), the time integral of the species flux
 * leaving through open boundaries, and the mass added by resetting cells
 * left dry: mass(t) = mass(0) - bnd_flux + clipped.  Like the water's clip
 * volume, the reset tally is kept per group of 64 cells in compensated FP64
 * and summed in a fixed order, so it is bitwise reproducible. */
swe_status swe_scalar_mass(const swe_state *s, double *mass, double *bnd_flux, double *clipped);

/* ---- diffusion of the species (section "Scalar advection-diffusion": the
 * governing eq. scalar_goveq with the diffusion tensor, reformulated by the
 * Cattaneo-type relaxation of eq. relaxation_terms; the relaxed flux of eq.
 * vecform_scalar2; the update of eq. scl:updateformula with the stiff
 * relaxation source by the locally implicit Euler step; the closure of
 * section "Scalar advection-diffusion closure relationships").  Per species
 * the auxiliary variables psi = (psi_x, psi_y) relax towards the gradient of
 * the concentration with relaxation time zeta; each edge carries the exact
 * solution of the two-wave Riemann problem of the linear relaxed system in
 * its normal direction (waves +- sqrt(K_nn / zeta)), with the edge's depth
 * the smaller of the two reconstructed depths and K the mean of the two
 * cells' tensors.  K = Km I + K^t, K^t = h u_* (alpha_T I + (alpha_L -
 * alpha_T) u u^T / |u|^2), u_* = |u| / c_f of the cell's friction closure.
 * Boundaries, standing internal walls and cells at or below h_min exchange
 * nothing by diffusion (mirrored states).  The relaxation waves of the
 * diffusing species bound the time step beside the water's.
 *
 * swe_state_set_diffusion: Km (ns doubles >= 0, m^2/s), alpha_L, alpha_T >= 0,
 * zeta > 0 [s]; psi0 (host, ns x n_cells x 2 doubles in original cell order,
 * or NULL = 0) the initial auxiliary variables.  Needs the species set first
 * (swe_state_set_scalars; setting species again removes the diffusion) and
 * no sources (SWE_EINVAL).  Allocates 4 ns n_cells values of the state's
 * precision (SWE_ENOMEM). */
swe_status swe_state_set_diffusion(swe_state *s, const double *Km, double alpha_L, double alpha_T, double zeta,
                                   const double *psi0);
/* Copies the auxiliary variables (ns x n_cells x 2 doubles, original cell
 * order) to host memory; nothing is written without diffusion. */
swe_status swe_state_read_psi(const swe_state *s, double *psi);

/* ---- external water sources and sinks S_h (the S_h paragraph of the
 * hydrodynamic closure relations; eq. swe_vectorial_form_sourceterms,
 * an explicit source in the continuity equation of eq.
 * hydrodynamicupdateformula: H += dt S_h after the fluxes, before the
 * friction split).  Each region has a series (linear in time, constant past
 * its ends, taken at the step's start time) of a total discharge [m^3/s]
 * spread evenly over the region's area (summed in ascending order), or of an
 * intensity [mm/h]; negative values remove water.  Modes: SWE_SRC_EXACT
 * adds or removes exactly dt S_h (a removal beyond the water a cell holds
 * after the fluxes sets SWE_ESINK; the step completes and the deficit is
 * clipped and tallied like a negative depth); SWE_SRC_AVAILABLE removes at
 * most that water (values must be <= 0); SWE_SRC_INFINITY removes all of it
 * (no series).  A cell a sink empties gets H = z exactly.  Removed water
 * carries the cell's species concentrations; added water carries none. */
enum { SWE_SRC_EXACT = 0, SWE_SRC_AVAILABLE = 1, SWE_SRC_INFINITY = 2 };
enum { SWE_SRC_DISCHARGE = 0, SWE_SRC_INTENSITY = 1 };
typedef struct {
    int32_t mode;       /* SWE_SRC_* mode */
    int32_t unit;       /* SWE_SRC_DISCHARGE or SWE_SRC_INTENSITY */
    const double *t;    /* n_pts increasing times [s] (host) */
    const double *v;    /* n_pts values (host) */
    int32_t n_pts;      /* >= 1, or 0 for SWE_SRC_INFINITY */
} swe_source;
/* Sets the sources of a state: cell_region (host, n_cells ints in original
 * cell order) gives each cell's index into src[n_src], or -1.  n_src = 0
 * removes them.  Copies everything; allocates per cell 4 bytes and per tile
 * 16 bytes of device memory.  States with sources keep their tile size under
 * swe_autotune and cannot join a batch.  SWE_EINVAL for bad modes, units,
 * series, region indices or an empty discharge region; SWE_ENOMEM. */
swe_status swe_state_set_sources(swe_state *s, const int32_t *cell_region, const swe_source *src, int32_t n_src);
/* Volume the sources have added since they were set (negative: removed),
 * compensated FP64 over per-tile accumulators in a fixed order.  With
 * sources the balance of swe_mass reads mass(t) = mass(0) - bnd_flux +
 * clipped + source volume. */
swe_status swe_source_volume(const swe_state *s, double *volume);

/* ---- morphodynamics (section "Morphodynamics": the Exner equation eq.
 * exner, updated by eq. exnerupdateformula with the HLL sediment flux eq.
 * exner_hll and the speeds of eq. exner_wave_assign / eq.
 * exner_wave_estimation; transport closures of Table sedtransport_closure).
 * Synchronous-decoupled: the bed moves every step with the hydrodynamic dt,
 * from the state at the step's start, and the water depth is kept as it
 * moves.  The Shields number is theta = |u|^2 / (c_f^2 (s - 1) g d_m) with
 * the cell's friction closure; dry (h <= h_min) and frictionless cells and
 * cells at their non-erodible bed carry no sediment; the transport is
 * aligned with the flow; dq_B,n/dq_n is taken at fixed depth and tangential
 * velocity; walls carry no sediment and open edges the cell's own normal
 * transport.  Sediment sources, local slope / curvature corrections and
 * Smart-Jaggi are not built. */
enum { SWE_SED_MPM = 0, SWE_SED_GRASS = 1, SWE_SED_EH = 2 };
typedef struct {
    int32_t closure;  /* SWE_SED_*: MPM alpha (theta - theta_cr)^m sqrt((s-1) g d^3); Grass alpha (|u| - u_cr)^m;
                         Engelund-Hansen 0.05 c_f^2 theta^(5/2) sqrt((s-1) g d^3) */
    double alpha;     /* MPM or Grass coefficient (>= 0) */
    double m;         /* MPM or Grass exponent (> 0) */
    double thr;       /* theta_cr (MPM) or u_cr [m/s] (Grass), >= 0 */
    double d_m;       /* representative grain diameter [m] > 0 */
    double s_rel;     /* relative density rho_s / rho > 1 */
    double porosity;  /* bed porosity in [0, 1) */
} swe_morpho;
/* Switches the Exner module on (mo != NULL) or off (mo == NULL).  z_rel
 * (host, n_cells doubles <= 0 in original cell order, or NULL) puts a
 * non-erodible bed that far below the current bed: cells at it carry no
 * sediment, and an update below it is clipped to it with the sediment volume
 * so added tallied.  The module runs with 256-cell tiles and excludes passive
 * species, external sources and batches (SWE_EINVAL).  Clears the sediment
 * tallies. */
swe_status swe_state_set_morpho(swe_state *s, const swe_morpho *mo, const double *z_rel);
/* Copies the bed elevation (n_cells doubles, original cell order) to host memory. */
swe_status swe_state_read_bed(const swe_state *s, double *z);
/* Sediment volume (1 - p) sum z |Omega| (compensated FP64, fixed order),
 * the volume that left through open boundaries, and the volume the fixed-bed
 * clip added since the module was switched on: volume(t) = volume(0) -
 * bnd + clipped.  The clip tally is kept per group of 64 cells in
 * compensated FP64 and summed in a fixed order (bitwise reproducible). */
swe_status swe_morpho_volume(const swe_state *s, double *volume, double *bnd, double *clipped);

/* Times k steps for each tile size (block size) in {128, 256, 512}, in
 * three interleaved rounds, keeps the size with the fastest round for this
 * state, and restores the state exactly as it was.
 * *block_size (may be NULL) receives the choice.  Results are bitwise
 * independent of the choice.  States with species, sources or a moving bed
 * keep their tile.  Allocates a copy of the state for the duration. */
swe_status swe_autotune(swe_state *s, int32_t k, int32_t *block_size);

/* ---- batched ensembles (many independent states stepped by one persistent
 * kernel per step, each with its own dt; paper motivation: ensemble and
 * calibration runs through batch execution).  All states of a batch share
 * precision and device. budget_bytes (0 = unlimited) bounds the summed
 * footprint; swe_batch_add returns SWE_EBUDGET when it would be exceeded. */
swe_status swe_batch_create(int32_t precision, int64_t budget_bytes, const swe_device *dev, swe_batch **out);
void swe_batch_destroy(swe_batch *b);
/* Adds a state with its own end time; *slot receives its id.  The batch
 * borrows the state: it must outlive its membership (remove it before
 * swe_state_destroy), and while a member it advances only through the batch
 * (swe_state_read and the diagnostics stay valid after swe_batch_step).
 * States with species, sources, a moving bed or the draining-time limiter
 * are refused (SWE_EINVAL), as are a state already in the batch and one on
 * another stream. */
swe_status swe_batch_add(swe_batch *b, swe_state *s, double t_end, int32_t *slot);
/* Removes (detaches) a state; the state itself stays valid. */
swe_status swe_batch_remove(swe_batch *b, int32_t slot);
/* Runs up to k steps of every unfinished member (one hipGraph of k
 * persistent launches) and waits.  *n_active (may be NULL) receives how many
 * members are still short of their end time. */
swe_status swe_batch_step(swe_batch *b, int32_t k, int32_t *n_active);
/* Issues the same work without waiting (for overlap and timing). */
swe_status swe_batch_launch(swe_batch *b, int32_t k);
/* The autotuner of the persistent batched step: times k launches over the
 * running members for each tile size in {128, 256, 512} (the persistent grid
 * follows the occupancy of each) in three interleaved rounds, keeps the size
 * with the fastest round, and restores every
 * member exactly as it was (state, boundary tallies, time level).
 * *block_size (may be NULL) receives the choice.  Results are bitwise
 * independent of the choice.  Allocates a copy of every running member for
 * the duration (SWE_ENOMEM). */
swe_status swe_batch_autotune(swe_batch *b, int32_t k, int32_t *block_size);
/* Per-member status after the last swe_batch_step: done flag (t >= t_end
 * or an error), error code (0 or SWE_E*), time and steps of the member in
 * slot `slot` (as returned by swe_batch_add); each output may be NULL. */
swe_status swe_batch_poll(swe_batch *b, int32_t slot, int32_t *done, int32_t *error, double *t, int64_t *steps);
int64_t swe_batch_footprint(const swe_batch *b);

/* For callers that cannot allocate device memory -- code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * persistent batched step of swe_batch_step without a batch object.  Runs
 * up to k steps of each of the n states (states[i] until t_end[i], the last
 * step shortened to land on it) in one persistent launch per step and
 * waits; *n_active (may be NULL) receives how many states are still short
 * of their end time and error-free.  Results are bitwise those of
 * swe_batch_step.  The work list (the states' kernel parameter blocks and
 * their (state, tile) pairs) is staged in a file-scope device array of the
 * library of fixed size (about 2.1 MiB, one copy per device, held until the
 * process ends) instead of memory the library allocates: the call allocates
 * no device memory and calls no allocating routine.  Limits: 1 <= n <= 64
 * states and at most 262144 tiles in total (about 67M cells at the default
 * 256-cell tiles); the states must share precision, tile size and stream,
 * and carry no species, sources, moving bed or limiter (SWE_EINVAL).  The
 * array is shared by every call on a device and keeps the last call's work
 * list: calls that overlap on one device (from several host threads or
 * streams) race.  Returns the first member error (SWE_ENONFINITE, ...) after
 * all n states have stepped. */
swe_status swe_batch_step_noalloc(swe_state *const *states, const double *t_end, int32_t n, int32_t k,
                                  int32_t *n_active);

const char *swe_last_error(void);
/* Library version string. */
const char *swe_version(void);

#ifdef __cplusplus
}
#endif
#endif
