/*
 * FP64 CPU oracle for the explicit first-order finite-volume shallow-water
 * step on a conforming triangulation.  TEST INFRASTRUCTURE ONLY: nothing on
 * the product path may include, link or call this.  It exists so that the
 * GPU library can be checked against a plain, slow, obviously correct
 * implementation written from the paper.
 *
 * The oracle loops over EDGES (each edge flux computed once), stores the
 * three per-edge contributions of every cell in its local edge order and
 * sums them in that order.  Compiled with -ffp-contract=off.
 *
 * Status codes: 0 ok, -1 invalid input, -2 out of memory, -4 non-finite
 * state, -7 no finite time step, -8 an exact sink exceeded a cell's water
 * (the step is complete; the deficit was clipped and tallied).
 */
#ifndef SWE_ORACLE_H
#define SWE_ORACLE_H
#include <stdint.h>

typedef struct om_mesh om_mesh;
typedef struct om_sim om_sim;

/* boundary kinds */
enum { OM_WALL = 0, OM_INFLOW_UNIFORM = 1, OM_OUTFLOW_ZEROGRAD = 2, OM_ZHYDROGRAPH = 3, OM_INFLOW_FROUDE = 4,
       OM_OUTFLOW_UNIFORM = 5, OM_OUTFLOW_WEIR = 6, OM_OUTFLOW_HQ = 7, OM_DYNAMIC_WALL = 8 };
#define OM_MAX_SPECIES 5
/* friction closures (Table friction_closure) */
enum { OM_MANNING = 0, OM_STRICKLER = 1, OM_CHEZY = 2, OM_BEZZOLA = 3 };

om_mesh *om_mesh_new(const double *node_xyz, int64_t n_nodes, const int32_t *tri, int64_t n_tri,
                     const int32_t *bnd_seg, const int32_t *bnd_tag, int64_t n_seg,
                     char *err, int err_len);
void om_mesh_free(om_mesh *m);
int64_t om_mesh_n_edges(const om_mesh *m);
int64_t om_mesh_n_boundary_edges(const om_mesh *m);
/* per-cell area, bed, and per cell-local edge: rho, outward unit normal, length */
void om_mesh_geometry(const om_mesh *m, double *area, double *zb, double *rho3,
                      double *nx3, double *ny3, double *len3, int32_t *nbr3);

om_sim *om_sim_new(const om_mesh *m, double g, double cfl, double h_min, double dt_max,
                   const double *H0, const double *h0, const double *qx0, const double *qy0,
                   const double *manning, int32_t n_bc, const int32_t *bc_tag,
                   const int32_t *bc_kind, const double *bc_slope, const int32_t *bc_npts,
                   const double *bc_t, const double *bc_Q, const double *bc_par, double t0, char *err,
                   int err_len);
void om_sim_free(om_sim *s);
/* closure and per-cell parameter (n, k_str, K_s or y_R); default Manning
 * with the array given to om_sim_new.  0 or -1 (message in err). */
int om_sim_set_friction(om_sim *s, int32_t kind, const double *par, char *err, int err_len);

double om_next_dt(const om_sim *s, double t_end);
int om_step(om_sim *s, double t_end, double *dt_taken);
int om_run_until(om_sim *s, double t_end, int64_t max_steps, int64_t *n_steps);
void om_get_state(const om_sim *s, double *H, double *qx, double *qy, double *t);
void om_set_state(om_sim *s, const double *H, const double *qx, const double *qy, double t);
void om_diag(const om_sim *s, double *mass, double *bnd_flux, double *clipped, int64_t *steps);
/* boundary-flux integral over the edges of boundary condition b (its index
 * in the list given to om_sim_new); positive: left the domain */
double om_bc_flux(const om_sim *s, int32_t b);
/* species diffusion by the relaxation system (eq. relaxation_terms,
 * vecform_scalar2, scl:updateformula); see swe_oracle.c */
int om_sim_set_diffusion(om_sim *s, const double *Km, double alpha_L, double alpha_T, double zeta,
                         const double *psi0, char *err, int elen);
void om_get_psi(const om_sim *s, double *psi);

/* single-edge pieces, exposed for the pin tests */
void om_hllc(double hL, double unL, double utL, double hR, double unR, double utR, double g,
             double F[3]);
double om_friction(double q_abs_scale, double h, double gn2, double dt, double h_min);
double om_friction_cf(int32_t kind, double par, double h);

/* passive scalars (advected): ns species (<= OM_MAX_SPECIES) with initial
 * concentrations phi0[ns][nc] (NULL = 0) and inflow concentrations
 * phi_in[nbc][ns] of the boundary conditions (NULL = 0).  0 or -1. */
int om_sim_set_scalars(om_sim *s, int32_t ns, const double *phi0, const double *phi_in, char *err, int err_len);
/* specific masses q = h phi, [ns][nc] */
void om_get_scalars(const om_sim *s, double *q);
void om_scalar_diag(const om_sim *s, double *mass, double *bnd, double *clipped);
double om_friction_closure(int32_t kind, double par, double q_abs, double h, double dt, double h_min);

/* external water sources and sinks S_h: cell_src[nc] gives each cell's
 * region (-1: none); region r has a mode, a unit (total discharge [m^3/s]
 * over the region, or intensity [mm/h]) and a series of npts[r] points,
 * concatenated in t and v (INFINITY sinks need none).  n_src = 0 removes
 * them.  0 or -1. */
enum { OM_SRC_EXACT = 0, OM_SRC_AVAILABLE = 1, OM_SRC_INFINITY = 2 };
enum { OM_SRC_DISCHARGE = 0, OM_SRC_INTENSITY = 1 };
int om_sim_set_sources(om_sim *s, const int32_t *cell_src, int32_t n_src, const int32_t *mode,
                       const int32_t *unit, const int32_t *npts, const double *t, const double *v, char *err,
                       int err_len);
/* morphodynamics (Exner, HLL sediment flux): closure OM_SED_* with its
 * alpha, exponent m and threshold (theta_cr, or u_cr for GRASS), grain
 * diameter d_m, relative density s, porosity p; z_rel[nc] (<= 0, NULL =
 * none) puts a non-erodible bed below the initial bed.  closure < 0
 * switches it off.  0 or -1. */
enum { OM_SED_MPM = 0, OM_SED_GRASS = 1, OM_SED_EH = 2 };
int om_sim_set_morpho(om_sim *s, int32_t closure, double alpha, double m, double thr, double d_m, double s_rel,
                      double porosity, const double *z_rel, char *err, int err_len);
void om_get_bed(const om_sim *s, double *z);
/* Cell beds per cell (instead of the node means) with surfaces H, or NULL
 * to keep each cell's depth.  0 or -1 (message in err). */
int om_sim_set_bed(om_sim *s, const double *z, const double *H, char *err, int err_len);
/* Threads of the OpenMP build (n > 0 sets them); the serial build returns 1. */
int om_threads(int n);
/* draining-time positivity limiter on (1) or off (0, the default) */
int om_sim_set_drain(om_sim *s, int on, char *err, int err_len);
void om_morpho_diag(const om_sim *s, double *volume, double *bnd, double *clipped);
/* one cell's normal transport, its derivative with respect to the normal
 * discharge, and the two HLL speeds, for the pin tests */
void om_sed_cell(int32_t closure, double alpha, double m, double thr, double d_m, double s_rel, double g, double h,
                 double u, double v, double cf2, double nx, double ny, double *qbn, double *D, double *l1,
                 double *l2);
/* volume the sources added so far (negative: removed); the balance is
 * M(t) = M(0) - bnd_flux + clipped + source volume */
double om_source_volume(const om_sim *s);
#endif
