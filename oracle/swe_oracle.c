/*
 * FP64 CPU oracle for the shallow-water step.  TEST INFRASTRUCTURE ONLY (see
 * swe_oracle.h).  Plain C, edge loop, no blocking, no fusion beyond what the
 * scheme states.  Every function names the passage of the paper it follows.
 *
 * Scheme (paper, section "Numerical solution" / "Hydrodynamics"):
 *   unknowns U = [H, qx, qy], h = H - z_B                 (eq. swe_vectorial_form)
 *   U_i^{n+1} = U_i^n - dt/|Omega_i| sum_j l_ij F_ij + dt S_i   (eq. hydrodynamicupdateformula)
 *   F_ij from the HLLC approximate Riemann solver         (HLLC paragraph, Toro 1994)
 *   bed slope by hydrostatic reconstruction of modified states, written in
 *   fluctuation form (well balanced)                       (source-term paragraph)
 *   friction by operator splitting after the flux update  (source-term paragraph,
 *                                                          eq. friction_closure, Table friction_closure)
 *   dt = CFL min_i min_j rho_ij / lambda_ij                (eq. CFL_condition)
 *   walls: reflective, frictionless, impermeable          (section "Boundary conditions")
 *
 * Readings where the paper is silent are listed where they are used.
 */
#include "swe_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* depth below which a reconstructed edge state is dry [m] */
#define OM_H_DRY 1e-12

struct om_mesh {
    int64_t nv, nc, ne, nb;
    double *x, *y, *zn;
    int32_t *tri;        /* 3*nc, counter-clockwise */
    double *area, *zb;   /* per cell */
    int32_t *eL, *eR;    /* cells of edge e; eR = -1 on the boundary */
    int32_t *ekL, *ekR;  /* local edge index of e inside L and R */
    int32_t *etag;       /* boundary tag, -1 when untagged */
    int8_t *eup;         /* tagged interior edge: 1 when L lies left of its segment (first node to second) */
    double *enx, *eny, *elen; /* unit normal pointing from L to R (outward of L), length */
    int32_t *cell_edge;  /* 3*nc: edge id of the cell's local edge k */
    double *rho;         /* 3*nc: twice the centroid-to-edge distance */
};

typedef struct {
    int32_t tag, kind, npts;
    double slope, length;  /* slope: energy slope, Froude number, crest elevation or collapse time */
    double par;            /* Poleni factor of a weir, collapse depth of a dynamic wall */
    double gone;           /* dynamic wall with a collapse depth: the time it is gone from (+inf until then) */
    double *t, *Q;
} om_bc;

struct om_sim {
    const om_mesh *m;
    double g, cfl, h_min, dt_max;
    double *H, *qx, *qy;
    double *z;           /* cell bed elevation (the mesh's, moved by the Exner module) */
    int32_t fkind;       /* friction closure (OM_MANNING ... OM_BEZZOLA) */
    double *gn2;         /* per cell: g n^2 (Manning), g / k^2 (Strickler), K_s (Chezy), y_R (Bezzola) */
    double t;
    int32_t nbc;
    om_bc *bc;
    int32_t *ebc;        /* per edge: index into bc[] or -1 (wall) */
    double *cont;        /* 9*nc: contribution of each local edge, 3 components */
    double bsum, bcomp;  /* Neumaier sum of dt * l * mass flux leaving the domain */
    double *bcsum;       /* per boundary condition: the same sum over its edges (sum, compensation) */
    double clip, clipc;  /* Neumaier sum of volume added by the positivity clip */
    int64_t steps;
    /* passive scalars (section "Scalar advection-diffusion"): per species c
     * the specific mass q_c = h phi_c, [ns][nc] */
    int32_t ns;
    double *sq, *sphi, *scont, *phi_in;
    double sbsum[OM_MAX_SPECIES], sbcomp[OM_MAX_SPECIES];
    double sclip[OM_MAX_SPECIES], sclipc[OM_MAX_SPECIES];  /* mass set by the dry-cell reset */
    /* diffusion of the species by the relaxation system of eq.
     * relaxation_terms: per species the molecular diffusivity dKm, the
     * dispersion coefficients daL, daT and the relaxation time dzeta; per
     * species and cell the auxiliary variables (psi_x, psi_y) [ns][nc][2]; per
     * cell at t^n its depth and turbulent dispersion tensor (h, Kxx, Kxy,
     * Kyy), with h = 0 for a cell at or below h_min; per species, cell and
     * local edge the diffusive contributions (q, psi_x, psi_y) */
    int diff;
    double dKm[OM_MAX_SPECIES], daL, daT, dzeta;
    double *spsi, *dK, *dcont;
    /* external water sources and sinks S_h: per region the mode (kind),
     * the series of its value (t, Q) and the factor from that value to a
     * rate in m/s (length); per cell the region or -1 */
    int32_t nsrc;
    om_bc *src;
    int32_t *csrc;
    double *sfac;        /* per cell: fraction of its water a sink left (species follow it) */
    double ssum, scomp;  /* Neumaier sum of the volume the sources added (negative: removed) */
    /* morphodynamics (Exner): closure and its parameters, porosity, the
     * non-erodible bed per cell, the per-(cell, local edge) bed
     * contributions l q_B, and the sediment tallies */
    int morpho;
    int32_t sclos;
    double salpha, sm, sthr, sd, srel, spor;
    double *zfix, *bcont;
    double bvsum, bvcomp;    /* sediment volume that left through open boundaries */
    double bclip, bclipc;    /* sediment volume added by the fixed-bed clip */
    /* draining-time positivity limiter: per cell theta = min(1, draining
     * time / dt), and per (cell, local edge) the mass leaving through it */
    int drain;
    double *theta, *dout;
    /* per-edge boundary volumes and per-cell clip / source volumes of the
     * step being taken: the loops fill them in any order (the OpenMP build
     * runs them on all cores), then the Neumaier sums take them in edge or
     * cell order, exactly as a serial loop would */
    double *ebvol, *cclip, *csrcv;
    unsigned char *eflag, *cflag;
};

static void seterr(char *err, int len, const char *msg) {
    if (err && len > 0) {
        strncpy(err, msg, (size_t)len - 1);
        err[len - 1] = 0;
    }
}

static void neumaier(double *sum, double *comp, double v) {
    double t = *sum + v;
    if (fabs(*sum) >= fabs(v))
        *comp += (*sum - t) + v;
    else
        *comp += (v - t) + *sum;
    *sum = t;
}

static int cmp_double(const void *p, const void *q) {
    double a = *(const double *)p, b = *(const double *)q;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* ------------------------------------------------------------------ mesh */
typedef struct {
    int32_t a, b, cell, k;
} half_edge;

static int cmp_half(const void *p, const void *q) {
    const half_edge *u = (const half_edge *)p, *v = (const half_edge *)q;
    if (u->a != v->a) return u->a < v->a ? -1 : 1;
    if (u->b != v->b) return u->b < v->b ? -1 : 1;
    if (u->cell != v->cell) return u->cell < v->cell ? -1 : 1;
    return 0;
}

typedef struct {
    int32_t a, b, tag, first;   /* first: the segment's first node as given */
} seg_key;

static int cmp_seg(const void *p, const void *q) {
    const seg_key *u = (const seg_key *)p, *v = (const seg_key *)q;
    if (u->a != v->a) return u->a < v->a ? -1 : 1;
    if (u->b != v->b) return u->b < v->b ? -1 : 1;
    return 0;
}

void om_mesh_free(om_mesh *m) {
    if (!m) return;
    free(m->x); free(m->y); free(m->zn); free(m->tri); free(m->area); free(m->zb);
    free(m->eL); free(m->eR); free(m->ekL); free(m->ekR); free(m->etag); free(m->eup);
    free(m->enx); free(m->eny); free(m->elen); free(m->cell_edge); free(m->rho);
    free(m);
}

/* Conforming triangulation (section "Domain discretization"): every interior
 * edge is shared by exactly two cells; n_ij points toward the neighbour.
 * Reading: the cell bed is the mean of its three node elevations (meshes
 * carry node elevations); the orientation of an interior edge is taken from
 * the cell with the smaller index. */
om_mesh *om_mesh_new(const double *xyz, int64_t nv, const int32_t *tri, int64_t nc,
                     const int32_t *seg, const int32_t *tag, int64_t ns, char *err, int elen) {
    om_mesh *m = (om_mesh *)calloc(1, sizeof(om_mesh));
    half_edge *he = NULL;
    seg_key *sk = NULL;
    if (!m) { seterr(err, elen, "out of memory"); return NULL; }
    if (nv < 3 || nc < 1) { seterr(err, elen, "empty mesh"); goto fail; }
    m->nv = nv;
    m->nc = nc;
    m->x = malloc(sizeof(double) * nv); m->y = malloc(sizeof(double) * nv);
    m->zn = malloc(sizeof(double) * nv);
    m->tri = malloc(sizeof(int32_t) * 3 * nc);
    m->area = malloc(sizeof(double) * nc); m->zb = malloc(sizeof(double) * nc);
    m->cell_edge = malloc(sizeof(int32_t) * 3 * nc);
    m->rho = malloc(sizeof(double) * 3 * nc);
    he = malloc(sizeof(half_edge) * 3 * nc);
    if (!m->x || !m->y || !m->zn || !m->tri || !m->area || !m->zb || !m->cell_edge || !m->rho || !he) {
        seterr(err, elen, "out of memory"); goto fail;
    }
    for (int64_t v = 0; v < nv; v++) {
        m->x[v] = xyz[3 * v]; m->y[v] = xyz[3 * v + 1]; m->zn[v] = xyz[3 * v + 2];
        if (!isfinite(m->x[v]) || !isfinite(m->y[v]) || !isfinite(m->zn[v])) {
            seterr(err, elen, "non-finite node coordinate"); goto fail;
        }
    }
    for (int64_t i = 0; i < nc; i++) {
        int32_t a = tri[3 * i], b = tri[3 * i + 1], c = tri[3 * i + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv || a == b || b == c || a == c) {
            seterr(err, elen, "bad triangle vertex index"); goto fail;
        }
        double cross = (m->x[b] - m->x[a]) * (m->y[c] - m->y[a]) - (m->y[b] - m->y[a]) * (m->x[c] - m->x[a]);
        if (cross < 0) { int32_t t = b; b = c; c = t; cross = -cross; }
        if (!(cross > 0)) { seterr(err, elen, "degenerate triangle"); goto fail; }
        m->tri[3 * i] = a; m->tri[3 * i + 1] = b; m->tri[3 * i + 2] = c;
        m->area[i] = 0.5 * cross;
        m->zb[i] = (m->zn[a] + m->zn[b] + m->zn[c]) / 3.0;
        for (int k = 0; k < 3; k++) {
            int32_t p = m->tri[3 * i + k], q = m->tri[3 * i + (k + 1) % 3];
            he[3 * i + k].a = p < q ? p : q;
            he[3 * i + k].b = p < q ? q : p;
            he[3 * i + k].cell = (int32_t)i;
            he[3 * i + k].k = k;
        }
    }
    qsort(he, (size_t)(3 * nc), sizeof(half_edge), cmp_half);
    /* count edges */
    int64_t ne = 0, nb = 0;
    for (int64_t h = 0; h < 3 * nc;) {
        int64_t g = h + 1;
        while (g < 3 * nc && he[g].a == he[h].a && he[g].b == he[h].b) g++;
        if (g - h > 2) { seterr(err, elen, "non-conforming edge shared by 3+ triangles"); goto fail; }
        if (g - h == 1) nb++;
        ne++;
        h = g;
    }
    m->ne = ne;
    m->nb = nb;
    m->eL = malloc(sizeof(int32_t) * ne); m->eR = malloc(sizeof(int32_t) * ne);
    m->ekL = malloc(sizeof(int32_t) * ne); m->ekR = malloc(sizeof(int32_t) * ne);
    m->etag = malloc(sizeof(int32_t) * ne);
    m->eup = malloc(sizeof(int8_t) * ne);
    m->enx = malloc(sizeof(double) * ne); m->eny = malloc(sizeof(double) * ne);
    m->elen = malloc(sizeof(double) * ne);
    if (!m->eL || !m->eR || !m->ekL || !m->ekR || !m->etag || !m->eup || !m->enx || !m->eny || !m->elen) {
        seterr(err, elen, "out of memory"); goto fail;
    }
    sk = malloc(sizeof(seg_key) * (ns > 0 ? ns : 1));
    if (!sk) { seterr(err, elen, "out of memory"); goto fail; }
    for (int64_t s = 0; s < ns; s++) {
        int32_t p = seg[2 * s], q = seg[2 * s + 1];
        if (p < 0 || q < 0 || p >= nv || q >= nv || p == q) { seterr(err, elen, "bad boundary segment"); goto fail; }
        sk[s].a = p < q ? p : q; sk[s].b = p < q ? q : p; sk[s].tag = tag[s]; sk[s].first = p;
    }
    qsort(sk, (size_t)ns, sizeof(seg_key), cmp_seg);
    int64_t matched = 0;
    int64_t e = 0;
    for (int64_t h = 0; h < 3 * nc; e++) {
        int64_t g = h + 1;
        while (g < 3 * nc && he[g].a == he[h].a && he[g].b == he[h].b) g++;
        /* he[] is sorted by cell within a key, so he[h] has the smaller cell */
        int32_t L = he[h].cell, kL = he[h].k;
        m->eL[e] = L; m->ekL[e] = kL;
        m->cell_edge[3 * L + kL] = (int32_t)e;
        int32_t p = m->tri[3 * L + kL], q = m->tri[3 * L + (kL + 1) % 3];
        double dx = m->x[q] - m->x[p], dy = m->y[q] - m->y[p];
        double l = sqrt(dx * dx + dy * dy);
        m->elen[e] = l;
        m->enx[e] = dy / l;   /* outward of a counter-clockwise cell */
        m->eny[e] = -dx / l;
        m->etag[e] = -1;
        m->eup[e] = 0;
        if (g - h == 2) {
            int32_t R = he[h + 1].cell, kR = he[h + 1].k;
            int32_t pR = m->tri[3 * R + kR];
            if (pR != q) { seterr(err, elen, "inconsistent orientation (overlapping triangles)"); goto fail; }
            m->eR[e] = R; m->ekR[e] = kR;
            m->cell_edge[3 * R + kR] = (int32_t)e;
            /* a tagged interior edge can carry an internal condition; L,
             * counter-clockwise, walks the edge from p to q, so it lies on
             * the left of the segment when the segment starts at p */
            seg_key key = {he[h].a, he[h].b, 0, 0};
            seg_key *f = ns > 0 ? bsearch(&key, sk, (size_t)ns, sizeof(seg_key), cmp_seg) : NULL;
            if (f) { m->etag[e] = f->tag; m->eup[e] = (int8_t)(f->first == p); matched++; }
        } else {
            m->eR[e] = -1; m->ekR[e] = -1;
            seg_key key = {he[h].a, he[h].b, 0, 0};
            seg_key *f = ns > 0 ? bsearch(&key, sk, (size_t)ns, sizeof(seg_key), cmp_seg) : NULL;
            if (f) { m->etag[e] = f->tag; matched++; }
        }
        h = g;
    }
    if (matched != ns) { seterr(err, elen, "segment is not an edge of the mesh"); goto fail; }
    /* rho_ij: twice the distance from the centroid of i to edge j
     * (eq. CFL_condition); the centroid is at a third of the height, so
     * rho = 2 * (2|Omega|/l) / 3. */
    for (int64_t i = 0; i < nc; i++)
        for (int k = 0; k < 3; k++) {
            double l = m->elen[m->cell_edge[3 * i + k]];
            m->rho[3 * i + k] = 4.0 * m->area[i] / (3.0 * l);
        }
    free(he);
    free(sk);
    return m;
fail:
    free(he);
    free(sk);
    om_mesh_free(m);
    return NULL;
}

int64_t om_mesh_n_edges(const om_mesh *m) { return m->ne; }
int64_t om_mesh_n_boundary_edges(const om_mesh *m) { return m->nb; }

void om_mesh_geometry(const om_mesh *m, double *area, double *zb, double *rho3, double *nx3,
                      double *ny3, double *len3, int32_t *nbr3) {
    for (int64_t i = 0; i < m->nc; i++) {
        if (area) area[i] = m->area[i];
        if (zb) zb[i] = m->zb[i];
        for (int k = 0; k < 3; k++) {
            int32_t e = m->cell_edge[3 * i + k];
            double s = (m->eL[e] == i) ? 1.0 : -1.0;
            if (rho3) rho3[3 * i + k] = m->rho[3 * i + k];
            if (nx3) nx3[3 * i + k] = s * m->enx[e];
            if (ny3) ny3[3 * i + k] = s * m->eny[e];
            if (len3) len3[3 * i + k] = m->elen[e];
            if (nbr3) nbr3[3 * i + k] = (m->eL[e] == i) ? m->eR[e] : m->eL[e];
        }
    }
}

/* -------------------------------------------------------------- simulation */
void om_sim_free(om_sim *s) {
    if (!s) return;
    for (int b = 0; b < s->nbc; b++) { free(s->bc[b].t); free(s->bc[b].Q); }
    free(s->z); free(s->bc); free(s->ebc); free(s->H); free(s->qx); free(s->qy); free(s->gn2); free(s->cont);
    free(s->sq); free(s->sphi); free(s->scont); free(s->phi_in);
    free(s->spsi); free(s->dK); free(s->dcont);
    for (int r = 0; r < s->nsrc; r++) { free(s->src[r].t); free(s->src[r].Q); }
    free(s->src); free(s->csrc); free(s->sfac);
    free(s->zfix); free(s->bcont);
    free(s->theta); free(s->dout);
    free(s->ebvol); free(s->eflag); free(s->cclip); free(s->csrcv); free(s->cflag); free(s->bcsum);
    free(s);
}

/* Initial conditions (section "Initial conditions"): region-defined surface
 * elevation H or depth h and discharges per cell, or dry.  Reading: a
 * surface below the cell bed means a dry cell (H = z). */
om_sim *om_sim_new(const om_mesh *m, double g, double cfl, double h_min, double dt_max,
                   const double *H0, const double *h0, const double *qx0, const double *qy0,
                   const double *manning, int32_t nbc, const int32_t *bc_tag, const int32_t *bc_kind,
                   const double *bc_slope, const int32_t *bc_npts, const double *bc_t,
                   const double *bc_Q, const double *bc_par, double t0, char *err, int elen) {
    om_sim *s = (om_sim *)calloc(1, sizeof(om_sim));
    if (!s) { seterr(err, elen, "out of memory"); return NULL; }
    int64_t nc = m->nc;
    s->m = m;
    s->g = g; s->cfl = cfl; s->h_min = h_min; s->dt_max = dt_max; s->t = t0;
    if (!(g > 0) || !(cfl > 0 && cfl <= 1) || !(h_min > 0) || !(dt_max > 0) || !isfinite(t0)) {
        seterr(err, elen, "bad parameters"); goto fail;
    }
    s->z = malloc(sizeof(double) * (nc > 0 ? nc : 1));
    if (s->z) memcpy(s->z, m->zb, sizeof(double) * nc);
    s->H = malloc(sizeof(double) * nc); s->qx = malloc(sizeof(double) * nc);
    s->qy = malloc(sizeof(double) * nc); s->gn2 = malloc(sizeof(double) * nc);
    s->cont = malloc(sizeof(double) * 9 * nc);
    s->ebc = malloc(sizeof(int32_t) * m->ne);
    s->bc = calloc((size_t)(nbc > 0 ? nbc : 1), sizeof(om_bc));
    s->ebvol = malloc(sizeof(double) * (m->ne > 0 ? m->ne : 1));
    s->eflag = malloc(m->ne > 0 ? (size_t)m->ne : 1);
    s->cclip = malloc(sizeof(double) * (nc > 0 ? nc : 1));
    s->csrcv = malloc(sizeof(double) * (nc > 0 ? nc : 1));
    s->cflag = malloc(nc > 0 ? (size_t)nc : 1);
    s->bcsum = calloc((size_t)2 * (nbc > 0 ? nbc : 1), sizeof(double));
    if (!s->z || !s->H || !s->qx || !s->qy || !s->gn2 || !s->cont || !s->ebc || !s->bc || !s->ebvol ||
        !s->eflag || !s->cclip || !s->csrcv || !s->cflag || !s->bcsum) {
        seterr(err, elen, "out of memory"); goto fail;
    }
    for (int64_t i = 0; i < nc; i++) {
        double H;
        if (H0) {
            H = H0[i] > m->zb[i] ? H0[i] : m->zb[i];
        } else {
            double h = h0 ? h0[i] : 0.0;
            if (!(h >= 0)) { seterr(err, elen, "negative or non-finite initial depth"); goto fail; }
            H = m->zb[i] + h;
        }
        double n = manning ? manning[i] : 0.0;
        double qx = qx0 ? qx0[i] : 0.0, qy = qy0 ? qy0[i] : 0.0;
        if (!isfinite(H) || !isfinite(qx) || !isfinite(qy) || !(n >= 0) || !isfinite(n)) {
            seterr(err, elen, "non-finite initial state or negative Manning n"); goto fail;
        }
        s->H[i] = H; s->qx[i] = qx; s->qy[i] = qy;
        s->gn2[i] = g * n * n;
    }
    s->nbc = nbc;
    int64_t off = 0;
    for (int b = 0; b < nbc; b++) {
        om_bc *B = &s->bc[b];
        B->tag = bc_tag[b]; B->kind = bc_kind[b]; B->slope = bc_slope ? bc_slope[b] : 0.0;
        B->npts = bc_npts ? bc_npts[b] : 0;
        B->par = bc_par ? bc_par[b] : 0.0;
        B->gone = INFINITY;
        if (B->kind < 0 || B->kind > OM_DYNAMIC_WALL) { seterr(err, elen, "unknown boundary kind"); goto fail; }
        if (B->kind == OM_DYNAMIC_WALL && B->par < 0.0) { seterr(err, elen, "a dynamic wall's collapse depth must be >= 0"); goto fail; }
        if (!isfinite(B->slope) || !isfinite(B->par)) { seterr(err, elen, "non-finite boundary parameter"); goto fail; }
        if (B->kind == OM_ZHYDROGRAPH && B->npts < 1) { seterr(err, elen, "zhydrograph needs a series"); goto fail; }
        if (B->kind == OM_INFLOW_FROUDE && (B->npts < 1 || !(B->slope > 0))) { seterr(err, elen, "froude inflow needs a hydrograph and a positive Froude number"); goto fail; }
        if (B->kind == OM_OUTFLOW_UNIFORM && !(B->slope > 0)) { seterr(err, elen, "uniform outflow needs a positive slope"); goto fail; }
        if (B->kind == OM_OUTFLOW_WEIR && !(B->par > 0)) { seterr(err, elen, "a weir needs a positive Poleni factor"); goto fail; }
        if (B->kind == OM_OUTFLOW_HQ && B->npts < 1) { seterr(err, elen, "an h-Q relation needs a table"); goto fail; }
        if (B->kind == OM_INFLOW_UNIFORM || B->kind == OM_ZHYDROGRAPH || B->kind == OM_INFLOW_FROUDE ||
            B->kind == OM_OUTFLOW_HQ) {
            if (B->kind == OM_INFLOW_UNIFORM && (B->npts < 1 || !(B->slope > 0))) { seterr(err, elen, "inflow needs a hydrograph and a positive slope"); goto fail; }
            B->t = malloc(sizeof(double) * B->npts); B->Q = malloc(sizeof(double) * B->npts);
            if (!B->t || !B->Q) { seterr(err, elen, "out of memory"); goto fail; }
            for (int k = 0; k < B->npts; k++) {
                B->t[k] = bc_t[off + k]; B->Q[k] = bc_Q[off + k];
                if (!isfinite(B->t[k]) || !isfinite(B->Q[k])) { seterr(err, elen, "non-finite boundary series"); goto fail; }
                if (k > 0 && !(B->t[k] > B->t[k - 1])) { seterr(err, elen, "hydrograph times must increase"); goto fail; }
                if (B->kind == OM_OUTFLOW_HQ && B->Q[k] < 0.0) { seterr(err, elen, "h-Q discharges must be >= 0"); goto fail; }
            }
        }
        off += B->npts;
    }
    for (int64_t e = 0; e < m->ne; e++) {
        s->ebc[e] = -1;
        if (m->etag[e] < 0) continue;
        if (m->eR[e] >= 0) {
            /* internal condition (section "Hydrodynamic BCs", internal BCs):
             * a static wall, a dynamic wall until its collapse time, or a
             * rating curve (h-Q relation) */
            for (int b = 0; b < nbc; b++) {
                if (s->bc[b].tag != m->etag[e]) continue;
                if (s->bc[b].kind != OM_WALL && s->bc[b].kind != OM_DYNAMIC_WALL && s->bc[b].kind != OM_OUTFLOW_HQ) {
                    seterr(err, elen, "interior edges take walls, dynamic walls and h-Q relations only"); goto fail;
                }
                s->ebc[e] = b;
                break;
            }
            continue;
        }
        for (int b = 0; b < nbc; b++) {
            if (s->bc[b].tag != m->etag[e]) continue;
            if (s->bc[b].kind != OM_WALL) s->ebc[e] = b;
            break;
        }
        if (s->ebc[e] >= 0) {
            om_bc *B = &s->bc[s->ebc[e]];
            if ((B->kind == OM_INFLOW_UNIFORM || B->kind == OM_OUTFLOW_UNIFORM) && !(s->gn2[m->eL[e]] > 0)) {
                seterr(err, elen, "uniform inflow or outflow edge next to a cell with Manning n = 0"); goto fail;
            }
        }
    }
    /* Length of each boundary condition: its edge lengths summed from the
     * smallest up (reading: a numbering-independent order). */
    for (int b = 0; b < nbc; b++) {
        int64_t cnt = 0;
        for (int64_t e = 0; e < m->ne; e++) cnt += (s->ebc[e] == b);
        double *ls = malloc(sizeof(double) * (cnt > 0 ? cnt : 1));
        if (!ls) { seterr(err, elen, "out of memory"); goto fail; }
        int64_t k = 0;
        for (int64_t e = 0; e < m->ne; e++)
            if (s->ebc[e] == b) ls[k++] = m->elen[e];
        qsort(ls, (size_t)cnt, sizeof(double), cmp_double);
        double L = 0.0;
        for (k = 0; k < cnt; k++) L += ls[k];
        s->bc[b].length = L;
        free(ls);
    }
    return s;
fail:
    om_sim_free(s);
    return NULL;
}

/* Hydrograph Q(t): linear interpolation, constant beyond the ends.
 * Reading: the boundary is evaluated at the old time level t^n. */
static double hydrograph(const om_bc *B, double t) {
    if (t <= B->t[0]) return B->Q[0];
    if (t >= B->t[B->npts - 1]) return B->Q[B->npts - 1];
    int k = 0;
    while (B->t[k + 1] < t) k++;
    double w = (t - B->t[k]) / (B->t[k + 1] - B->t[k]);
    return B->Q[k] + w * (B->Q[k + 1] - B->Q[k]);
}

/* ---------------------------------------------------------------------------
 * External water sources and sinks (section "Closure relationships" of the
 * hydrodynamics, the S_h paragraph; eq. swe_vectorial_form_sourceterms): a
 * rate S_h [m/s], an explicit source in the continuity equation of eq.
 * hydrodynamicupdateformula, H += dt S_h, before the friction split.
 * Region r holds a series (linear in time, constant past its ends, taken at
 * t^n) of a total discharge [m^3/s], spread evenly over the region's area,
 * or of an intensity [mm/h].  Modes: EXACT adds or removes exactly dt S_h
 * (a removal larger than the cell's water after the fluxes is an error, -8);
 * AVAILABLE removes at most that water; INFINITY removes all of it.
 * Readings: "available water" is the depth after the flux update; a cell
 * emptied by a sink gets H = z exactly; added water carries no species,
 * removed water carries the cell's concentrations.
 * ------------------------------------------------------------------------ */
int om_sim_set_sources(om_sim *s, const int32_t *cell_src, int32_t nsrc, const int32_t *mode,
                       const int32_t *unit, const int32_t *npts, const double *t, const double *v, char *err,
                       int elen) {
    const om_mesh *m = s->m;
    for (int r = 0; r < s->nsrc; r++) { free(s->src[r].t); free(s->src[r].Q); }
    free(s->src); free(s->csrc); free(s->sfac);
    s->src = NULL; s->csrc = NULL; s->sfac = NULL; s->nsrc = 0;
    s->ssum = 0.0; s->scomp = 0.0;
    if (nsrc == 0) return 0;
    if (nsrc < 0 || !cell_src || !mode || !unit || !npts) { seterr(err, elen, "bad source list"); return -1; }
    s->src = calloc((size_t)nsrc, sizeof(om_bc));
    s->csrc = malloc(sizeof(int32_t) * (size_t)m->nc);
    s->sfac = malloc(sizeof(double) * (size_t)m->nc);
    if (!s->src || !s->csrc || !s->sfac) { seterr(err, elen, "out of memory"); return -1; }
    s->nsrc = nsrc;
    int64_t off = 0;
    for (int r = 0; r < nsrc; r++) {
        om_bc *B = &s->src[r];
        B->kind = mode[r];
        B->npts = npts[r];
        if (mode[r] < OM_SRC_EXACT || mode[r] > OM_SRC_INFINITY) { seterr(err, elen, "unknown source mode"); return -1; }
        if (unit[r] != OM_SRC_DISCHARGE && unit[r] != OM_SRC_INTENSITY) { seterr(err, elen, "unknown source unit"); return -1; }
        if (mode[r] != OM_SRC_INFINITY && (npts[r] < 1 || !t || !v)) { seterr(err, elen, "a source needs a series"); return -1; }
        if (npts[r] < 0) { seterr(err, elen, "bad source list"); return -1; }
        if (npts[r] > 0) {
            B->t = malloc(sizeof(double) * (size_t)npts[r]);
            B->Q = malloc(sizeof(double) * (size_t)npts[r]);
            if (!B->t || !B->Q) { seterr(err, elen, "out of memory"); return -1; }
            for (int k = 0; k < npts[r]; k++) {
                B->t[k] = t[off + k];
                B->Q[k] = v[off + k];
                if (!isfinite(B->t[k]) || !isfinite(B->Q[k])) { seterr(err, elen, "non-finite source series"); return -1; }
                if (k > 0 && !(B->t[k] > B->t[k - 1])) { seterr(err, elen, "source times must increase"); return -1; }
                if (mode[r] == OM_SRC_AVAILABLE && B->Q[k] > 0.0) { seterr(err, elen, "only exact sources add water"); return -1; }
            }
            off += npts[r];
        }
    }
    /* region areas summed in ascending order (independent of numbering) */
    double *ar = malloc(sizeof(double) * (size_t)(m->nc > 0 ? m->nc : 1));
    if (!ar) { seterr(err, elen, "out of memory"); return -1; }
    for (int r = 0; r < nsrc; r++) {
        int64_t k = 0;
        for (int64_t i = 0; i < m->nc; i++)
            if (cell_src[i] == r) ar[k++] = m->area[i];
        qsort(ar, (size_t)k, sizeof(double), cmp_double);
        double A = 0.0;
        for (int64_t j = 0; j < k; j++) A += ar[j];
        if (unit[r] == OM_SRC_DISCHARGE) {
            if (!(A > 0.0) && mode[r] != OM_SRC_INFINITY) { free(ar); seterr(err, elen, "empty source region"); return -1; }
            s->src[r].length = 1.0 / A;
        } else {
            s->src[r].length = 1.0 / 3.6e6;   /* mm/h -> m/s */
        }
    }
    free(ar);
    for (int64_t i = 0; i < m->nc; i++) {
        if (cell_src[i] < -1 || cell_src[i] >= nsrc) { seterr(err, elen, "source region out of range"); return -1; }
        s->csrc[i] = cell_src[i];
    }
    return 0;
}

double om_source_volume(const om_sim *s) { return s->ssum + s->scomp; }

/* Inflow "froude(discharge, Froude number)" (the supplementary feature
 * table's inflow options): the unit discharge q = Q / length enters with the
 * depth at which the flow has the given Froude number, u = Fr sqrt(g h) and
 * q = u h, so h = (q / (Fr sqrt(g)))^(2/3).  Returns 0 when Q <= 0 (wall). */
static int froude_ghost(const om_sim *s, const om_bc *B, double t, double *hg, double *ung, double *qin) {
    double Q = hydrograph(B, t);
    if (!(Q > 0)) return 0;
    double q = Q / B->length;
    double h = pow(q / (B->slope * sqrt(s->g)), 2.0 / 3.0);
    *hg = h;
    *ung = -q / h;
    if (qin) *qin = q;
    return 1;
}

/* Normal depth of a unit discharge q >= 0 under the cell's power-law
 * friction coefficient gn2 = g n^2 on the energy slope S (Manning's formula
 * q = h^(5/3) sqrt(S) / n solved for h). */
static double normal_depth(const om_sim *s, double gn2, double q, double S) {
    double n = sqrt(gn2 / s->g);
    return pow(n * q / sqrt(S), 0.6);
}

/* Outflow discharge per unit length of the imposed-discharge outflows, from
 * the surface H and bed z of the boundary cell:
 *  weir(crest elevation z_w, Poleni factor mu): Poleni's free-overflow law
 *  q = (2/3) mu sqrt(2g) d^(3/2) with the head d = H - max(z_w, z) (a crest
 *  below the cell's bed counts at the bed);
 *  h-Q relation: Q(H) from the table (linear, constant past its ends)
 *  spread over the boundary length.  Zero for a dry cell. */
static double imposed_outflow(const om_sim *s, const om_bc *B, double H, double z) {
    if (!(H - z > 0.0)) return 0.0;
    if (B->kind == OM_OUTFLOW_WEIR) {
        double crest = B->slope > z ? B->slope : z;
        double d = H - crest;
        if (!(d > 0.0)) return 0.0;
        return (2.0 / 3.0) * B->par * sqrt(2.0 * s->g) * (d * sqrt(d));
    }
    return hydrograph(B, H) / B->length;
}

/* ---------------------------------------------------------------------------
 * Morphodynamics (section "Morphodynamics": eq. exner; numerics: eq.
 * exnerupdateformula with the HLL sediment flux eq. exner_hll, speeds eq.
 * exner_wave_assign and eq. exner_wave_estimation; closures of Table
 * sedtransport_closure).  Synchronous-decoupled: the bed moves with the
 * hydrodynamic dt, from the state at t^n.  Readings:
 *  - Shields parameter theta = |u|^2 / (c_f^2 (s-1) g d_m) with the cell's
 *    friction closure (u_* = |u| / c_f); frictionless or dry cells (h <=
 *    h_min) and cells at their non-erodible bed carry no sediment;
 *  - the transport is aligned with the flow: q_B = Phi(|u|) u / |u|;
 *  - dq_B,n / dq_n is taken at fixed depth and fixed tangential velocity:
 *    (Phi'(|u|) cos^2 a + Phi(|u|) / |u| sin^2 a) / h, cos a = u_n / |u|;
 *  - walls carry no sediment; open hydrodynamic edges carry the cell's own
 *    normal transport (zero gradient of the bed and of the transport);
 *  - the water depth is kept when the bed moves (H += z^{n+1} - z^n);
 *  - a bed update below the non-erodible bed is clipped to it and the
 *    sediment volume so added is tallied;
 *  - when both HLL speeds vanish the flux is the mean of the two normal
 *    transports.
 * ------------------------------------------------------------------------ */
static double sed_K(double d, double srel, double g) { return sqrt((srel - 1.0) * g * d * d * d); }

/* transport magnitude Phi(|u|) and dPhi/d|u| at fixed depth */
static void sed_mag(int32_t clos, double alpha, double mexp, double thr, double d, double srel, double g,
                    double umag, double cf2, double *phi, double *dphi) {
    *phi = 0.0;
    *dphi = 0.0;
    if (!(umag > 0.0)) return;
    if (clos == OM_SED_GRASS) {
        double e = umag - thr;
        if (e > 0.0) {
            *phi = alpha * pow(e, mexp);
            *dphi = alpha * mexp * pow(e, mexp - 1.0);
        }
        return;
    }
    if (!(cf2 > 0.0)) return;
    double theta = umag * umag / (cf2 * ((srel - 1.0) * g * d));
    double K = sed_K(d, srel, g);
    if (clos == OM_SED_MPM) {
        double e = theta - thr;
        if (e > 0.0) {
            *phi = alpha * pow(e, mexp) * K;
            *dphi = alpha * mexp * pow(e, mexp - 1.0) * K * (2.0 * theta / umag);
        }
    } else {
        *phi = 0.05 * cf2 * pow(theta, 2.5) * K;
        *dphi = 5.0 * *phi / umag;
    }
}

/* Normal transport q_B.n, its derivative dq_B,n/dq_n and the two speeds
 * lambda_1 <= 0 <= lambda_2 of one cell for the unit normal (nx, ny). */
void om_sed_cell(int32_t clos, double alpha, double mexp, double thr, double d, double srel, double g, double h,
                 double u, double v, double cf2, double nx, double ny, double *qbn, double *D, double *l1,
                 double *l2) {
    double umag = sqrt(u * u + v * v);
    double phi, dphi;
    sed_mag(clos, alpha, mexp, thr, d, srel, g, umag, cf2, &phi, &dphi);
    double un = u * nx + v * ny;
    double dd = 0.0, qn = 0.0;
    if (phi > 0.0 && h > 0.0) {
        double ca = un / umag;
        qn = phi * ca;
        dd = (dphi * (ca * ca) + (phi / umag) * (1.0 - ca * ca)) / h;
    }
    double c = sqrt(g * (h > 0.0 ? h : 0.0));
    double a = un - c;
    double r = sqrt(a * a + 4.0 * dd * (c * c));
    *qbn = qn;
    *D = dd;
    *l1 = 0.5 * (a - r);
    *l2 = 0.5 * (a + r);
}

static double cell_cf2(const om_sim *s, int64_t i, double h) {
    double par = s->gn2[i];
    if (!(par > 0.0)) return 0.0;
    if (s->fkind == OM_MANNING || s->fkind == OM_STRICKLER) return cbrt(h) / par;  /* h^(1/3) / (g n^2) */
    double cf = om_friction_cf(s->fkind, par, h);
    return cf * cf;
}

static void sed_state(const om_sim *s, int64_t i, double nx, double ny, double *qbn, double *l1, double *l2) {
    double h = s->H[i] - s->z[i];
    double u = 0.0, v = 0.0, cf2 = 0.0;
    int moves = h > s->h_min && !(s->zfix && s->z[i] <= s->zfix[i]);
    if (h > s->h_min) { u = s->qx[i] / h; v = s->qy[i] / h; }
    if (moves) cf2 = cell_cf2(s, i, h);
    double D;
    om_sed_cell(moves ? s->sclos : OM_SED_MPM, moves ? s->salpha : 0.0, s->sm, s->sthr, s->sd, s->srel, s->g, h, u,
                v, moves ? cf2 : 0.0, nx, ny, qbn, &D, l1, l2);
}

/* Bed contributions of one edge (n from L to R, outward of L). */
static void sed_edge(om_sim *s, int32_t L, int32_t R, int kL, int kR, double l, double nx, double ny, int open,
                     double dt, double *bst, double *bstc) {
    double qL, l1L, l2L;
    sed_state(s, L, nx, ny, &qL, &l1L, &l2L);
    double q;
    if (R >= 0) {
        double qR, l1R, l2R;
        sed_state(s, R, nx, ny, &qR, &l1R, &l2R);
        double lm = l1L < l1R ? l1L : l1R;
        double lp = l2L > l2R ? l2L : l2R;
        if (lp > lm) q = (lp * qL - lm * qR + lp * lm * (s->z[R] - s->z[L])) / (lp - lm);
        else q = 0.5 * (qL + qR);
        s->bcont[3 * L + kL] = l * q;
        s->bcont[3 * R + kR] = -(l * q);
    } else {
        q = open ? qL : 0.0;
        s->bcont[3 * L + kL] = l * q;
        if (open) neumaier(bst, bstc, dt * (l * q));
    }
}

int om_sim_set_morpho(om_sim *s, int32_t clos, double alpha, double mexp, double thr, double d, double srel,
                      double porosity, const double *z_rel, char *err, int elen) {
    const om_mesh *m = s->m;
    free(s->zfix); free(s->bcont);
    s->zfix = NULL; s->bcont = NULL; s->morpho = 0;
    s->bvsum = s->bvcomp = s->bclip = s->bclipc = 0.0;
    if (clos < 0) return 0;
    if (clos > OM_SED_EH) { seterr(err, elen, "unknown sediment transport closure"); return -1; }
    if (!(alpha >= 0) || !isfinite(alpha) || !(mexp > 0) || !isfinite(mexp) || !(thr >= 0) || !isfinite(thr) ||
        !(d > 0) || !isfinite(d) || !(srel > 1) || !isfinite(srel) || !(porosity >= 0 && porosity < 1)) {
        seterr(err, elen, "bad sediment parameters"); return -1;
    }
    s->bcont = calloc((size_t)(3 * m->nc + 1), sizeof(double));
    if (!s->bcont) { seterr(err, elen, "out of memory"); return -1; }
    if (z_rel) {
        s->zfix = malloc(sizeof(double) * (size_t)(m->nc > 0 ? m->nc : 1));
        if (!s->zfix) { seterr(err, elen, "out of memory"); return -1; }
        for (int64_t i = 0; i < m->nc; i++) {
            if (!(z_rel[i] <= 0.0)) { seterr(err, elen, "the fixed bed lies at or below the bed (z_rel <= 0)"); return -1; }
            s->zfix[i] = s->z[i] + z_rel[i];
        }
    }
    s->sclos = clos; s->salpha = alpha; s->sm = mexp; s->sthr = thr; s->sd = d; s->srel = srel; s->spor = porosity;
    s->morpho = 1;
    return 0;
}

/* ---------------------------------------------------------------------------
 * Draining-time positivity limiter (an option that replaces the clip; the
 * paper is silent on positivity).  Reading of the draining-time idea for
 * explicit finite volumes: a cell can lose at most the water it holds in a
 * step, so every flux that leaves a cell acts only for that cell's draining
 * time T = h |Omega| / (sum of its outgoing mass fluxes l F_h), i.e. is
 * scaled by theta = min(1, T / dt); the three components scale together, so
 * a still lake (no mass flux) is untouched and the state stays well
 * balanced.  Depths then stay >= 0 up to rounding; the clip remains for that
 * rounding and is tallied as before.
 * ------------------------------------------------------------------------ */
int om_sim_set_drain(om_sim *s, int on, char *err, int elen) {
    free(s->theta); free(s->dout);
    s->theta = NULL; s->dout = NULL; s->drain = 0;
    if (!on) return 0;
    for (int64_t e = 0; e < s->m->ne; e++)
        if (s->m->eR[e] >= 0 && s->ebc[e] >= 0 && s->bc[s->ebc[e]].kind == OM_OUTFLOW_HQ) {
            seterr(err, elen, "internal h-Q relations and the draining-time limiter do not combine");
            return -1;
        }
    size_t nc = (size_t)(s->m->nc > 0 ? s->m->nc : 1);
    s->theta = malloc(sizeof(double) * nc);
    s->dout = calloc(3 * nc, sizeof(double));
    if (!s->theta || !s->dout) { seterr(err, elen, "out of memory"); return -1; }
    s->drain = 1;
    return 0;
}

/* Cell beds given per cell instead of the node means (a restart of a run
 * whose bed moved, or a bed stored at lower precision), with the surface
 * H per cell, or NULL to keep each cell's depth; a surface below its bed
 * is a dry cell (H = z), as in the initial conditions. */
int om_sim_set_bed(om_sim *s, const double *z, const double *H, char *err, int elen) {
    const int64_t nc = s->m->nc;
    for (int64_t i = 0; i < nc; i++)
        if (!isfinite(z[i]) || (H && !isfinite(H[i]))) { seterr(err, elen, "non-finite bed or surface"); return -1; }
    for (int64_t i = 0; i < nc; i++) {
        double Hn = H ? H[i] : z[i] + (s->H[i] - s->z[i]);
        s->H[i] = Hn > z[i] ? Hn : z[i];
        s->z[i] = z[i];
    }
    return 0;
}

void om_get_bed(const om_sim *s, double *z) { memcpy(z, s->z, sizeof(double) * (size_t)s->m->nc); }

/* Sediment volume (1 - p) sum z |Omega| (Neumaier), the volume that left
 * through open boundaries, and the volume the fixed-bed clip added: the
 * balance reads V(t) = V(0) - bnd + clipped. */
void om_morpho_diag(const om_sim *s, double *vol, double *bnd, double *clipped) {
    double sum = 0.0, comp = 0.0;
    for (int64_t i = 0; i < s->m->nc; i++) neumaier(&sum, &comp, (1.0 - s->spor) * s->z[i] * s->m->area[i]);
    if (vol) *vol = sum + comp;
    if (bnd) *bnd = s->bvsum + s->bvcomp;
    if (clipped) *clipped = s->bclip + s->bclipc;
}

/* Inflow "uniform(discharge, slope)" (section "Hydrodynamic BCs"): the given
 * discharge is spread over the boundary length; reading: the boundary state
 * carries the Manning normal depth for that unit discharge, q = h^{5/3}
 * sqrt(S) / n, flowing into the domain.  Returns 0 when Q <= 0 (edge acts as
 * a wall); *qin (may be NULL) receives q. */
static int inflow_ghost(const om_sim *s, const om_bc *B, int32_t cell, double t, double *hg, double *ung,
                        double *qin) {
    double Q = hydrograph(B, t);
    if (!(Q > 0)) return 0;
    double q = Q / B->length;
    double n = sqrt(s->gn2[cell] / s->g);
    double h = pow(n * q / sqrt(B->slope), 0.6);
    *hg = h;
    *ung = -q / h;   /* the normal points out of the domain */
    if (qin) *qin = q;
    return 1;
}

/* HLLC flux in the edge frame (Toro 1994; Toro 2001 ch. 10), for
 * reconstructed depths hL, hR >= 0, normal and tangential velocities.
 * Wave speeds: two-rarefaction estimates with the dry-bed forms; readings:
 * c_s is clamped at 0; ties at S = 0 resolve as listed below; identical
 * states return the physical flux and two dry sides return zero. */
void om_hllc(double hL, double unL, double utL, double hR, double unR, double utR, double g, double F[3]) {
    if (hL <= 0.0 && hR <= 0.0) { F[0] = 0.0; F[1] = 0.0; F[2] = 0.0; return; }
    if (hL == hR && unL == unR && utL == utR) {
        F[0] = hL * unL;
        F[1] = hL * unL * unL + 0.5 * g * hL * hL;
        F[2] = hL * unL * utL;
        return;
    }
    double cL = sqrt(g * hL), cR = sqrt(g * hR);
    double SL, SR;
    if (hL <= 0.0) {
        SL = unR - 2.0 * cR;
        SR = unR + cR;
    } else if (hR <= 0.0) {
        SL = unL - cL;
        SR = unL + 2.0 * cL;
    } else {
        double a = 0.5 * (cL + cR) + 0.25 * (unL - unR);
        double us = 0.5 * (unL + unR) + cL - cR;
        double cs = a > 0.0 ? a : 0.0;
        SL = fmin(unL - cL, us - cs);
        SR = fmax(unR + cR, us + cs);
    }
    double Ss = (SL * hR * (unR - SR) - SR * hL * (unL - SL)) / (hR * (unR - SR) - hL * (unL - SL));
    double FL[3] = {hL * unL, hL * unL * unL + 0.5 * g * hL * hL, hL * unL * utL};
    double FR[3] = {hR * unR, hR * unR * unR + 0.5 * g * hR * hR, hR * unR * utR};
    if (0.0 <= SL) {
        F[0] = FL[0]; F[1] = FL[1]; F[2] = FL[2];
    } else if (SR <= 0.0) {
        F[0] = FR[0]; F[1] = FR[1]; F[2] = FR[2];
    } else if (0.0 <= Ss) {
        double f = hL * (SL - unL) / (SL - Ss);
        F[0] = FL[0] + SL * (f - hL);
        F[1] = FL[1] + SL * (f * Ss - hL * unL);
        F[2] = FL[2] + SL * (f * utL - hL * utL);
    } else {
        double f = hR * (SR - unR) / (SR - Ss);
        F[0] = FR[0] + SR * (f - hR);
        F[1] = FR[1] + SR * (f * Ss - hR * unR);
        F[2] = FR[2] + SR * (f * utR - hR * utR);
    }
}

/* Friction split (eq. friction_closure with the Manning closure): the ODE
 * dq/dt = -g n^2 |q| q / h^{7/3} with h frozen has the exact one-step
 * solution q / (1 + dt g n^2 |q| / h^{7/3}).  Reading: this is the
 * semi-implicit integrator; thin films (h <= h_min) lose their discharge.
 * Returns the factor applied to q. */
double om_friction(double qabs, double h, double gn2, double dt, double h_min) {
    if (!(h > h_min)) return 0.0;
    return 1.0 / (1.0 + dt * gn2 * qabs / pow(h, 7.0 / 3.0));
}

/* Dimensionless friction coefficient c_f of the log-type closures of Table
 * friction_closure: Chezy (par = K_s) and Bezzola (par = y_R).  Reading: the
 * printed "log" is the natural logarithm, and the Chezy row is taken as
 * printed (6.25 + log(h/K_s) above K_s, 6.25 at or below). */
double om_friction_cf(int32_t kind, double par, double h) {
    if (kind == OM_CHEZY) return h > par ? 6.25 + log(h / par) : 6.25;
    double r = h / par;
    if (r > 2.0) return 2.5 * sqrt(1.0 - 1.0 / r) * log(10.9 * r);
    if (r >= 0.5) return 1.25 * sqrt(r) * log(10.9 * r);
    return 1.5;
}

/* Friction split for every closure of Table friction_closure.  With
 * S_f = u|u| / (g h c_f^2) (eq. friction_closure) the momentum sink is
 * g h S_f = |q| q / (h^2 c_f^2), so the exact one-step factor is
 * 1 / (1 + dt |q| / (h^2 c_f^2)); for the power-law closures (Manning,
 * Strickler: c_f^2 = h^{1/3} / (g n^2), n = 1/k_str) this is the Manning form
 * above.  par <= 0 means no friction. */
double om_friction_closure(int32_t kind, double par, double qabs, double h, double dt, double h_min) {
    if (kind == OM_MANNING || kind == OM_STRICKLER) return om_friction(qabs, h, par, dt, h_min);
    if (!(h > h_min)) return 0.0;
    if (!(par > 0)) return 1.0;
    double cf = om_friction_cf(kind, par, h);
    return 1.0 / (1.0 + dt * qabs / (h * h * cf * cf));
}

/* Selects the friction closure (Table friction_closure) and its per-cell
 * parameter: Manning n, Strickler k_str, Chezy K_s or Bezzola y_R (all >= 0;
 * 0 = frictionless).  The inflow ghost's normal depth has a closed form only
 * for the power-law closures, so inflow conditions require Manning or
 * Strickler (with a positive parameter on their cells). */
int om_sim_set_friction(om_sim *s, int32_t kind, const double *par, char *err, int elen) {
    const om_mesh *m = s->m;
    if (kind < OM_MANNING || kind > OM_BEZZOLA) { seterr(err, elen, "unknown friction closure"); return -1; }
    for (int64_t i = 0; i < m->nc; i++) {
        double p = par ? par[i] : 0.0;
        if (!(p >= 0) || !isfinite(p)) { seterr(err, elen, "negative or non-finite friction parameter"); return -1; }
        if (kind == OM_MANNING) s->gn2[i] = s->g * p * p;
        else if (kind == OM_STRICKLER) s->gn2[i] = p > 0 ? s->g / (p * p) : 0.0;
        else s->gn2[i] = p;
    }
    s->fkind = kind;
    for (int64_t e = 0; e < m->ne; e++) {
        if (s->ebc[e] < 0) continue;
        int k = s->bc[s->ebc[e]].kind;
        if (k != OM_INFLOW_UNIFORM && k != OM_OUTFLOW_UNIFORM) continue;
        if (kind == OM_CHEZY || kind == OM_BEZZOLA) {
            seterr(err, elen, "uniform inflow or outflow needs the Manning or Strickler closure"); return -1;
        }
        if (!(s->gn2[m->eL[e]] > 0)) { seterr(err, elen, "uniform inflow or outflow edge next to a frictionless cell"); return -1; }
    }
    return 0;
}

static void cell_velocity(const om_sim *s, int32_t i, double *h, double *u, double *v) {
    *h = s->H[i] - s->z[i];
    if (*h > s->h_min) { *u = s->qx[i] / *h; *v = s->qy[i] / *h; }
    else { *u = 0.0; *v = 0.0; }
}

/* eq. CFL_condition: dt = CFL min_i min_j rho_ij / (|u.n_ij| + sqrt(g h_i))
 * over wet cells; readings: inflow ghosts count with their own state on
 * their edge, dt is capped by the parameter dt_max and by t_end - t. */
double om_next_dt(const om_sim *s, double t_end) {
    const om_mesh *m = s->m;
    double best = INFINITY;
    /* the minimum does not depend on the order cells are visited in */
#pragma omp parallel for schedule(static) reduction(min : best)
    for (int64_t i = 0; i < m->nc; i++) {
        double h, u, v;
        cell_velocity(s, (int32_t)i, &h, &u, &v);
        if (!(h > s->h_min)) continue;
        double c = sqrt(s->g * h);
        for (int k = 0; k < 3; k++) {
            int32_t e = m->cell_edge[3 * i + k];
            double sg = (m->eL[e] == i) ? 1.0 : -1.0;
            double nx = sg * m->enx[e], ny = sg * m->eny[e];
            double un = u * nx + v * ny;
            double lam = fabs(un) + c;
            if (s->diff) {
                /* reading: the relaxation waves +-sqrt(K_nn / zeta) of the
                 * diffusing species bound the step too */
                double kt = 0.0, um2 = u * u + v * v, cf2 = cell_cf2(s, i, h);
                if (um2 > 0.0 && cf2 > 0.0) {
                    double a = h * sqrt(um2 / cf2), dd = (s->daL - s->daT) / um2;
                    kt = a * (s->daT + dd * (u * nx + v * ny) * (u * nx + v * ny));
                }
                double kmax = 0.0;
                for (int q = 0; q < s->ns; q++) kmax = s->dKm[q] > kmax ? s->dKm[q] : kmax;
                double lamd = fabs(un) + sqrt((kmax + kt) / s->dzeta);
                if (lamd > lam) lam = lamd;
            }
            double r = m->rho[3 * i + k] / lam;
            if (r < best) best = r;
        }
    }
    for (int64_t e = 0; e < m->ne; e++) {
        if (s->ebc[e] < 0) continue;
        const om_bc *B = &s->bc[s->ebc[e]];
        if (B->kind != OM_INFLOW_UNIFORM) continue;
        double hg, ung;
        if (!inflow_ghost(s, B, m->eL[e], s->t, &hg, &ung, NULL)) continue;
        double lam = fabs(ung) + sqrt(s->g * hg);
        double r = m->rho[3 * m->eL[e] + m->ekL[e]] / lam;
        if (r < best) best = r;
    }
    for (int64_t e = 0; e < m->ne; e++) {
        if (s->ebc[e] < 0) continue;
        const om_bc *B = &s->bc[s->ebc[e]];
        if (B->kind != OM_INFLOW_FROUDE) continue;
        double hg, ung;
        if (!froude_ghost(s, B, s->t, &hg, &ung, NULL)) continue;
        double lam = fabs(ung) + sqrt(s->g * hg);
        double r = m->rho[3 * m->eL[e] + m->ekL[e]] / lam;
        if (r < best) best = r;
    }
    /* z-hydrograph ghosts: still water, lambda = sqrt(g h_g) while wet */
    for (int64_t e = 0; e < m->ne; e++) {
        if (s->ebc[e] < 0) continue;
        const om_bc *B = &s->bc[s->ebc[e]];
        if (B->kind != OM_ZHYDROGRAPH) continue;
        double hg = hydrograph(B, s->t) - s->z[m->eL[e]];
        if (hg < OM_H_DRY) continue;
        double r = m->rho[3 * m->eL[e] + m->ekL[e]] / sqrt(s->g * hg);
        if (r < best) best = r;
    }
    double dt = s->cfl * best;
    if (s->dt_max < dt) dt = s->dt_max;
    if (t_end - s->t < dt) dt = t_end - s->t;
    return dt;
}


/* ---------------------------------------------------------------------------
 * Passive scalars (section "Scalar advection-diffusion": eq. scalar_goveq
 * without the diffusion tensor, and the update eq. scl:updateformula with
 * the advective fluxes A_ij only).  Per species c the specific mass
 * q_c = h phi_c.  Readings: the advective flux of an edge is the HLLC mass
 * flux F_h (the one the hydrodynamic update uses) times the concentration of
 * the cell the water leaves; phi = q/h in cells with water (q and h are
 * carried by the same mass flux, so thin films keep their concentration),
 * 0 in dry ones;
 * walls carry nothing, zero-gradient and prescribed-surface edges repeat the
 * interior concentration, inflow edges carry their condition's inflow
 * concentration; a cell left dry by the step (the water's positivity clip)
 * keeps no scalar, and the mass removed or added is tallied.  The diffusive
 * part (the relaxed SVT flux) is not built.
 * ------------------------------------------------------------------------ */
int om_sim_set_scalars(om_sim *s, int32_t ns, const double *phi0, const double *phi_in, char *err, int elen) {
    const om_mesh *m = s->m;
    int64_t nc = m->nc;
    if (ns < 0 || ns > OM_MAX_SPECIES) { seterr(err, elen, "between 0 and 5 species"); return -1; }
    free(s->sq); free(s->sphi); free(s->scont); free(s->phi_in);
    free(s->spsi); free(s->dK); free(s->dcont);
    s->spsi = s->dK = s->dcont = NULL;
    s->diff = 0;
    s->sq = calloc((size_t)(ns * nc + 1), sizeof(double));
    s->sphi = calloc((size_t)(ns * nc + 1), sizeof(double));
    s->scont = calloc((size_t)(3 * ns * nc + 1), sizeof(double));
    s->phi_in = calloc((size_t)(ns * (s->nbc > 0 ? s->nbc : 1) + 1), sizeof(double));
    if (!s->sq || !s->sphi || !s->scont || !s->phi_in) { seterr(err, elen, "out of memory"); return -1; }
    for (int c = 0; c < ns; c++) {
        for (int64_t i = 0; i < nc; i++) {
            double p = phi0 ? phi0[c * nc + i] : 0.0;
            if (!isfinite(p)) { seterr(err, elen, "non-finite initial concentration"); return -1; }
            double h = s->H[i] - s->z[i];
            s->sq[c * nc + i] = h > 0.0 ? h * p : 0.0;
        }
        for (int b = 0; b < s->nbc; b++) {
            double p = phi_in ? phi_in[b * ns + c] : 0.0;
            if (!isfinite(p)) { seterr(err, elen, "non-finite inflow concentration"); return -1; }
            s->phi_in[b * ns + c] = p;
        }
        s->sbsum[c] = 0.0; s->sbcomp[c] = 0.0;
        s->sclip[c] = 0.0; s->sclipc[c] = 0.0;
    }
    s->ns = ns;
    return 0;
}

void om_get_scalars(const om_sim *s, double *q) {
    if (q) memcpy(q, s->sq, (size_t)s->ns * (size_t)s->m->nc * sizeof(double));
}

/* Diffusion of the species (section "Scalar advection-diffusion"): the
 * Cattaneo-type relaxation of eq. relaxation_terms adds per species the
 * auxiliary variables psi = (psi_x, psi_y), which relax towards the gradient
 * of the concentration with relaxation time zeta; the species flux gains the
 * diffusive part -h K psi, and psi the flux -(phi / zeta) n (eq.
 * vecform_scalar2).  K = K^m I + K^t (section "Scalar advection-diffusion
 * closure relationships"): K^m per species, and the turbulent dispersion
 * scaled by the friction velocity u_* = |u| / c_f and the depth; reading
 * (the Elder form the two coefficients imply): K^t = h u_* (alpha_T I +
 * (alpha_L - alpha_T) u u^T / |u|^2), with c_f from the cell's friction
 * closure (none in frictionless cells).  Km (ns values >= 0), alpha_L,
 * alpha_T >= 0, zeta > 0; psi0 (ns x nc x 2, or NULL = 0) the initial
 * auxiliary variables.  Needs the species set first. */
int om_sim_set_diffusion(om_sim *s, const double *Km, double alpha_L, double alpha_T, double zeta,
                         const double *psi0, char *err, int elen) {
    const int64_t nc = s->m->nc;
    if (s->ns < 1) { seterr(err, elen, "diffusion needs species"); return -1; }
    if (!(zeta > 0.0) || !isfinite(zeta)) { seterr(err, elen, "the relaxation time must be positive"); return -1; }
    if (!(alpha_L >= 0.0) || !(alpha_T >= 0.0) || !isfinite(alpha_L) || !isfinite(alpha_T)) {
        seterr(err, elen, "dispersion coefficients must be >= 0"); return -1;
    }
    for (int c = 0; c < s->ns; c++)
        if (!(Km[c] >= 0.0) || !isfinite(Km[c])) { seterr(err, elen, "diffusivities must be >= 0"); return -1; }
    free(s->spsi); free(s->dK); free(s->dcont);
    s->spsi = calloc((size_t)(2 * s->ns * nc + 1), sizeof(double));
    s->dK = calloc((size_t)(4 * nc + 1), sizeof(double));
    s->dcont = calloc((size_t)(9 * s->ns * nc + 1), sizeof(double));
    if (!s->spsi || !s->dK || !s->dcont) { seterr(err, elen, "out of memory"); return -1; }
    if (psi0) {
        for (int64_t k = 0; k < 2 * s->ns * nc; k++) {
            if (!isfinite(psi0[k])) { seterr(err, elen, "non-finite auxiliary variable"); return -1; }
            s->spsi[k] = psi0[k];
        }
    }
    for (int c = 0; c < s->ns; c++) s->dKm[c] = Km[c];
    s->daL = alpha_L; s->daT = alpha_T; s->dzeta = zeta;
    s->diff = 1;
    return 0;
}

void om_get_psi(const om_sim *s, double *psi) {
    if (psi && s->diff) memcpy(psi, s->spsi, (size_t)2 * s->ns * (size_t)s->m->nc * sizeof(double));
}

/* Depth and turbulent dispersion tensor (h, Kxx, Kxy, Kyy) of every cell at
 * t^n; h = 0 marks a cell at or below h_min, which takes part in no
 * diffusive exchange. */
static void diffusion_cells(om_sim *s) {
    for (int64_t i = 0; i < s->m->nc; i++) {
        double *K = s->dK + 4 * i;
        double h = s->H[i] - s->z[i];
        K[0] = K[1] = K[2] = K[3] = 0.0;
        if (!(h > s->h_min)) continue;
        K[0] = h;
        double u = s->qx[i] / h, v = s->qy[i] / h;
        double um2 = u * u + v * v;
        double cf2 = cell_cf2(s, i, h);
        if (!(um2 > 0.0) || !(cf2 > 0.0)) continue;
        double us = sqrt(um2 / cf2);          /* u_* = |u| / c_f */
        double a = h * us;
        double d = (s->daL - s->daT) / um2;
        K[1] = a * (s->daT + d * u * u);
        K[2] = a * (d * u * v);
        K[3] = a * (s->daT + d * v * v);
    }
}

/* The interface flux of the relaxation system of species c on one side of
 * an edge that carries no diffusive exchange (a boundary, an internal wall,
 * or a neighbour at or below h_min), for a cell above h_min (cells at or
 * below it receive no contribution, and their psi is reset to zero by the
 * update): the mirrored ghost (phi, -psi_n, psi_t)
 * gives the exact two-wave solution psi_n* = 0 (no diffusive flux of the
 * species) and phi* = phi - sqrt(K_nn zeta) psi_n, where the species flux
 * vanishes and psi receives -(phi* / zeta) n.  (nx, ny) is the outward normal
 * of cell K. */
static void diffusion_mirror(const om_sim *s, int c, int32_t K, int kK, double l, double nx, double ny) {
    const int64_t nc = s->m->nc;
    const double *Kt = s->dK + 4 * K;
    if (!(Kt[0] > 0.0)) return;  /* a cell at or below h_min takes part in nothing */
    const double *ps = s->spsi + 2 * (c * nc + K);
    double knn = s->dKm[c] + (Kt[1] * nx * nx + 2.0 * Kt[2] * nx * ny + Kt[3] * ny * ny);
    double psn = ps[0] * nx + ps[1] * ny;
    double phs = s->sphi[c * nc + K] - sqrt(knn * s->dzeta) * psn;
    double *d = s->dcont + 9 * (c * nc + K) + 3 * kK;
    d[0] = 0.0;
    d[1] = l * (-(phs / s->dzeta) * nx);
    d[2] = l * (-(phs / s->dzeta) * ny);
}

/* Diffusive contributions of the edge e between L and R (n from L to R) for
 * every species: the exact solution of the linear two-wave Riemann problem
 * of the relaxation system in the edge's normal direction, with the
 * interface depth the smaller of the two reconstructed depths hLs, hRs of
 * the hydrodynamic flux (the wetted cross-section the edge shares; a cell
 * next to a much deeper one then cannot receive more than its own depth
 * carries, which keeps the update stable on thin layers) and the diffusion
 * tensor the mean of the two cells' (readings).  Waves +-sqrt(K_nn / zeta) carry the invariants
 * phi -+ sqrt(K_nn zeta) psi_n, so
 *   psi_n* = (psi_nL + psi_nR) / 2 + (phi_R - phi_L) / (2 sqrt(K_nn zeta)),
 *   phi*   = (phi_L + phi_R) / 2 + sqrt(K_nn zeta) (psi_nR - psi_nL) / 2,
 * and the edge carries D_q = -h (K_nn psi_n* + K_nt psi_t) (psi_t the mean
 * tangential component) and D_psi = -(phi* / zeta) n. */
static void diffusion_edge(om_sim *s, int64_t e, int32_t L, int32_t R, int kL, int kR, double l, double nx,
                           double ny, int closed, double hLs, double hRs) {
    const int64_t nc = s->m->nc;
    const double hi = hLs < hRs ? hLs : hRs;
    for (int c = 0; c < s->ns; c++) {
        const double *KL = s->dK + 4 * L;
        if (R < 0 || closed || !(KL[0] > 0.0) || !(s->dK[4 * R] > 0.0) || !(hi > 0.0)) {
            diffusion_mirror(s, c, L, kL, l, nx, ny);
            if (R >= 0) diffusion_mirror(s, c, R, kR, l, -nx, -ny);
            continue;
        }
        const double *KR = s->dK + 4 * R;
        double h = hi;
        double kxx = s->dKm[c] + 0.5 * (KL[1] + KR[1]);
        double kxy = 0.5 * (KL[2] + KR[2]);
        double kyy = s->dKm[c] + 0.5 * (KL[3] + KR[3]);
        double knn = kxx * nx * nx + 2.0 * kxy * nx * ny + kyy * ny * ny;
        double knt = -kxx * nx * ny + kxy * (nx * nx - ny * ny) + kyy * nx * ny;
        const double *pL = s->spsi + 2 * (c * nc + L), *pR = s->spsi + 2 * (c * nc + R);
        double pnL = pL[0] * nx + pL[1] * ny, pnR = pR[0] * nx + pR[1] * ny;
        double ptL = -pL[0] * ny + pL[1] * nx, ptR = -pR[0] * ny + pR[1] * nx;
        double fL = s->sphi[c * nc + L], fR = s->sphi[c * nc + R];
        double Dq, fs;
        if (knn > 0.0) {
            double r = sqrt(knn * s->dzeta);
            double pns = 0.5 * (pnL + pnR) + (fR - fL) / (2.0 * r);
            fs = 0.5 * (fL + fR) + 0.5 * r * (pnR - pnL);
            Dq = -h * (knn * pns + knt * (0.5 * (ptL + ptR)));
        } else {
            fs = 0.5 * (fL + fR);
            Dq = 0.0;
        }
        double Dx = -(fs / s->dzeta) * nx, Dy = -(fs / s->dzeta) * ny;
        double *dL = s->dcont + 9 * (c * nc + L) + 3 * kL;
        double *dR = s->dcont + 9 * (c * nc + R) + 3 * kR;
        dL[0] = l * Dq; dL[1] = l * Dx; dL[2] = l * Dy;
        dR[0] = -(l * Dq); dR[1] = -(l * Dx); dR[2] = -(l * Dy);
    }
    (void)e;
}

/* per species: total mass sum q_c |Omega|, the time integral of the mass
 * flux leaving through open boundaries, and the mass added by resetting
 * cells left dry (mass(t) = mass(0) - bnd + clipped) */
void om_scalar_diag(const om_sim *s, double *mass, double *bnd, double *clipped) {
    for (int c = 0; c < s->ns; c++) {
        double sum = 0.0, comp = 0.0;
        for (int64_t i = 0; i < s->m->nc; i++) neumaier(&sum, &comp, s->sq[c * s->m->nc + i] * s->m->area[i]);
        if (mass) mass[c] = sum + comp;
        if (bnd) bnd[c] = s->sbsum[c] + s->sbcomp[c];
        if (clipped) clipped[c] = s->sclip[c] + s->sclipc[c];
    }
}

/* Scalar contributions of one edge for every species.  R < 0: a boundary
 * edge; `wall` and `inflow_b` (index of an active inflow condition, or -1)
 * describe its ghost. */
static void scalar_edge(om_sim *s, int32_t L, int32_t R, int kL, int kR, double l, double F0, int wall,
                        int inflow_b, int open, double dt, double *bst, double *bstc) {
    const int64_t nc = s->m->nc;
    for (int c = 0; c < s->ns; c++) {
        const double *ph = s->sphi + c * nc;
        double phL = ph[L], phR;
        if (R >= 0) phR = ph[R];
        else if (wall) phR = phL;
        else if (inflow_b >= 0) phR = s->phi_in[inflow_b * s->ns + c];
        else phR = phL;
        double A = F0 * (F0 >= 0.0 ? phL : phR);
        s->scont[3 * (c * nc + L) + kL] = l * A;
        if (R >= 0) s->scont[3 * (c * nc + R) + kR] = -(l * A);
        else if (open) neumaier(&bst[c], &bstc[c], dt * (l * A));
    }
}

/* The numerical flux of edge e (HLLC, or a boundary condition's ghost or
 * imposed discharge) at t^n, in the edge's frame (n from L to R), with the
 * reconstructed depths on its two sides. */
typedef struct {
    double F[3];
    double hLs, hRs;
    int wall, open, inflow_b;
} edge_flux_t;

/* A dynamic wall (section "Hydrodynamic BCs": it collapses at a given time
 * or at a given water depth) stands before its collapse time and,
 * with a collapse depth, before the end of the first step that started with
 * a cell next to it at that depth (reading: the wall holds through that
 * step and is gone from the next; dynamic_wall_depths sets the time). */
static int wall_stands(const om_sim *s, const om_bc *B) {
    return s->t < B->slope && s->t < B->gone;
}

/* An interior edge that is a standing internal wall (a static wall, or a
 * standing dynamic wall). */
static int internal_wall(const om_sim *s, int64_t e) {
    if (s->m->eR[e] < 0 || s->ebc[e] < 0) return 0;
    const om_bc *B = &s->bc[s->ebc[e]];
    return B->kind == OM_WALL || (B->kind == OM_DYNAMIC_WALL && wall_stands(s, B));
}

/* Dynamic walls with a collapse depth: one that stands at t^n with a cell on
 * either side of one of its edges (the one cell of a boundary edge) at or
 * above that depth h = H - z is gone from t^n + dt on. */
static void dynamic_wall_depths(om_sim *s, double dt) {
    const om_mesh *m = s->m;
    for (int64_t e = 0; e < m->ne; e++) {
        if (s->ebc[e] < 0) continue;
        om_bc *B = &s->bc[s->ebc[e]];
        if (B->kind != OM_DYNAMIC_WALL || !(B->par > 0.0) || !wall_stands(s, B)) continue;
        const int32_t L = m->eL[e], R = m->eR[e];
        if (s->H[L] - s->z[L] >= B->par || (R >= 0 && s->H[R] - s->z[R] >= B->par)) B->gone = s->t + dt;
    }
}

/* An interior edge that carries an internal rating curve. */
static int internal_hq(const om_sim *s, int64_t e) {
    return s->m->eR[e] >= 0 && s->ebc[e] >= 0 && s->bc[s->ebc[e]].kind == OM_OUTFLOW_HQ;
}

/* One side K of an internal wall, with K's outward normal (nx, ny): the
 * reflective wall flux of K's own state, as on the domain boundary. */
static void wall_side(om_sim *s, int32_t K, int kK, double nx, double ny, double l) {
    double hK, uK, vK;
    cell_velocity(s, K, &hK, &uK, &vK);
    double un = uK * nx + vK * ny, ut = -uK * ny + vK * nx;
    double hs = s->H[K] - s->z[K];
    if (hs < OM_H_DRY) hs = 0.0;
    double F[3];
    om_hllc(hs, un, ut, hs, -un, ut, s->g, F);
    F[0] = 0.0;
    double P = 0.5 * s->g * hs * hs;
    double dn = F[1] - P;
    s->cont[9 * K + 3 * kK + 0] = l * F[0];
    s->cont[9 * K + 3 * kK + 1] = l * (dn * nx - F[2] * ny);
    s->cont[9 * K + 3 * kK + 2] = l * (dn * ny + F[2] * nx);
    for (int c = 0; c < s->ns; c++) s->scont[3 * (c * s->m->nc + K) + kK] = 0.0;
    if (s->diff)
        for (int c = 0; c < s->ns; c++) diffusion_mirror(s, c, K, kK, l, nx, ny);
    if (s->morpho) s->bcont[3 * K + kK] = 0.0;
}

/* An internal rating curve (section "Hydrodynamic BCs", internal BCs; the
 * upstream side, where the table acts, is the one left of the tag's
 * segments): the table's discharge at the upstream cell's surface,
 * q = Q(H_U) / (the curve's length), crosses the edge from the cell U on the
 * left of the tag's segment to the other cell D.  U's side is the imposed
 * outflow of its own state, F = (q, q^2/h + g h^2/2, q u_t); D's side is the
 * wall flux of its own state with the mass flux -q; the species cross with
 * U's concentrations; neither sediment nor diffusion crosses. */
static void hq_edge(om_sim *s, int64_t e) {
    const om_mesh *m = s->m;
    const int up = m->eup[e];
    const int32_t U = up ? m->eL[e] : m->eR[e], D = up ? m->eR[e] : m->eL[e];
    const int kU = up ? m->ekL[e] : m->ekR[e], kD = up ? m->ekR[e] : m->ekL[e];
    const double sg = up ? 1.0 : -1.0;   /* U's outward normal is sg n */
    const double nx = sg * m->enx[e], ny = sg * m->eny[e], l = m->elen[e];
    const double q = imposed_outflow(s, &s->bc[s->ebc[e]], s->H[U], s->z[U]);
    double hU, uU, vU;
    cell_velocity(s, U, &hU, &uU, &vU);
    double utU = -uU * ny + vU * nx;
    double hs = s->H[U] - s->z[U];
    if (hs < OM_H_DRY) hs = 0.0;
    double F1 = (hs > 0.0 ? q * (q / hs) : 0.0) + 0.5 * s->g * hs * hs;
    double F2 = q * utU;
    double dn = F1 - 0.5 * s->g * hs * hs;
    s->cont[9 * U + 3 * kU + 0] = l * q;
    s->cont[9 * U + 3 * kU + 1] = l * (dn * nx - F2 * ny);
    s->cont[9 * U + 3 * kU + 2] = l * (dn * ny + F2 * nx);
    wall_side(s, D, kD, -nx, -ny, l);
    s->cont[9 * D + 3 * kD + 0] = -(l * q);
    const int64_t nc = m->nc;
    for (int c = 0; c < s->ns; c++) {
        double A = q * s->sphi[c * nc + U];
        s->scont[3 * (c * nc + U) + kU] = l * A;
        s->scont[3 * (c * nc + D) + kD] = -(l * A);
    }
    if (s->diff)
        for (int c = 0; c < s->ns; c++) diffusion_mirror(s, c, U, kU, l, nx, ny);
    if (s->morpho) s->bcont[3 * U + kU] = 0.0;
}

static void edge_flux(const om_sim *s, int64_t e, edge_flux_t *out) {
    const om_mesh *m = s->m;
    const double g = s->g;
    int32_t L = m->eL[e], R = m->eR[e];
    double nx = m->enx[e], ny = m->eny[e], l = m->elen[e];
    double hL, uL, vL, hR, uR, vR;
    cell_velocity(s, L, &hL, &uL, &vL);
    double HL = s->H[L], zL = s->z[L];
    double unL = uL * nx + vL * ny, utL = -uL * ny + vL * nx;
    double HR, zR, unR, utR;
    int wall = 0, open = 0, inflow_b = -1, imposed = 0;
    double qin = 0.0;  /* an active inflow's unit discharge */
    if (R >= 0) {
        cell_velocity(s, R, &hR, &uR, &vR);
        HR = s->H[R]; zR = s->z[R];
        unR = uR * nx + vR * ny; utR = -uR * ny + vR * nx;
    } else {
        int b = s->ebc[e];
        const om_bc *B = b >= 0 ? &s->bc[b] : NULL;
        double hg, ung;
        zR = zL;
        if (B && B->kind == OM_OUTFLOW_ZEROGRAD) {
            /* transmissive: the ghost repeats the interior state */
            HR = HL; unR = unL; utR = utL; open = 1;
        } else if (B && B->kind == OM_INFLOW_UNIFORM && inflow_ghost(s, B, L, s->t, &hg, &ung, &qin)) {
            HR = zL + hg; unR = ung; utR = 0.0; open = 1; inflow_b = b;
        } else if (B && B->kind == OM_INFLOW_FROUDE && froude_ghost(s, B, s->t, &hg, &ung, &qin)) {
            HR = zL + hg; unR = ung; utR = 0.0; open = 1; inflow_b = b;
        } else if (B && B->kind == OM_OUTFLOW_UNIFORM) {
            /* uniform(slope) outflow: the ghost carries the normal depth
             * of the cell's outflowing unit discharge with the cell's
             * velocity (reading: the paper asks for a depth at outflows
             * without saying which; no outflow gives a dry ghost) */
            double qn = hL * unL;
            hg = normal_depth(s, s->gn2[L], qn > 0.0 ? qn : 0.0, B->slope);
            HR = zL + hg; unR = unL; utR = utL; open = 1;
        } else if (B && (B->kind == OM_OUTFLOW_WEIR || B->kind == OM_OUTFLOW_HQ)) {
            HR = HL; unR = unL; utR = utL; open = 1; imposed = 1;
        } else if (B && B->kind == OM_DYNAMIC_WALL && !wall_stands(s, B)) {
            /* a dynamic wall once it is gone: transmissive */
            HR = HL; unR = unL; utR = utL; open = 1;
        } else if (B && B->kind == OM_ZHYDROGRAPH) {
            /* "zhydrograph" (section "Hydrodynamic BCs", water surface
             * elevation series).  Reading: the ghost is still water at the
             * prescribed surface over the cell's bed, like a reservoir or
             * sea level; the flux then lets water in or out. */
            HR = hydrograph(B, s->t); unR = 0.0; utR = 0.0; open = 1;
        } else {
            /* reflective wall: mirror the normal velocity */
            HR = HL; unR = -unL; utR = utL; wall = 1;
        }
    }
    /* hydrostatic reconstruction of modified states at the edge.
     * Reading: a reconstructed depth under OM_H_DRY counts as dry, so the
     * contact speed never divides two underflowed products; a dry side
     * never loses mass, so this keeps depths non-negative. */
    double zs = zL > zR ? zL : zR;
    double hLs = HL - zs; if (hLs < OM_H_DRY) hLs = 0.0;
    double hRs = HR - zs; if (hRs < OM_H_DRY) hRs = 0.0;
    double F[3];
    if (imposed) {
        /* weir or h-Q outflow: the boundary discharge q leaves carrying
         * the cell's state: F = (q, q^2/h + g h^2/2, q u_t) */
        double q = imposed_outflow(s, &s->bc[s->ebc[e]], HL, zL);
        F[0] = q;
        F[1] = (hLs > 0.0 ? q * (q / hLs) : 0.0) + 0.5 * g * hLs * hLs;
        F[2] = q * utL;
    } else {
        om_hllc(hLs, unL, utL, hRs, unR, utR, g, F);
    }
    if (inflow_b >= 0) {
        /* an inflow imposes its discharge (section "Hydrodynamic BCs": the
         * inflow condition is set from the given discharge).  Reading: the
         * edge's mass flux is the unit discharge q itself, the momentum
         * flux that of the Riemann problem between the cell and the
         * boundary state above; the volume that enters is then the
         * hydrograph's in sub- and supercritical flow alike, and uniform
         * flow at the boundary state stays in equilibrium */
        F[0] = -qin;
    }
    if (wall) F[0] = 0.0;   /* impermeable: no mass crosses a wall */
    out->F[0] = F[0]; out->F[1] = F[1]; out->F[2] = F[2];
    out->hLs = hLs; out->hRs = hRs;
    out->wall = wall; out->open = open; out->inflow_b = inflow_b;
}

int om_step(om_sim *s, double t_end, double *dt_taken) {
    const om_mesh *m = s->m;
    const double g = s->g;
    double dt = om_next_dt(s, t_end);
    if (dt_taken) *dt_taken = dt;
    if (!(dt > 0.0) || !isfinite(dt)) return -7;
    dynamic_wall_depths(s, dt);
    memset(s->cont, 0, sizeof(double) * 9 * (size_t)m->nc);
    double bstep = 0.0, bstepc = 0.0;
    int deficit = 0;   /* an exact sink asked for more water than a cell held */
    double bvst = 0.0, bvstc = 0.0;   /* sediment leaving through open boundaries this step */
    double sbst[OM_MAX_SPECIES] = {0}, sbstc[OM_MAX_SPECIES] = {0};
    for (int c = 0; c < s->ns; c++) {
        /* concentrations of the state at t^n (zero in dry cells) */
        for (int64_t i = 0; i < m->nc; i++) {
            double h = s->H[i] - s->z[i];
            s->sphi[c * m->nc + i] = h > 0.0 ? s->sq[c * m->nc + i] / h : 0.0;
        }
    }
    if (s->ns > 0) memset(s->scont, 0, sizeof(double) * 3 * (size_t)(s->ns * m->nc));
    if (s->diff) {
        diffusion_cells(s);
        memset(s->dcont, 0, sizeof(double) * 9 * (size_t)(s->ns * m->nc));
    }
    if (s->drain) {
        /* draining time: the water each cell loses through its edges this
         * step, summed in local edge order, against the water it holds */
        for (int64_t e = 0; e < m->ne; e++) {
            if (internal_wall(s, e)) {
                s->dout[3 * m->eL[e] + m->ekL[e]] = 0.0;
                s->dout[3 * m->eR[e] + m->ekR[e]] = 0.0;
                continue;
            }
            edge_flux_t ef;
            edge_flux(s, e, &ef);
            double l = m->elen[e];
            s->dout[3 * m->eL[e] + m->ekL[e]] = l * ef.F[0];
            if (m->eR[e] >= 0) s->dout[3 * m->eR[e] + m->ekR[e]] = -(l * ef.F[0]);
        }
        for (int64_t i = 0; i < m->nc; i++) {
            const double *o = s->dout + 3 * i;
            double out = (o[0] > 0.0 ? o[0] : 0.0) + (o[1] > 0.0 ? o[1] : 0.0) + (o[2] > 0.0 ? o[2] : 0.0);
            double h = s->H[i] - s->z[i];
            double vol = (h > 0.0 ? h : 0.0) * m->area[i];
            double leave = out * dt;
            s->theta[i] = leave > vol ? vol / leave : 1.0;
        }
    }
    /* every edge writes only its own two contribution slots, so the edge
     * loop may run in any order; the species and sediment passes accumulate
     * per edge and stay serial */
    const int par_edges = s->ns == 0 && !s->morpho;
#pragma omp parallel for schedule(static) if (par_edges)
    for (int64_t e = 0; e < m->ne; e++) {
        int32_t L = m->eL[e], R = m->eR[e];
        double nx = m->enx[e], ny = m->eny[e], l = m->elen[e];
        s->eflag[e] = 0;
        if (internal_wall(s, e)) {
            /* each side sees a wall: its own reflected state */
            wall_side(s, L, m->ekL[e], nx, ny, l);
            wall_side(s, R, m->ekR[e], -nx, -ny, l);
            continue;
        }
        if (internal_hq(s, e)) {
            hq_edge(s, e);
            continue;
        }
        edge_flux_t ef;
        edge_flux(s, e, &ef);
        double F[3] = {ef.F[0], ef.F[1], ef.F[2]};
        double hLs = ef.hLs, hRs = ef.hRs;
        int wall = ef.wall, open = ef.open, inflow_b = ef.inflow_b;
        if (s->drain) {
            /* the flux leaves its upwind cell for at most that cell's
             * draining time: scaled by theta of the cell the water leaves */
            double th = F[0] > 0.0 ? s->theta[L] : (F[0] < 0.0 && R >= 0 ? s->theta[R] : 1.0);
            F[0] = F[0] * th;
            F[1] = F[1] * th;
            F[2] = F[2] * th;
        }
        /* fluctuations: the flux minus each side's own reconstructed pressure
         * (the bed-slope source in well-balanced form, using sum_j l n = 0) */
        double PL = 0.5 * g * hLs * hLs, PR = 0.5 * g * hRs * hRs;
        double dLn = F[1] - PL, dRn = F[1] - PR;
        double cL0 = l * F[0];
        double cLx = l * (dLn * nx - F[2] * ny);
        double cLy = l * (dLn * ny + F[2] * nx);
        int kL = m->ekL[e];
        s->cont[9 * L + 3 * kL + 0] = cL0;
        s->cont[9 * L + 3 * kL + 1] = cLx;
        s->cont[9 * L + 3 * kL + 2] = cLy;
        if (R >= 0) {
            int kR = m->ekR[e];
            s->cont[9 * R + 3 * kR + 0] = -(l * F[0]);
            s->cont[9 * R + 3 * kR + 1] = -(l * (dRn * nx - F[2] * ny));
            s->cont[9 * R + 3 * kR + 2] = -(l * (dRn * ny + F[2] * nx));
        } else if (open) {
            s->ebvol[e] = dt * cL0;
            s->eflag[e] = 1;
        }
        if (s->ns > 0)
            scalar_edge(s, L, R, kL, R >= 0 ? m->ekR[e] : 0, l, F[0], wall, inflow_b, open, dt, sbst, sbstc);
        if (s->diff) diffusion_edge(s, e, L, R, kL, R >= 0 ? m->ekR[e] : 0, l, nx, ny, R < 0, hLs, hRs);
        if (s->morpho)
            sed_edge(s, L, R, kL, R >= 0 ? m->ekR[e] : 0, l, nx, ny, open, dt, &bvst, &bvstc);
    }
    /* volume through open boundary edges this step, in edge order, in
     * total and per boundary condition */
    for (int64_t e = 0; e < m->ne; e++)
        if (s->eflag[e]) {
            neumaier(&bstep, &bstepc, s->ebvol[e]);
            double *a = s->bcsum + 2 * s->ebc[e];
            neumaier(&a[0], &a[1], s->ebvol[e]);
        }
    int nonfinite = 0;
#pragma omp parallel for schedule(static) reduction(| : nonfinite, deficit)
    for (int64_t i = 0; i < m->nc; i++) {
        const double *c = &s->cont[9 * i];
        unsigned char flag = 0;
        double Rh = c[0] + c[3] + c[6];
        double Rx = c[1] + c[4] + c[7];
        double Ry = c[2] + c[5] + c[8];
        double w = dt * (1.0 / m->area[i]);
        double H = s->H[i] - w * Rh;
        double qx = s->qx[i] - w * Rx;
        double qy = s->qy[i] - w * Ry;
        if (s->csrc && s->csrc[i] >= 0) {
            /* external source or sink, explicit in the continuity equation */
            const om_bc *B = &s->src[s->csrc[i]];
            double hf = H - s->z[i];
            double avail = hf > 0.0 ? hf : 0.0;
            double dh;
            int empty = 0;
            if (B->kind == OM_SRC_INFINITY) {
                dh = -avail;
                empty = 1;
            } else {
                dh = dt * (hydrograph(B, s->t) * B->length);
                if (dh < -avail) {
                    if (B->kind == OM_SRC_AVAILABLE) { dh = -avail; empty = 1; }
                    else deficit = 1;
                }
            }
            if (empty) { if (avail > 0.0) H = s->z[i]; }
            else H = H + dh;
            s->csrcv[i] = dh * m->area[i];
            flag |= 1;
            double hn = H - s->z[i];
            s->sfac[i] = (dh < 0.0 && hf > 0.0) ? (hn > 0.0 ? hn / hf : 0.0) : 1.0;
        }
        double h = H - s->z[i];
        double f = om_friction_closure(s->fkind, s->gn2[i], sqrt(qx * qx + qy * qy), h, dt, s->h_min);
        qx = qx * f;
        qy = qy * f;
        if (h < 0.0) {
            /* positivity: the scheme's CFL does not bound the outflow of a
             * cell draining through several edges; clip and account for it */
            s->cclip[i] = -h * m->area[i];
            flag |= 2;
            H = s->z[i];
            qx = 0.0; qy = 0.0;
        }
        if (!isfinite(H) || !isfinite(qx) || !isfinite(qy)) nonfinite = 1;
        s->cflag[i] = flag;
        s->H[i] = H; s->qx[i] = qx; s->qy[i] = qy;
    }
    /* the sources' and the clip's volumes, each summed in cell order */
    for (int64_t i = 0; i < m->nc; i++)
        if (s->cflag[i] & 1) neumaier(&s->ssum, &s->scomp, s->csrcv[i]);
    for (int64_t i = 0; i < m->nc; i++)
        if (s->cflag[i] & 2) neumaier(&s->clip, &s->clipc, s->cclip[i]);
    if (nonfinite) return -4;
    for (int c = 0; c < s->ns; c++) {
        /* eq. scl:updateformula: the advective fluxes, plus the diffusive
         * ones and the relaxation of the auxiliary variables (its stiff
         * source -psi/zeta by the locally implicit Euler step) when the
         * species diffuse */
        double *q = s->sq + c * m->nc;
        for (int64_t i = 0; i < m->nc; i++) {
            const double *k = s->scont + 3 * (c * m->nc + i);
            double w = dt * (1.0 / m->area[i]);
            double Rq;
            if (s->diff) {
                const double *d = s->dcont + 9 * (c * m->nc + i);
                Rq = (k[0] + d[0]) + (k[1] + d[3]) + (k[2] + d[6]);
                double Rx = d[1] + d[4] + d[7];
                double Ry = d[2] + d[5] + d[8];
                double *ps = s->spsi + 2 * (c * m->nc + i);
                double rel = 1.0 + dt / s->dzeta;
                ps[0] = (ps[0] - w * Rx) / rel;
                ps[1] = (ps[1] - w * Ry) / rel;
                /* psi of a cell that took part in no exchange (at or below
                 * h_min at t^n), or that the step left dry, is reset */
                if (!(s->dK[4 * i] > 0.0) || !(s->H[i] - s->z[i] > 0.0)) { ps[0] = 0.0; ps[1] = 0.0; }
                if (!isfinite(ps[0]) || !isfinite(ps[1])) return -4;
            } else {
                Rq = k[0] + k[1] + k[2];
            }
            q[i] = q[i] - w * Rq;
            if (s->csrc && s->csrc[i] >= 0) q[i] = q[i] * s->sfac[i];
            /* a cell left without water keeps no scalar (the positivity
             * clip of the water, step 6, is mirrored here and tallied) */
            if (!(s->H[i] - s->z[i] > 0.0)) {
                neumaier(&s->sclip[c], &s->sclipc[c], -q[i] * m->area[i]);
                q[i] = 0.0;
            }
            if (!isfinite(q[i])) return -4;
        }
        neumaier(&s->sbsum[c], &s->sbcomp[c], sbst[c] + sbstc[c]);
    }
    neumaier(&s->bsum, &s->bcomp, bstep + bstepc);
    if (s->morpho) {
        /* eq. exnerupdateformula; the water depth is kept as the bed moves */
        for (int64_t i = 0; i < m->nc; i++) {
            const double *k = s->bcont + 3 * i;
            double Rz = k[0] + k[1] + k[2];
            double w = dt * (1.0 / m->area[i]);
            double zn = s->z[i] - (w * Rz) / (1.0 - s->spor);
            if (s->zfix && zn < s->zfix[i]) {
                neumaier(&s->bclip, &s->bclipc, (1.0 - s->spor) * (s->zfix[i] - zn) * m->area[i]);
                zn = s->zfix[i];
            }
            s->H[i] = s->H[i] + (zn - s->z[i]);
            s->z[i] = zn;
        }
        neumaier(&s->bvsum, &s->bvcomp, bvst + bvstc);
    }
    s->t += dt;
    s->steps++;
    return deficit ? -8 : 0;
}

/* Threads the OpenMP build uses (n > 0 sets them); 1 in the serial build. */
int om_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

int om_run_until(om_sim *s, double t_end, int64_t max_steps, int64_t *n_steps) {
    int64_t n = 0;
    int rc = 0;
    while (s->t < t_end && (max_steps <= 0 || n < max_steps)) {
        double dt;
        rc = om_step(s, t_end, &dt);
        if (rc) break;
        n++;
    }
    if (n_steps) *n_steps = n;
    return rc;
}

void om_get_state(const om_sim *s, double *H, double *qx, double *qy, double *t) {
    int64_t nc = s->m->nc;
    if (H) memcpy(H, s->H, sizeof(double) * nc);
    if (qx) memcpy(qx, s->qx, sizeof(double) * nc);
    if (qy) memcpy(qy, s->qy, sizeof(double) * nc);
    if (t) *t = s->t;
}

void om_set_state(om_sim *s, const double *H, const double *qx, const double *qy, double t) {
    int64_t nc = s->m->nc;
    memcpy(s->H, H, sizeof(double) * nc);
    memcpy(s->qx, qx, sizeof(double) * nc);
    memcpy(s->qy, qy, sizeof(double) * nc);
    s->t = t;
}

/* Diagnostics: volume M = sum (H - z)|Omega| (Neumaier), the integral of
 * the mass flux leaving through open boundaries, and the clipped volume.
 * The scheme is conservative: M(t) = M(0) - bnd_flux + clipped. */
void om_diag(const om_sim *s, double *mass, double *bnd, double *clipped, int64_t *steps) {
    double sum = 0.0, comp = 0.0;
    for (int64_t i = 0; i < s->m->nc; i++)
        neumaier(&sum, &comp, (s->H[i] - s->z[i]) * s->m->area[i]);
    if (mass) *mass = sum + comp;
    if (bnd) *bnd = s->bsum + s->bcomp;
    if (clipped) *clipped = s->clip + s->clipc;
    if (steps) *steps = s->steps;
}

/* The part of the boundary-flux integral that crossed the edges of boundary
 * condition b (positive: left the domain); 0 for an index out of range. */
double om_bc_flux(const om_sim *s, int32_t b) {
    if (b < 0 || b >= s->nbc) return 0.0;
    return s->bcsum[2 * b] + s->bcsum[2 * b + 1];
}
