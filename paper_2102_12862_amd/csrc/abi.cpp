// C ABI of the shallow-water library (declared in include/swe.h): handles,
// device layout, hipGraph-captured stepping, diagnostics, autotuning and
// batched ensembles.  Host code only: every step of the method runs in the
// kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "meshprep.h"
#include "swe.h"
#include "swe_internal.h"

using namespace swe;

static_assert(NBR_FLIP == NBR_FLIP_BIT, "flip bit");

namespace {

thread_local std::string g_err;

swe_status fail(swe_status code, const std::string &msg) {
    g_err = msg;
    return code;
}

// The FP32 surface's 16-bit low part, as the kernels code it: the rest
// H - hi in units of 2^(e-40) for hi = m 2^e, m in [1/2, 1) (2^-16 of an
// ulp of hi), rounded to nearest and clamped to the int16 range.
int16_t lo_code_host(float hi, double rest) {
    int e = 0;
    (void)std::frexp(hi, &e);
    const double k = std::nearbyint(std::ldexp(rest, 40 - e));
    return int16_t(std::fmin(std::fmax(k, -32768.0), 32767.0));
}
double lo_value_host(float hi, int16_t k) {
    int e = 0;
    (void)std::frexp(hi, &e);
    return std::ldexp(double(k), e - 40);
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t _e = (expr);                                                           \
        if (_e != hipSuccess)                                                             \
            return fail(SWE_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

struct DevMem {
    swe_device dev{};
    bool cb = false;
    void set(const swe_device *d) {
        if (d) dev = *d;
        cb = d && d->alloc && d->free;
    }
    void *alloc(size_t n) {
        n = std::max<size_t>(n, 256);
        if (cb) return dev.alloc(n, dev.ctx);
        void *p = nullptr;
        return hipMalloc(&p, n) == hipSuccess ? p : nullptr;
    }
    void release(void *p) {
        if (!p) return;
        if (cb)
            dev.free(p, dev.ctx);
        else
            (void)hipFree(p);
    }
    hipStream_t stream() const { return (hipStream_t)dev.hip_stream; }
};

// Tile edge lists of one mesh for one precision and tile size.
struct TileGeom {
    void *edges = nullptr;
    int *ew1 = nullptr;
    int *eoff = nullptr;
    int ntiles = 0;
    // points an instance at these lists
    template <typename T> void bind(Inst<T> &I) const {
        I.edges = dev_ptr((const Edge<T> *)edges);
        I.ew1 = dev_ptr((const int *)ew1);
        I.eoff = dev_ptr((const int *)eoff);
        I.ntiles = ntiles;
    }
};
constexpr int TILES[3] = {128, 256, 512};
constexpr int AUTOTUNE_ROUNDS = 3;  // interleaved timing rounds per tile size
int tile_index(int tile) { return tile == 128 ? 0 : tile == 256 ? 1 : tile == 512 ? 2 : -1; }

size_t vec4_bytes(int prec) { return prec == SWE_FP32 ? sizeof(float4) : sizeof(double4); }

swe_status check_flags(int flags) {
    if (flags & FLAG_NONFINITE) return fail(SWE_ENONFINITE, "state became non-finite");
    if (flags & FLAG_NEGDEPTH) return fail(SWE_ENEGDEPTH, "negative depth under the error policy");
    if (flags & FLAG_NODT) return fail(SWE_ENODT, "no finite positive time step");
    if (flags & FLAG_SINK) return fail(SWE_ESINK, "an exact sink asked for more water than a cell held");
    return SWE_OK;
}

bool valid_tile(int b) { return tile_index(b) >= 0; }

}  // namespace

struct swe_mesh {
    DevMem mem;
    HostMesh H;
    double *area = nullptr;  // |cell| in FP64 (mass sums, clip volume)
    TileGeom geom[2][3];     // [precision][tile size]
    ~swe_mesh() {
        mem.release(area);
        for (auto &row : geom)
            for (auto &g : row) {
                mem.release(g.edges);
                mem.release(g.ew1);
                mem.release(g.eoff);
            }
    }
    swe_status ensure_area() {
        if (area) return SWE_OK;
        area = (double *)mem.alloc((size_t)H.nc * sizeof(double));
        if (!area) return fail(SWE_ENOMEM, "device allocation failed (mesh areas)");
        HIP_TRY(hipMemcpyAsync(area, H.area.data(), (size_t)H.nc * sizeof(double), hipMemcpyHostToDevice,
                               mem.stream()));
        HIP_TRY(hipStreamSynchronize(mem.stream()));
        return SWE_OK;
    }
    // the tile edge lists for (precision, tile), built and uploaded on first use
    template <typename T> swe_status ensure_tiles(int prec, int tile) {
        TileGeom &g = geom[prec][tile_index(tile)];
        if (g.edges) return SWE_OK;
        swe_status st = ensure_area();
        if (st) return st;
        std::vector<TileEdge> te;
        std::vector<int32_t> eoff;
        if (!build_tile_edges(H, tile, te, eoff)) return fail(SWE_EINVAL, "cannot build tile edge lists");
        std::vector<Edge<T>> ed(te.size());
        std::vector<int> w1(te.size());
        for (size_t k = 0; k < te.size(); k++) {
            ed[k].w0 = te[k].w0;
            ed[k].lx = T(te[k].lx);
            ed[k].ly = T(te[k].ly);
            w1[k] = te[k].w1;
        }
        g.edges = mem.alloc(std::max<size_t>(ed.size(), 1) * sizeof(Edge<T>));
        g.ew1 = (int *)mem.alloc(std::max<size_t>(w1.size(), 1) * sizeof(int));
        g.eoff = (int *)mem.alloc(eoff.size() * sizeof(int));
        if (!g.edges || !g.ew1 || !g.eoff) return fail(SWE_ENOMEM, "device allocation failed (tile edges)");
        hipStream_t s = mem.stream();
        if (!ed.empty()) {
            HIP_TRY(hipMemcpyAsync(g.edges, ed.data(), ed.size() * sizeof(Edge<T>), hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(g.ew1, w1.data(), w1.size() * sizeof(int), hipMemcpyHostToDevice, s));
        }
        HIP_TRY(hipMemcpyAsync(g.eoff, eoff.data(), eoff.size() * sizeof(int), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        g.ntiles = (int)(eoff.size() - 1);
        return SWE_OK;
    }
};

struct swe_state {
    swe_mesh *m = nullptr;
    swe_params p{};
    DevMem mem;
    int prec = SWE_FP64;
    void *U0 = nullptr, *U1 = nullptr, *cellp = nullptr;
    int *slot_kbc = nullptr;
    double *slot_acc = nullptr;
    BCdev *bcs = nullptr;
    double *hydro = nullptr;
    Ctrl *ctrl = nullptr;
    double2 *partials = nullptr;
    double *mass_out = nullptr;
    int16_t *L0 = nullptr, *L1 = nullptr;  // FP32: 16-bit low parts of the surface (ping-pong with U0/U1)
    double *clip_acc = nullptr;  // per 64-cell group: compensated clip volume
    int ngroups = 0;
    Ctrl *hctrl = nullptr;    // pinned host copy of the control block
    double *hbuf = nullptr;   // pinned scratch (t_end, mass results)
    int nslots = 0, n_bc = 0;
    // passive species: specific masses [ns][n] (ping-pong with U0/U1), inflow
    // concentrations [n_bc][ns], per-slot boundary accumulators, reset tallies
    int ns = 0;
    void *Q0 = nullptr, *Q1 = nullptr, *phi_in = nullptr;
    // diffusion of the species: auxiliary variables [ns][n] pairs (ping-pong)
    void *P0 = nullptr, *P1 = nullptr;
    int diff = 0;
    double dKm[MAX_SPECIES] = {}, dKmax = 0.0, daL = 0.0, daT = 0.0, dzeta = 1.0;
    double *sslot_acc = nullptr, *sclip_acc = nullptr;
    // external sources: per device cell the region, per region its record
    // and series, per tile (at the smallest tile size) a volume accumulator
    int nsrc = 0, src_tiles = 0;
    int *src_cell = nullptr;
    BCdev *srcs = nullptr;
    double *src_series = nullptr, *src_acc = nullptr;
    // morphodynamics: the non-erodible bed (device order, or none), per
    // boundary slot the sediment outflow, the fixed-bed clip tally
    int morpho = 0;
    void *zfix = nullptr;
    void *theta = nullptr;  // draining factors of the step (limiter on)
    int *iw_bc = nullptr;   // per interior-tag index: its wall condition or -1
    double *bslot_acc = nullptr, *bclip_acc = nullptr;
    int tile = 256, spg = 32;
    int phase = 0;  // step launches issued so far, mod 3 (selects the control slot)
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};  // one per starting phase
    int g_k = 0, g_tile = 0;
    Inst<float> inst32{};
    Inst<double> inst64{};

    ~swe_state() {
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        for (void *q : {U0, U1, (void *)L0, (void *)L1, cellp, (void *)slot_kbc, (void *)slot_acc, (void *)bcs,
                        (void *)hydro, (void *)ctrl,
                        (void *)partials, (void *)mass_out, (void *)clip_acc, theta, (void *)iw_bc})
            mem.release(q);
        drop_species();
        drop_sources();
        drop_morpho();
        if (hctrl) (void)hipHostFree(hctrl);
        if (hbuf) (void)hipHostFree(hbuf);
    }
    hipStream_t stream() const { return mem.stream(); }
    void drop_species() {
        drop_diffusion();
        for (void *q : {Q0, Q1, phi_in, (void *)sslot_acc, (void *)sclip_acc}) mem.release(q);
        Q0 = Q1 = phi_in = nullptr;
        sslot_acc = sclip_acc = nullptr;
        ns = 0;
        bind_species();
    }
    void drop_diffusion() {
        mem.release(P0);
        mem.release(P1);
        P0 = P1 = nullptr;
        diff = 0;
        bind_diffusion();
    }
    void bind_diffusion() {
        inst32.P0 = dev_ptr((float *)P0);
        inst32.P1 = dev_ptr((float *)P1);
        inst64.P0 = dev_ptr((double *)P0);
        inst64.P1 = dev_ptr((double *)P1);
        inst32.diff = inst64.diff = diff;
        for (int c = 0; c < MAX_SPECIES; c++) inst32.dKm[c] = inst64.dKm[c] = dKm[c];
        inst32.dKmax = inst64.dKmax = dKmax;
        inst32.daL = inst64.daL = daL;
        inst32.daT = inst64.daT = daT;
        inst32.dzeta = inst64.dzeta = dzeta;
    }
    void drop_morpho() {
        for (void *q : {zfix, (void *)bslot_acc, (void *)bclip_acc}) mem.release(q);
        zfix = nullptr;
        bslot_acc = bclip_acc = nullptr;
        morpho = 0;
        inst32.morpho = inst64.morpho = 0;
        inst32.zfix = nullptr;
        inst64.zfix = nullptr;
        inst32.bslot_acc = inst64.bslot_acc = nullptr;
        inst32.bclip_acc = inst64.bclip_acc = nullptr;
    }
    void drop_sources() {
        for (void *q : {(void *)src_cell, (void *)srcs, (void *)src_series, (void *)src_acc}) mem.release(q);
        src_cell = nullptr;
        srcs = nullptr;
        src_series = src_acc = nullptr;
        nsrc = src_tiles = 0;
        bind_sources();
    }
    void bind_sources() {
        inst32.nsrc = inst64.nsrc = nsrc;
        inst32.src_cell = inst64.src_cell = dev_ptr((const int *)src_cell);
        inst32.srcs = inst64.srcs = srcs;
        inst32.src_acc = inst64.src_acc = src_acc;
    }
    // copies the species buffers into both kernel parameter blocks
    void bind_species() {
        inst32.Q0 = dev_ptr((float *)Q0);
        inst32.Q1 = dev_ptr((float *)Q1);
        inst32.phi_in = (const float *)phi_in;
        inst64.Q0 = dev_ptr((double *)Q0);
        inst64.Q1 = dev_ptr((double *)Q1);
        inst64.phi_in = (const double *)phi_in;
        inst32.sslot_acc = inst64.sslot_acc = sslot_acc;
        inst32.sclip_acc = inst64.sclip_acc = sclip_acc;
        inst32.ns = inst64.ns = ns;
    }
    // the current time level as last read from the device
    const CtrlSlot &lvl() const { return hctrl->s[phase]; }
    void drop_graphs() {
        for (auto &g : gexec)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    }
    hipError_t launch_one_on(hipStream_t s, int ph) {
        return prec == SWE_FP32 ? launch_step<float>(inst32, tile, ph, s) : launch_step<double>(inst64, tile, ph, s);
    }
    hipError_t launch_one() {
        hipError_t e = launch_one_on(stream(), phase);
        phase = (phase + 1) % 3;
        return e;
    }
    swe_status set_t_end(double t_end) {
        hbuf[0] = t_end;
        HIP_TRY(hipMemcpyAsync(&ctrl->t_end, hbuf, sizeof(double), hipMemcpyHostToDevice, stream()));
        return SWE_OK;
    }
    swe_status read_ctrl() {
        HIP_TRY(hipMemcpyAsync(hctrl, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream()));
        HIP_TRY(hipStreamSynchronize(stream()));
        return SWE_OK;
    }
    // FP32: the codes of the low parts of the current level's surfaces
    // (device order) into lo; FP64: lo left empty
    swe_status read_lo(std::vector<int16_t> &lo) {
        lo.clear();
        if (prec != SWE_FP32) return SWE_OK;
        lo.resize((size_t)m->H.nc);
        const int16_t *src = lvl().cur ? L1 : L0;
        HIP_TRY(hipMemcpyAsync(lo.data(), src, lo.size() * sizeof(int16_t), hipMemcpyDeviceToHost, stream()));
        HIP_TRY(hipStreamSynchronize(stream()));
        return SWE_OK;
    }
    // k captured steps starting at launch phase ph
    swe_status graph(int k, int ph) {
        if (g_k != k || g_tile != tile) drop_graphs();
        if (gexec[ph]) return SWE_OK;
        if (!cap) HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t gr = nullptr;
        HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < k; i++) {
            hipError_t e = launch_one_on(cap, (ph + i) % 3);
            if (e != hipSuccess) {
                hipGraph_t dummy = nullptr;
                (void)hipStreamEndCapture(cap, &dummy);
                if (dummy) (void)hipGraphDestroy(dummy);
                return fail(SWE_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
            }
        }
        HIP_TRY(hipStreamEndCapture(cap, &gr));
        hipError_t e = hipGraphInstantiate(&gexec[ph], gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return fail(SWE_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        g_k = k;
        g_tile = tile;
        return SWE_OK;
    }
    swe_status launch_graph() {
        swe_status st = graph(spg, phase);
        if (st) return st;
        HIP_TRY(hipGraphLaunch(gexec[phase], stream()));
        phase = (phase + spg) % 3;
        return SWE_OK;
    }
    // switches the tile size (block size) of the step kernel
    swe_status set_tile(int t) {
        swe_status st = prec == SWE_FP32 ? m->ensure_tiles<float>(prec, t) : m->ensure_tiles<double>(prec, t);
        if (st) return st;
        const TileGeom &g = m->geom[prec][tile_index(t)];
        g.bind(inst32);
        g.bind(inst64);
        tile = t;
        return SWE_OK;
    }
    // recomputes the CFL minimum of the current level, after the terms that
    // bound the step have changed (diffusion switched on or off)
    swe_status reseed_dt() {
        const unsigned long long inf = INF_BITS;
        HIP_TRY(hipMemcpyAsync(&ctrl->m[phase].bits, &inf, sizeof inf, hipMemcpyHostToDevice, stream()));
        HIP_TRY(prec == SWE_FP32 ? launch_dt_init<float>(inst32, tile, phase, stream())
                                 : launch_dt_init<double>(inst64, tile, phase, stream()));
        HIP_TRY(hipStreamSynchronize(stream()));
        return read_ctrl();
    }
    // moves the current level to control slot `to` (aligning with a batch)
    swe_status realign(int to) {
        if (to == phase) return SWE_OK;
        swe_status st = read_ctrl();
        if (st) return st;
        Ctrl c = *hctrl;
        c.s[to] = hctrl->s[phase];
        c.m[to] = hctrl->m[phase];
        c.m[(to + 1) % 3].bits = INF_BITS;
        c.m[(to + 2) % 3].bits = INF_BITS;
        *hctrl = c;
        HIP_TRY(hipMemcpyAsync(ctrl, hctrl, sizeof(Ctrl), hipMemcpyHostToDevice, stream()));
        HIP_TRY(hipStreamSynchronize(stream()));
        phase = to;
        return SWE_OK;
    }
};

extern "C" {

static_assert(FR_MANNING == SWE_FRICTION_MANNING && FR_STRICKLER == SWE_FRICTION_STRICKLER &&
                  FR_CHEZY == SWE_FRICTION_CHEZY && FR_BEZZOLA == SWE_FRICTION_BEZZOLA,
              "friction closure numbering");
static_assert(SED_MPM == SWE_SED_MPM && SED_GRASS == SWE_SED_GRASS && SED_EH == SWE_SED_EH,
              "sediment closure numbering");
static_assert(SRC_EXACT == SWE_SRC_EXACT && SRC_AVAILABLE == SWE_SRC_AVAILABLE && SRC_INFINITY == SWE_SRC_INFINITY,
              "source mode numbering");

void swe_params_default(swe_params *p) {
    if (!p) return;
    p->g = 9.81;
    p->cfl = 0.9;
    p->h_min = 1e-4;
    p->dt_max = std::numeric_limits<double>::infinity();
    p->precision = SWE_FP64;
    p->neg_depth_policy = SWE_NEG_CLIP;
    p->block_size = 0;
    p->steps_per_graph = 0;
    p->renumber = 1;
    p->friction = SWE_FRICTION_MANNING;
    p->limiter = SWE_LIMIT_NONE;
}

const char *swe_last_error(void) { return g_err.c_str(); }
const char *swe_version(void) { return "swe-gfx950 1.0"; }

swe_status swe_mesh_create(const double *node_xyz, int64_t n_nodes, const int32_t *tri, int64_t n_tri,
                           const int32_t *bnd_seg, const int32_t *bnd_tag, int64_t n_seg,
                           const swe_params *params, const swe_device *dev, swe_mesh **out) {
    if (!out) return fail(SWE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!node_xyz || !tri || n_nodes <= 0 || n_tri <= 0) return fail(SWE_EINVAL, "empty mesh");
    if (n_seg < 0 || (n_seg > 0 && (!bnd_seg || !bnd_tag))) return fail(SWE_EINVAL, "bad boundary segments");
    swe_params P;
    swe_params_default(&P);
    if (params) P = *params;
    std::unique_ptr<swe_mesh> m(new (std::nothrow) swe_mesh());
    if (!m) return fail(SWE_ENOMEM, "out of host memory");
    m->mem.set(dev);
    std::string err;
    try {
        if (!prepare_mesh(node_xyz, n_nodes, tri, n_tri, bnd_seg, bnd_tag, n_seg, P.renumber != 0, m->H, err))
            return fail(SWE_EINVAL, err);
    } catch (const std::bad_alloc &) {
        return fail(SWE_ENOMEM, "out of host memory");
    }
    *out = m.release();
    return SWE_OK;
}

void swe_mesh_destroy(swe_mesh *m) { delete m; }

void swe_mesh_info(const swe_mesh *m, int64_t *n_cells, int64_t *n_edges, int64_t *n_boundary_edges) {
    if (!m) return;
    if (n_cells) *n_cells = m->H.nc;
    if (n_edges) *n_edges = m->H.ne;
    if (n_boundary_edges) *n_boundary_edges = m->H.nb;
}

swe_status swe_mesh_check(const swe_mesh *m, int32_t tile) {
    if (!m) return fail(SWE_EINVAL, "mesh is NULL");
    if (!valid_tile(tile)) return fail(SWE_EINVAL, "tile must be 128, 256 or 512");
    std::vector<TileEdge> te;
    std::vector<int32_t> eoff;
    if (!build_tile_edges(m->H, tile, te, eoff)) return fail(SWE_EINVAL, "cannot build tile edge lists");
    const std::string err = check_tile_edges(m->H, tile, te, eoff);
    if (!err.empty()) return fail(SWE_EINVAL, err);
    return SWE_OK;
}

int64_t swe_state_footprint(const swe_mesh *m, int32_t precision) {
    if (!m) return 0;
    const int64_t n = m->H.nc, ns = (int64_t)m->H.slot_tag.size();
    const int64_t v4 = (int64_t)vec4_bytes(precision);
    // FP32 adds the low parts of the surface (two buffers of 2 bytes per cell)
    const int64_t lo = precision == SWE_FP32 ? 2 * n * 2 : 0;
    const int64_t state = 2 * n * v4 + lo + n * v4 / 2 + ns * (4 + 16) + (int64_t)sizeof(Ctrl) + MASS_BLOCKS * 16 +
                          4096;
    // tile edge list (about 1.7 edges per cell: record + other-cell id) and FP64 areas
    const int64_t edge = precision == SWE_FP32 ? 12 + 4 : 24 + 4;
    const int64_t geom = n * 8 + (n * 7 / 4) * edge + 4 * (n / 128 + 2);
    return state + geom;
}

swe_status swe_state_init(const swe_mesh *m, const swe_params *params, const double *H0, const double *h0,
                          const double *qx0, const double *qy0, const double *manning, const swe_bc *bcs,
                          int32_t n_bc, double t0, swe_state **out) {
    if (!out) return fail(SWE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!m) return fail(SWE_EINVAL, "mesh is NULL");
    swe_params P;
    swe_params_default(&P);
    if (params) P = *params;
    if (!(P.g > 0) || !std::isfinite(P.g)) return fail(SWE_EINVAL, "g must be positive");
    if (!(P.cfl > 0 && P.cfl <= 1)) return fail(SWE_EINVAL, "cfl must lie in (0, 1]");
    if (!(P.h_min > 0) || !std::isfinite(P.h_min)) return fail(SWE_EINVAL, "h_min must be positive");
    if (!(P.dt_max > 0)) return fail(SWE_EINVAL, "dt_max must be positive");
    if (P.precision != SWE_FP32 && P.precision != SWE_FP64) return fail(SWE_EINVAL, "unknown precision");
    if (P.neg_depth_policy != SWE_NEG_CLIP && P.neg_depth_policy != SWE_NEG_ERROR)
        return fail(SWE_EINVAL, "unknown negative-depth policy");
    if (P.block_size != 0 && !valid_tile(P.block_size)) return fail(SWE_EINVAL, "block_size must be 0, 128, 256 or 512");
    if (P.steps_per_graph < 0 || P.steps_per_graph > 4096) return fail(SWE_EINVAL, "steps_per_graph out of range");
    if (P.friction < SWE_FRICTION_MANNING || P.friction > SWE_FRICTION_BEZZOLA)
        return fail(SWE_EINVAL, "unknown friction closure");
    if (P.limiter != SWE_LIMIT_NONE && P.limiter != SWE_LIMIT_DRAIN) return fail(SWE_EINVAL, "unknown limiter");
    if (H0 && h0) return fail(SWE_EINVAL, "give H0 or h0, not both");
    if (!std::isfinite(t0)) return fail(SWE_EINVAL, "t0 must be finite");
    if (n_bc < 0 || n_bc > MAX_BC || (n_bc > 0 && !bcs)) return fail(SWE_EINVAL, "bad boundary-condition list");

    const HostMesh &M = m->H;
    const int64_t n = M.nc;
    const int prec = P.precision;
    // initial state in device order
    std::vector<double> H((size_t)n), qx((size_t)n), qy((size_t)n), gn2((size_t)n);
    for (int64_t i = 0; i < n; i++) {
        const int32_t p = M.inv[i];
        // the bed the state carries: FP32 states keep it in single precision,
        // and an initial depth or a clamped surface refers to that bed
        const double z = prec == SWE_FP32 ? double(float(M.zb[p])) : M.zb[p];
        double Hi;
        if (H0) {
            if (!std::isfinite(H0[i])) return fail(SWE_EINVAL, "non-finite initial surface");
            Hi = H0[i] > z ? H0[i] : z;  // a surface below the bed is a dry cell
        } else {
            const double d = h0 ? h0[i] : 0.0;
            if (!(d >= 0) || !std::isfinite(d)) return fail(SWE_EINVAL, "negative or non-finite initial depth");
            Hi = z + d;
        }
        const double a = qx0 ? qx0[i] : 0.0, b = qy0 ? qy0[i] : 0.0, nn = manning ? manning[i] : 0.0;
        if (!std::isfinite(a) || !std::isfinite(b)) return fail(SWE_EINVAL, "non-finite initial discharge");
        if (!(nn >= 0) || !std::isfinite(nn)) return fail(SWE_EINVAL, "friction parameter must be finite and >= 0");
        H[p] = Hi;
        qx[p] = a;
        qy[p] = b;
        // friction coefficient as the kernels use it: g n^2 for the power
        // laws (Strickler: n = 1/k_str), K_s or y_R for the log types
        if (P.friction == SWE_FRICTION_MANNING)
            gn2[p] = P.g * nn * nn;
        else if (P.friction == SWE_FRICTION_STRICKLER)
            gn2[p] = nn > 0 ? P.g / (nn * nn) : 0.0;
        else
            gn2[p] = nn;
    }
    // boundary conditions
    std::vector<BCdev> hb((size_t)std::max(n_bc, 1));
    std::vector<double> hydro;
    std::vector<size_t> hoff((size_t)std::max(n_bc, 1));
    for (int b = 0; b < n_bc; b++) {
        const swe_bc &B = bcs[b];
        if (B.kind < SWE_BC_WALL || B.kind > SWE_BC_DYNAMIC_WALL) return fail(SWE_EINVAL, "unknown boundary kind");
        if (!std::isfinite(B.slope) || !std::isfinite(B.par)) return fail(SWE_EINVAL, "non-finite boundary parameter");
        hb[b] = BCdev{B.kind, 0, B.slope, 0.0, nullptr, nullptr, B.par};
        hoff[b] = hydro.size();
        if (B.kind == SWE_BC_DYNAMIC_WALL && B.par < 0.0)
            return fail(SWE_EINVAL, "a dynamic wall's collapse depth must be >= 0");
        if ((B.kind == SWE_BC_INFLOW_UNIFORM || B.kind == SWE_BC_INFLOW_FROUDE || B.kind == SWE_BC_OUTFLOW_UNIFORM) &&
            !(B.slope > 0))
            return fail(SWE_EINVAL, "uniform and froude conditions need a positive slope or Froude number");
        if (B.kind == SWE_BC_OUTFLOW_WEIR && !(B.par > 0)) return fail(SWE_EINVAL, "a weir needs a positive Poleni factor");
        if (B.kind == SWE_BC_INFLOW_UNIFORM || B.kind == SWE_BC_ZHYDROGRAPH || B.kind == SWE_BC_INFLOW_FROUDE ||
            B.kind == SWE_BC_OUTFLOW_HQ) {
            if (B.n_pts < 1 || !B.t || !B.Q) return fail(SWE_EINVAL, "inflows, zhydrograph and h-Q need a series");
            for (int k = 0; k < B.n_pts; k++) {
                if (!std::isfinite(B.t[k]) || !std::isfinite(B.Q[k])) return fail(SWE_EINVAL, "non-finite hydrograph");
                if (k > 0 && !(B.t[k] > B.t[k - 1])) return fail(SWE_EINVAL, "hydrograph times must increase");
                if (B.kind == SWE_BC_OUTFLOW_HQ && B.Q[k] < 0.0) return fail(SWE_EINVAL, "h-Q discharges must be >= 0");
            }
            hb[b].npts = B.n_pts;
            hydro.insert(hydro.end(), B.t, B.t + B.n_pts);
            hydro.insert(hydro.end(), B.Q, B.Q + B.n_pts);
        }
    }
    // internal conditions on tagged interior edges: walls, dynamic walls and
    // rating curves (h-Q relations)
    std::vector<int> iwb(MAX_IW_TAGS + 1, -1);
    bool iw_hq = false;
    for (size_t k = 0; k < M.iw_tags.size(); k++)
        for (int b = 0; b < n_bc; b++) {
            if (bcs[b].tag != M.iw_tags[k]) continue;
            if (bcs[b].kind != SWE_BC_WALL && bcs[b].kind != SWE_BC_DYNAMIC_WALL && bcs[b].kind != SWE_BC_OUTFLOW_HQ)
                return fail(SWE_EINVAL, "interior edges take walls, dynamic walls and h-Q relations only");
            iwb[k] = b;
            iw_hq = iw_hq || bcs[b].kind == SWE_BC_OUTFLOW_HQ;
            break;
        }
    if (iw_hq && P.limiter == SWE_LIMIT_DRAIN)
        return fail(SWE_EINVAL, "internal h-Q relations and the draining-time limiter do not combine");
    int iw_on = 0;
    for (int v : iwb) iw_on |= v >= 0;
    const int nslots = (int)M.slot_tag.size();
    std::vector<int> kbc((size_t)std::max(nslots, 1), BC_WALL);
    std::vector<std::vector<double>> lens((size_t)std::max(n_bc, 1));
    // an internal rating curve spreads its discharge over the length of its
    // interior edges (each counted once, on its upstream side)
    for (int64_t p = 0; p < M.nc; p++)
        for (int k = 0; k < 3; k++) {
            const int32_t iw = M.iw_slot[3 * p + k];
            if (iw < 0 || !M.iw_up[3 * p + k] || iwb[iw] < 0 || bcs[iwb[iw]].kind != SWE_BC_OUTFLOW_HQ) continue;
            const double lx = M.lx[3 * p + k], ly = M.ly[3 * p + k];
            lens[iwb[iw]].push_back(std::sqrt(lx * lx + ly * ly));
        }
    for (int s = 0; s < nslots; s++) {
        const int32_t tg = M.slot_tag[s];
        if (tg < 0) continue;
        for (int b = 0; b < n_bc; b++) {
            if (bcs[b].tag != tg) continue;
            if (bcs[b].kind == SWE_BC_WALL) break;
            kbc[s] = bcs[b].kind | (b << 4);
            lens[b].push_back(M.slot_len[s]);
            const bool unif = bcs[b].kind == SWE_BC_INFLOW_UNIFORM || bcs[b].kind == SWE_BC_OUTFLOW_UNIFORM;
            if (unif && P.friction >= SWE_FRICTION_CHEZY)
                return fail(SWE_EINVAL, "uniform inflow or outflow needs the Manning or Strickler closure");
            if (unif && !(gn2[M.slot_cell[s]] > 0))
                return fail(SWE_EINVAL, "uniform inflow or outflow edge next to a frictionless cell");
            break;
        }
    }
    // boundary length: edge lengths summed in ascending order, so the value
    // does not depend on how cells or edges are numbered
    for (int b = 0; b < n_bc; b++) {
        std::sort(lens[b].begin(), lens[b].end());
        double L = 0.0;
        for (double x : lens[b]) L += x;
        hb[b].length = L;
    }

    std::unique_ptr<swe_state> S(new (std::nothrow) swe_state());
    if (!S) return fail(SWE_ENOMEM, "out of host memory");
    S->m = const_cast<swe_mesh *>(m);
    S->p = P;
    S->mem = m->mem;
    S->prec = prec;
    S->nslots = nslots;
    S->n_bc = n_bc;
    S->tile = P.block_size ? P.block_size : 256;
    S->spg = P.steps_per_graph ? P.steps_per_graph : 32;
    swe_status st = prec == SWE_FP32 ? S->m->ensure_tiles<float>(prec, S->tile)
                                     : S->m->ensure_tiles<double>(prec, S->tile);
    if (st) return st;

    const size_t v4 = vec4_bytes(prec);
    S->U0 = S->mem.alloc((size_t)n * v4);
    S->U1 = S->mem.alloc((size_t)n * v4);
    if (prec == SWE_FP32) {
        S->L0 = (int16_t *)S->mem.alloc((size_t)std::max<int64_t>(n, 1) * sizeof(int16_t));
        S->L1 = (int16_t *)S->mem.alloc((size_t)std::max<int64_t>(n, 1) * sizeof(int16_t));
        if (!S->L0 || !S->L1) return fail(SWE_ENOMEM, "device allocation failed (state)");
    }
    S->cellp = S->mem.alloc((size_t)n * v4 / 2);
    S->slot_kbc = (int *)S->mem.alloc(sizeof(int) * std::max(nslots, 1));
    S->slot_acc = (double *)S->mem.alloc(2 * sizeof(double) * std::max(nslots, 1));
    S->bcs = (BCdev *)S->mem.alloc(sizeof(BCdev) * std::max(n_bc, 1));
    S->hydro = (double *)S->mem.alloc(sizeof(double) * std::max<size_t>(hydro.size(), 1));
    S->ctrl = (Ctrl *)S->mem.alloc(sizeof(Ctrl));
    S->partials = (double2 *)S->mem.alloc(sizeof(double2) * MASS_BLOCKS);
    S->mass_out = (double *)S->mem.alloc(4 * sizeof(double));
    S->ngroups = (int)((n + 63) / 64);
    S->clip_acc = (double *)S->mem.alloc(2 * sizeof(double) * std::max(S->ngroups, 1));
    S->iw_bc = (int *)S->mem.alloc(sizeof(int) * iwb.size());
    if (!S->iw_bc) return fail(SWE_ENOMEM, "device allocation failed (state)");
    if (P.limiter == SWE_LIMIT_DRAIN) {
        S->theta = S->mem.alloc((size_t)n * (prec == SWE_FP32 ? sizeof(float) : sizeof(double)));
        if (!S->theta) return fail(SWE_ENOMEM, "device allocation failed (limiter)");
    }
    if (!S->U0 || !S->U1 || !S->cellp || !S->slot_kbc || !S->slot_acc || !S->bcs || !S->hydro || !S->ctrl ||
        !S->partials || !S->mass_out || !S->clip_acc)
        return fail(SWE_ENOMEM, "device allocation failed (state)");
    HIP_TRY(hipHostMalloc((void **)&S->hctrl, sizeof(Ctrl), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&S->hbuf, 64, hipHostMallocDefault));
    for (int b = 0; b < n_bc; b++)
        if (hb[b].npts) {
            hb[b].t = S->hydro + hoff[b];
            hb[b].Q = S->hydro + hoff[b] + hb[b].npts;
        }

    hipStream_t s = S->stream();
    auto upload = [&](auto tag) -> swe_status {
        using T = decltype(tag);
        std::vector<V4<T>> u((size_t)n);
        std::vector<V2<T>> cp((size_t)n);
        std::vector<int16_t> lo(sizeof(T) == 4 ? (size_t)n : 0);
        for (int64_t p = 0; p < n; p++) {
            u[p].x = T(H[p]);
            // FP32 stores the surface as hi + lo
            if (sizeof(T) == 4) lo[p] = lo_code_host(float(u[p].x), H[p] - double(u[p].x));
            u[p].y = T(qx[p]);
            u[p].z = T(qy[p]);
            u[p].w = T(M.zb[p]);
            // FP64 keeps |cell| (the update divides by it); FP32 stores 1/|cell|
            cp[p].x = sizeof(T) == 8 ? T(M.area[p]) : T(1.0 / M.area[p]);
            cp[p].y = T(gn2[p]);
        }
        HIP_TRY(hipMemcpyAsync(S->U0, u.data(), u.size() * sizeof(V4<T>), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(S->U1, u.data(), u.size() * sizeof(V4<T>), hipMemcpyHostToDevice, s));
        if (!lo.empty()) {
            HIP_TRY(hipMemcpyAsync(S->L0, lo.data(), lo.size() * sizeof(int16_t), hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(S->L1, lo.data(), lo.size() * sizeof(int16_t), hipMemcpyHostToDevice, s));
        }
        HIP_TRY(hipMemcpyAsync(S->cellp, cp.data(), cp.size() * sizeof(V2<T>), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        return SWE_OK;
    };
    st = prec == SWE_FP32 ? upload(float()) : upload(double());
    if (st) return st;
    std::vector<double> zeros((size_t)2 * std::max(nslots, 1), 0.0);
    HIP_TRY(hipMemcpyAsync(S->slot_kbc, kbc.data(), sizeof(int) * kbc.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(S->slot_acc, zeros.data(), sizeof(double) * zeros.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(S->clip_acc, 0, 2 * sizeof(double) * std::max(S->ngroups, 1), s));
    HIP_TRY(hipMemcpyAsync(S->bcs, hb.data(), sizeof(BCdev) * hb.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(S->iw_bc, iwb.data(), sizeof(int) * iwb.size(), hipMemcpyHostToDevice, s));
    if (!hydro.empty())
        HIP_TRY(hipMemcpyAsync(S->hydro, hydro.data(), sizeof(double) * hydro.size(), hipMemcpyHostToDevice, s));
    Ctrl c;
    std::memset(&c, 0, sizeof(c));
    c.s[0].t = t0;
    for (auto &mm : c.m) mm.bits = INF_BITS;
    c.t_end = std::numeric_limits<double>::infinity();
    *S->hctrl = c;
    S->phase = 0;
    HIP_TRY(hipMemcpyAsync(S->ctrl, S->hctrl, sizeof(Ctrl), hipMemcpyHostToDevice, s));

    auto fill_inst = [&](auto &I, auto tag) {
        using T = decltype(tag);
        I.U0 = dev_ptr((V4<T> *)S->U0);
        I.U1 = dev_ptr((V4<T> *)S->U1);
        I.L0 = dev_ptr(S->L0);
        I.L1 = dev_ptr(S->L1);
        const TileGeom &tg = m->geom[prec][tile_index(S->tile)];
        I.cellp = dev_ptr((const V2<T> *)S->cellp);
        tg.bind(I);
        I.slot_kbc = dev_ptr((const int *)S->slot_kbc);
        I.slot_acc = dev_ptr(S->slot_acc);
        I.bcs = S->bcs;
        I.area = dev_ptr((const double *)m->area);
        I.ctrl = S->ctrl;
        I.clip_acc = dev_ptr(S->clip_acc);
        I.ngroups = S->ngroups;
        I.n = (int)n;
        I.ntiles = tg.ntiles;
        I.g = P.g;
        I.sqrtg = std::sqrt(P.g);
        I.sqrt2g = std::sqrt(2.0 * P.g);
        I.cfl = P.cfl;
        I.h_min = P.h_min;
        I.dt_max = P.dt_max;
        I.neg_policy = P.neg_depth_policy;
        I.friction = P.friction;
        I.drain = P.limiter == SWE_LIMIT_DRAIN;
        I.iw_bc = S->iw_bc;
        I.iw_on = iw_on;
        I.theta = dev_ptr((T *)S->theta);
    };
    if (prec == SWE_FP32) {
        fill_inst(S->inst32, float());
        HIP_TRY(launch_dt_init<float>(S->inst32, S->tile, S->phase, s));
    } else {
        fill_inst(S->inst64, double());
        HIP_TRY(launch_dt_init<double>(S->inst64, S->tile, S->phase, s));
    }
    st = S->read_ctrl();
    if (st) return st;
    *out = S.release();
    return SWE_OK;
}

void swe_state_destroy(swe_state *s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream());
    delete s;
}

swe_status swe_step(swe_state *s, double *dt_taken) {
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    swe_status st = s->set_t_end(std::numeric_limits<double>::infinity());
    if (st) return st;
    const long long before = s->lvl().steps;
    HIP_TRY(s->launch_one());
    st = s->read_ctrl();
    if (st) return st;
    st = check_flags(s->hctrl->flags);
    if (st) return st;
    if (s->lvl().steps == before) return fail(SWE_ENODT, "step did not advance");
    if (dt_taken) *dt_taken = s->lvl().dt;
    return SWE_OK;
}

swe_status swe_run_until(swe_state *s, double t_end, int64_t *n_steps) {
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (std::isnan(t_end)) return fail(SWE_EINVAL, "t_end is NaN");
    swe_status st = s->set_t_end(t_end);
    if (st) return st;
    st = s->read_ctrl();
    if (st) return st;
    const long long start = s->lvl().steps;
    if (n_steps) *n_steps = 0;
    st = check_flags(s->hctrl->flags);
    if (st) return st;
    while (s->lvl().t < t_end) {
        const double t_before = s->lvl().t;
        st = s->launch_graph();
        if (st) return st;
        st = s->read_ctrl();
        if (st) return st;
        if (n_steps) *n_steps = s->lvl().steps - start;
        st = check_flags(s->hctrl->flags);
        if (st) return st;
        if (!(s->lvl().t > t_before)) return fail(SWE_ENODT, "time does not advance (step underflow)");
    }
    return SWE_OK;
}

swe_status swe_launch_steps(swe_state *s, double t_end, int64_t k) {
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (k < 0) return fail(SWE_EINVAL, "negative step count");
    swe_status st = s->set_t_end(t_end);
    if (st) return st;
    int64_t left = k;
    while (left >= s->spg) {
        st = s->launch_graph();
        if (st) return st;
        left -= s->spg;
    }
    for (; left > 0; left--) HIP_TRY(s->launch_one());
    return SWE_OK;
}

swe_status swe_sync(swe_state *s) {
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    swe_status st = s->read_ctrl();
    if (st) return st;
    return check_flags(s->hctrl->flags);
}

swe_status swe_prepare_graphs(swe_state *s, int32_t steps_per_graph) {
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (steps_per_graph < 0 || steps_per_graph > 4096) return fail(SWE_EINVAL, "steps_per_graph out of range");
    if (steps_per_graph > 0) s->spg = steps_per_graph;
    for (int ph = 0; ph < 3; ph++) {
        swe_status st = s->graph(s->spg, ph);
        if (st) return st;
    }
    return SWE_OK;
}

swe_status swe_state_read(const swe_state *cs, double *H, double *h, double *qx, double *qy, double *t) {
    swe_state *s = const_cast<swe_state *>(cs);
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    swe_status st = s->read_ctrl();
    if (st) return st;
    const HostMesh &M = s->m->H;
    const int64_t n = M.nc;
    const void *src = s->lvl().cur ? s->U1 : s->U0;
    auto rd = [&](auto tag) -> swe_status {
        using T = decltype(tag);
        std::vector<V4<T>> u((size_t)n);
        std::vector<int16_t> lo;
        HIP_TRY(hipMemcpyAsync(u.data(), src, u.size() * sizeof(V4<T>), hipMemcpyDeviceToHost, s->stream()));
        swe_status r = s->read_lo(lo);
        if (r) return r;
        for (int64_t i = 0; i < n; i++) {
            const int32_t d = M.inv[i];
            const V4<T> &v = u[d];
            const double Hs = lo.empty() ? double(v.x) : double(v.x) + lo_value_host(float(v.x), lo[d]);
            if (H) H[i] = Hs;
            if (h) h[i] = Hs - double(v.w);
            if (qx) qx[i] = double(v.y);
            if (qy) qy[i] = double(v.z);
        }
        return SWE_OK;
    };
    st = s->prec == SWE_FP32 ? rd(float()) : rd(double());
    if (st) return st;
    if (t) *t = s->lvl().t;
    return SWE_OK;
}

swe_status swe_mass(const swe_state *cs, double *mass, double *bnd_flux, double *clipped, int64_t *steps) {
    swe_state *s = const_cast<swe_state *>(cs);
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (s->prec == SWE_FP32)
        HIP_TRY(launch_mass<float>(s->inst32, s->partials, s->mass_out, s->nslots, s->phase, s->stream()));
    else
        HIP_TRY(launch_mass<double>(s->inst64, s->partials, s->mass_out, s->nslots, s->phase, s->stream()));
    HIP_TRY(launch_pair_sum(s->clip_acc, std::max(s->ngroups, 1), s->mass_out + 2, s->stream()));
    HIP_TRY(hipMemcpyAsync(s->hbuf + 1, s->mass_out, 3 * sizeof(double), hipMemcpyDeviceToHost, s->stream()));
    swe_status st = s->read_ctrl();
    if (st) return st;
    if (mass) *mass = s->hbuf[1];
    if (bnd_flux) *bnd_flux = s->hbuf[2];
    if (clipped) *clipped = s->hbuf[3];
    if (steps) *steps = s->lvl().steps;
    return SWE_OK;
}

swe_status swe_boundary_flux(const swe_state *cs, int32_t tag, double *volume) {
    swe_state *s = const_cast<swe_state *>(cs);
    if (!s || !volume) return fail(SWE_EINVAL, "state or volume is NULL");
    const HostMesh &M = s->m->H;
    const int nslots = (int)M.slot_tag.size();
    std::vector<double> acc((size_t)2 * std::max(nslots, 1));
    HIP_TRY(hipMemcpyAsync(acc.data(), s->slot_acc, acc.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream()));
    HIP_TRY(hipStreamSynchronize(s->stream()));
    // compensated sum over the tag's slots in slot order
    double sm = 0.0, cp = 0.0;
    for (int k = 0; k < nslots; k++) {
        if (M.slot_tag[k] != tag) continue;
        for (double v : {acc[2 * k], acc[2 * k + 1]}) {
            const double t = sm + v;
            cp += std::fabs(sm) >= std::fabs(v) ? (sm - t) + v : (v - t) + sm;
            sm = t;
        }
    }
    *volume = sm + cp;
    return SWE_OK;
}

swe_status swe_state_set_scalars(swe_state *s, int32_t ns, const double *phi0, const double *phi_in) {
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (ns > 0 && s->morpho) return fail(SWE_EINVAL, "species and a moving bed do not combine");
    if (ns > 0 && s->p.limiter == SWE_LIMIT_DRAIN) return fail(SWE_EINVAL, "species and the draining-time limiter do not combine");
    if (ns < 0 || ns > MAX_SPECIES) return fail(SWE_EINVAL, "between 0 and 5 species");
    const HostMesh &M = s->m->H;
    const int64_t n = M.nc;
    for (int64_t k = 0; phi0 && k < (int64_t)ns * n; k++)
        if (!std::isfinite(phi0[k])) return fail(SWE_EINVAL, "non-finite initial concentration");
    for (int64_t k = 0; phi_in && k < (int64_t)ns * s->n_bc; k++)
        if (!std::isfinite(phi_in[k])) return fail(SWE_EINVAL, "non-finite inflow concentration");
    swe_status st = s->read_ctrl();
    if (st) return st;
    s->drop_graphs();
    const bool had_diff = s->diff;
    s->drop_species();
    if (ns == 0) return had_diff ? s->reseed_dt() : SWE_OK;
    if (s->tile != SPECIES_TILE) {
        st = s->set_tile(SPECIES_TILE);
        if (st) return st;
    }
    const size_t es = s->prec == SWE_FP32 ? sizeof(float) : sizeof(double);
    const int nb = std::max(s->n_bc, 1);
    s->Q0 = s->mem.alloc((size_t)ns * n * es);
    s->Q1 = s->mem.alloc((size_t)ns * n * es);
    s->phi_in = s->mem.alloc((size_t)ns * nb * es);
    s->sslot_acc = (double *)s->mem.alloc(2 * sizeof(double) * (size_t)ns * std::max(s->nslots, 1));
    const size_t sclip_n = (size_t)2 * ns * std::max(s->ngroups, 1);
    s->sclip_acc = (double *)s->mem.alloc(sizeof(double) * sclip_n);
    if (!s->Q0 || !s->Q1 || !s->phi_in || !s->sslot_acc || !s->sclip_acc) {
        s->drop_species();
        return fail(SWE_ENOMEM, "device allocation failed (species)");
    }
    hipStream_t q = s->stream();
    const void *cur = s->lvl().cur ? s->U1 : s->U0;
    void *qcur = s->lvl().cur ? s->Q1 : s->Q0;
    // q = h phi of the current state (0 in dry cells), in device order
    auto up = [&](auto tag) -> swe_status {
        using T = decltype(tag);
        std::vector<V4<T>> u((size_t)n);
        std::vector<int16_t> lo;
        HIP_TRY(hipMemcpyAsync(u.data(), cur, u.size() * sizeof(V4<T>), hipMemcpyDeviceToHost, q));
        swe_status r = s->read_lo(lo);
        if (r) return r;
        std::vector<T> qh((size_t)ns * n), pin((size_t)ns * nb, T(0));
        for (int c = 0; c < ns; c++)
            for (int64_t i = 0; i < n; i++) {
                const int32_t d = M.inv[i];
                const V4<T> &v = u[d];
                const double h = (lo.empty() ? double(v.x) : double(v.x) + lo_value_host(float(v.x), lo[d])) - double(v.w);
                const double p = phi0 ? phi0[(size_t)c * n + i] : 0.0;
                qh[(size_t)c * n + M.inv[i]] = h > 0.0 ? T(h * p) : T(0);
            }
        for (int64_t k = 0; phi_in && k < (int64_t)ns * s->n_bc; k++) pin[k] = T(phi_in[k]);
        HIP_TRY(hipMemcpyAsync(qcur, qh.data(), qh.size() * sizeof(T), hipMemcpyHostToDevice, q));
        HIP_TRY(hipMemcpyAsync(s->phi_in, pin.data(), pin.size() * sizeof(T), hipMemcpyHostToDevice, q));
        std::vector<double> z((size_t)2 * ns * std::max(s->nslots, 1), 0.0);
        HIP_TRY(hipMemcpyAsync(s->sslot_acc, z.data(), z.size() * sizeof(double), hipMemcpyHostToDevice, q));
        HIP_TRY(hipMemsetAsync(s->sclip_acc, 0, sclip_n * sizeof(double), q));
        HIP_TRY(hipStreamSynchronize(q));
        return SWE_OK;
    };
    st = s->prec == SWE_FP32 ? up(float()) : up(double());
    if (st) {
        s->drop_species();
        return st;
    }
    s->ns = ns;
    s->bind_species();
    return had_diff ? s->reseed_dt() : SWE_OK;
}

swe_status swe_state_set_diffusion(swe_state *s, const double *Km, double alpha_L, double alpha_T, double zeta,
                                   const double *psi0) {
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (s->ns < 1) return fail(SWE_EINVAL, "diffusion needs species (swe_state_set_scalars first)");
    if (s->nsrc > 0) return fail(SWE_EINVAL, "diffusing species and sources do not combine");
    if (!Km) return fail(SWE_EINVAL, "Km is NULL");
    if (!(zeta > 0) || !std::isfinite(zeta)) return fail(SWE_EINVAL, "the relaxation time must be positive");
    if (!(alpha_L >= 0) || !(alpha_T >= 0) || !std::isfinite(alpha_L) || !std::isfinite(alpha_T))
        return fail(SWE_EINVAL, "dispersion coefficients must be >= 0");
    for (int c = 0; c < s->ns; c++)
        if (!(Km[c] >= 0) || !std::isfinite(Km[c])) return fail(SWE_EINVAL, "diffusivities must be >= 0");
    const HostMesh &M = s->m->H;
    const int64_t n = M.nc;
    for (int64_t k = 0; psi0 && k < (int64_t)2 * s->ns * n; k++)
        if (!std::isfinite(psi0[k])) return fail(SWE_EINVAL, "non-finite auxiliary variable");
    swe_status st = s->read_ctrl();
    if (st) return st;
    s->drop_graphs();
    s->drop_diffusion();
    const size_t es = s->prec == SWE_FP32 ? sizeof(float) : sizeof(double);
    const size_t cnt = (size_t)2 * s->ns * std::max<int64_t>(n, 1);
    s->P0 = s->mem.alloc(cnt * es);
    s->P1 = s->mem.alloc(cnt * es);
    if (!s->P0 || !s->P1) {
        s->drop_diffusion();
        return fail(SWE_ENOMEM, "device allocation failed (diffusion)");
    }
    // psi in device order, into both buffers
    auto up = [&](auto tag) -> swe_status {
        using T = decltype(tag);
        std::vector<T> p(cnt, T(0));
        for (int c = 0; c < s->ns && psi0; c++)
            for (int64_t i = 0; i < n; i++)
                for (int k = 0; k < 2; k++)
                    p[2 * ((size_t)c * n + M.inv[i]) + k] = T(psi0[2 * ((size_t)c * n + i) + k]);
        HIP_TRY(hipMemcpyAsync(s->P0, p.data(), cnt * es, hipMemcpyHostToDevice, s->stream()));
        HIP_TRY(hipMemcpyAsync(s->P1, p.data(), cnt * es, hipMemcpyHostToDevice, s->stream()));
        HIP_TRY(hipStreamSynchronize(s->stream()));
        return SWE_OK;
    };
    st = s->prec == SWE_FP32 ? up(float()) : up(double());
    if (st) {
        s->drop_diffusion();
        return st;
    }
    s->dKmax = 0.0;
    for (int c = 0; c < MAX_SPECIES; c++) {
        s->dKm[c] = c < s->ns ? Km[c] : 0.0;
        s->dKmax = std::max(s->dKmax, s->dKm[c]);
    }
    s->daL = alpha_L;
    s->daT = alpha_T;
    s->dzeta = zeta;
    s->diff = 1;
    s->bind_diffusion();
    return s->reseed_dt();
}

swe_status swe_state_read_psi(const swe_state *cs, double *psi) {
    swe_state *s = const_cast<swe_state *>(cs);
    if (!s || !psi) return fail(SWE_EINVAL, "state or psi is NULL");
    if (!s->diff) return SWE_OK;
    swe_status st = s->read_ctrl();
    if (st) return st;
    const HostMesh &M = s->m->H;
    const int64_t n = M.nc;
    const size_t cnt = (size_t)2 * s->ns * n;
    const void *src = s->lvl().cur ? s->P1 : s->P0;
    auto rd = [&](auto tag) -> swe_status {
        using T = decltype(tag);
        std::vector<T> p(cnt);
        HIP_TRY(hipMemcpyAsync(p.data(), src, cnt * sizeof(T), hipMemcpyDeviceToHost, s->stream()));
        HIP_TRY(hipStreamSynchronize(s->stream()));
        for (int c = 0; c < s->ns; c++)
            for (int64_t i = 0; i < n; i++)
                for (int k = 0; k < 2; k++)
                    psi[2 * ((size_t)c * n + i) + k] = double(p[2 * ((size_t)c * n + M.inv[i]) + k]);
        return SWE_OK;
    };
    return s->prec == SWE_FP32 ? rd(float()) : rd(double());
}

swe_status swe_state_set_sources(swe_state *s, const int32_t *cell_region, const swe_source *src, int32_t n_src) {
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (n_src > 0 && s->diff) return fail(SWE_EINVAL, "sources and diffusing species do not combine");
    if (n_src > 0 && s->morpho) return fail(SWE_EINVAL, "sources and a moving bed do not combine");
    if (n_src < 0 || n_src > MAX_BC) return fail(SWE_EINVAL, "between 0 and 64 sources");
    if (n_src > 0 && (!cell_region || !src)) return fail(SWE_EINVAL, "bad source list");
    const HostMesh &M = s->m->H;
    const int64_t n = M.nc;
    std::vector<BCdev> rec((size_t)std::max(n_src, 1));
    std::vector<double> series;
    std::vector<size_t> off((size_t)std::max(n_src, 1));
    for (int r = 0; r < n_src; r++) {
        const swe_source &X = src[r];
        if (X.mode < SWE_SRC_EXACT || X.mode > SWE_SRC_INFINITY) return fail(SWE_EINVAL, "unknown source mode");
        if (X.unit != SWE_SRC_DISCHARGE && X.unit != SWE_SRC_INTENSITY) return fail(SWE_EINVAL, "unknown source unit");
        if (X.n_pts < 0 || (X.mode != SWE_SRC_INFINITY && (X.n_pts < 1 || !X.t || !X.v)))
            return fail(SWE_EINVAL, "a source needs a series");
        for (int k = 0; k < X.n_pts; k++) {
            if (!std::isfinite(X.t[k]) || !std::isfinite(X.v[k])) return fail(SWE_EINVAL, "non-finite source series");
            if (k > 0 && !(X.t[k] > X.t[k - 1])) return fail(SWE_EINVAL, "source times must increase");
            if (X.mode == SWE_SRC_AVAILABLE && X.v[k] > 0.0) return fail(SWE_EINVAL, "only exact sources add water");
        }
        rec[r] = BCdev{X.mode, X.mode == SWE_SRC_INFINITY ? 0 : X.n_pts, 0.0, 0.0, nullptr, nullptr};
        off[r] = series.size();
        if (X.mode != SWE_SRC_INFINITY) {
            series.insert(series.end(), X.t, X.t + X.n_pts);
            series.insert(series.end(), X.v, X.v + X.n_pts);
        }
    }
    std::vector<int> dcell((size_t)n, -1);
    std::vector<std::vector<double>> areas((size_t)std::max(n_src, 1));
    for (int64_t i = 0; n_src > 0 && i < n; i++) {
        const int32_t r = cell_region[i];
        if (r < -1 || r >= n_src) return fail(SWE_EINVAL, "source region out of range");
        dcell[M.inv[i]] = r;
        if (r >= 0) areas[r].push_back(M.area[M.inv[i]]);
    }
    // factor from a series value to a rate in m/s; region areas summed in
    // ascending order, so the value does not depend on the numbering
    for (int r = 0; r < n_src; r++) {
        std::sort(areas[r].begin(), areas[r].end());
        double A = 0.0;
        for (double a : areas[r]) A += a;
        if (src[r].unit == SWE_SRC_DISCHARGE) {
            if (!(A > 0.0) && src[r].mode != SWE_SRC_INFINITY) return fail(SWE_EINVAL, "empty source region");
            rec[r].length = A > 0.0 ? 1.0 / A : 0.0;
        } else {
            rec[r].length = 1.0 / 3.6e6;  // mm/h -> m/s
        }
    }
    s->drop_graphs();
    s->drop_sources();
    if (n_src == 0) return SWE_OK;
    const int tiles = (int)((n + 127) / 128);  // the most tiles any tile size gives
    s->src_cell = (int *)s->mem.alloc(sizeof(int) * (size_t)n);
    s->srcs = (BCdev *)s->mem.alloc(sizeof(BCdev) * (size_t)n_src);
    s->src_series = (double *)s->mem.alloc(sizeof(double) * std::max<size_t>(series.size(), 1));
    s->src_acc = (double *)s->mem.alloc(2 * sizeof(double) * (size_t)std::max(tiles, 1));
    if (!s->src_cell || !s->srcs || !s->src_series || !s->src_acc) {
        s->drop_sources();
        return fail(SWE_ENOMEM, "device allocation failed (sources)");
    }
    for (int r = 0; r < n_src; r++)
        if (rec[r].npts) {
            rec[r].t = s->src_series + off[r];
            rec[r].Q = s->src_series + off[r] + rec[r].npts;
        }
    hipStream_t q = s->stream();
    std::vector<double> z((size_t)2 * std::max(tiles, 1), 0.0);
    auto up = [&]() -> swe_status {
        HIP_TRY(hipMemcpyAsync(s->src_cell, dcell.data(), sizeof(int) * dcell.size(), hipMemcpyHostToDevice, q));
        HIP_TRY(hipMemcpyAsync(s->srcs, rec.data(), sizeof(BCdev) * (size_t)n_src, hipMemcpyHostToDevice, q));
        if (!series.empty())
            HIP_TRY(hipMemcpyAsync(s->src_series, series.data(), sizeof(double) * series.size(),
                                   hipMemcpyHostToDevice, q));
        HIP_TRY(hipMemcpyAsync(s->src_acc, z.data(), sizeof(double) * z.size(), hipMemcpyHostToDevice, q));
        HIP_TRY(hipStreamSynchronize(q));
        return SWE_OK;
    };
    swe_status st = up();
    if (st) {
        s->drop_sources();
        return st;
    }
    s->nsrc = n_src;
    s->src_tiles = tiles;
    s->bind_sources();
    return SWE_OK;
}

swe_status swe_state_set_morpho(swe_state *s, const swe_morpho *mo, const double *z_rel) {
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (!mo) {
        s->drop_graphs();
        s->drop_morpho();
        return SWE_OK;
    }
    if (mo->closure < SWE_SED_MPM || mo->closure > SWE_SED_EH) return fail(SWE_EINVAL, "unknown sediment closure");
    auto fin = [](double x) { return std::isfinite(x); };
    if (!(mo->alpha >= 0) || !fin(mo->alpha) || !(mo->m > 0) || !fin(mo->m) || !(mo->thr >= 0) || !fin(mo->thr) ||
        !(mo->d_m > 0) || !fin(mo->d_m) || !(mo->s_rel > 1) || !fin(mo->s_rel) ||
        !(mo->porosity >= 0 && mo->porosity < 1))
        return fail(SWE_EINVAL, "bad sediment parameters");
    if (s->ns > 0 || s->nsrc > 0) return fail(SWE_EINVAL, "a moving bed excludes species and sources");
    if (s->p.limiter == SWE_LIMIT_DRAIN) return fail(SWE_EINVAL, "a moving bed and the draining-time limiter do not combine");
    const HostMesh &M = s->m->H;
    const int64_t n = M.nc;
    for (int64_t i = 0; z_rel && i < n; i++)
        if (!(z_rel[i] <= 0.0)) return fail(SWE_EINVAL, "the fixed bed lies at or below the bed (z_rel <= 0)");
    swe_status st = s->read_ctrl();
    if (st) return st;
    s->drop_graphs();
    s->drop_morpho();
    if (s->tile != SPECIES_TILE) {
        st = s->set_tile(SPECIES_TILE);
        if (st) return st;
    }
    const size_t es = s->prec == SWE_FP32 ? sizeof(float) : sizeof(double);
    const int nsl = std::max(s->nslots, 1);
    s->bslot_acc = (double *)s->mem.alloc(2 * sizeof(double) * (size_t)nsl);
    const size_t bclip_n = (size_t)2 * std::max(s->ngroups, 1);
    s->bclip_acc = (double *)s->mem.alloc(sizeof(double) * bclip_n);
    if (z_rel) s->zfix = s->mem.alloc(es * (size_t)n);
    if (!s->bslot_acc || !s->bclip_acc || (z_rel && !s->zfix)) {
        s->drop_morpho();
        return fail(SWE_ENOMEM, "device allocation failed (morphodynamics)");
    }
    hipStream_t q = s->stream();
    const void *cur = s->lvl().cur ? s->U1 : s->U0;
    auto up = [&](auto tag) -> swe_status {
        using T = decltype(tag);
        std::vector<double> z((size_t)2 * nsl, 0.0);
        HIP_TRY(hipMemcpyAsync(s->bslot_acc, z.data(), z.size() * sizeof(double), hipMemcpyHostToDevice, q));
        HIP_TRY(hipMemsetAsync(s->bclip_acc, 0, bclip_n * sizeof(double), q));
        if (z_rel) {
            std::vector<V4<T>> u((size_t)n);
            HIP_TRY(hipMemcpyAsync(u.data(), cur, u.size() * sizeof(V4<T>), hipMemcpyDeviceToHost, q));
            HIP_TRY(hipStreamSynchronize(q));
            std::vector<T> zf((size_t)n);
            for (int64_t i = 0; i < n; i++) {
                const int32_t d = M.inv[i];
                zf[d] = T(double(u[d].w) + z_rel[i]);
            }
            HIP_TRY(hipMemcpyAsync(s->zfix, zf.data(), zf.size() * sizeof(T), hipMemcpyHostToDevice, q));
        }
        HIP_TRY(hipStreamSynchronize(q));
        return SWE_OK;
    };
    st = s->prec == SWE_FP32 ? up(float()) : up(double());
    if (st) {
        s->drop_morpho();
        return st;
    }
    const double g = s->p.g;
    auto bind = [&](auto &I, auto tag) {
        using T = decltype(tag);
        I.morpho = 1;
        I.sclos = mo->closure;
        I.salpha = mo->alpha;
        I.sm = mo->m;
        I.sthr = mo->thr;
        // the same operations as the Shields number and K are written with
        I.srgd = (mo->s_rel - 1.0) * g * mo->d_m;
        I.sK = std::sqrt((mo->s_rel - 1.0) * g * mo->d_m * mo->d_m * mo->d_m);
        I.spor = mo->porosity;
        I.zfix = dev_ptr((const T *)s->zfix);
        I.bslot_acc = s->bslot_acc;
        I.bclip_acc = s->bclip_acc;
    };
    bind(s->inst32, float());
    bind(s->inst64, double());
    s->morpho = 1;
    return SWE_OK;
}

swe_status swe_state_read_bed(const swe_state *cs, double *z) {
    swe_state *s = const_cast<swe_state *>(cs);
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (!z) return SWE_OK;
    swe_status st = s->read_ctrl();
    if (st) return st;
    const HostMesh &M = s->m->H;
    const int64_t n = M.nc;
    const void *src = s->lvl().cur ? s->U1 : s->U0;
    auto rd = [&](auto tag) -> swe_status {
        using T = decltype(tag);
        std::vector<V4<T>> u((size_t)n);
        HIP_TRY(hipMemcpyAsync(u.data(), src, u.size() * sizeof(V4<T>), hipMemcpyDeviceToHost, s->stream()));
        HIP_TRY(hipStreamSynchronize(s->stream()));
        for (int64_t i = 0; i < n; i++) z[i] = double(u[M.inv[i]].w);
        return SWE_OK;
    };
    return s->prec == SWE_FP32 ? rd(float()) : rd(double());
}

swe_status swe_morpho_volume(const swe_state *cs, double *volume, double *bnd, double *clipped) {
    swe_state *s = const_cast<swe_state *>(cs);
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (!s->morpho) return fail(SWE_EINVAL, "the bed is not moving (no morphodynamics)");
    hipStream_t q = s->stream();
    if (s->prec == SWE_FP32)
        HIP_TRY(launch_bed_volume<float>(s->inst32, s->partials, s->mass_out, s->phase, q));
    else
        HIP_TRY(launch_bed_volume<double>(s->inst64, s->partials, s->mass_out, s->phase, q));
    HIP_TRY(launch_pair_sum(s->bslot_acc, std::max(s->nslots, 1), s->mass_out + 1, q));
    HIP_TRY(launch_pair_sum(s->bclip_acc, std::max(s->ngroups, 1), s->mass_out + 2, q));
    HIP_TRY(hipMemcpyAsync(s->hbuf + 1, s->mass_out, 3 * sizeof(double), hipMemcpyDeviceToHost, q));
    HIP_TRY(hipStreamSynchronize(q));
    if (volume) *volume = s->hbuf[1];
    if (bnd) *bnd = s->hbuf[2];
    if (clipped) *clipped = s->hbuf[3];
    return SWE_OK;
}

swe_status swe_source_volume(const swe_state *cs, double *volume) {
    swe_state *s = const_cast<swe_state *>(cs);
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (!volume) return SWE_OK;
    *volume = 0.0;
    if (s->nsrc == 0) return SWE_OK;
    HIP_TRY(launch_pair_sum(s->src_acc, s->src_tiles, s->mass_out, s->stream()));
    HIP_TRY(hipMemcpyAsync(s->hbuf + 1, s->mass_out, sizeof(double), hipMemcpyDeviceToHost, s->stream()));
    HIP_TRY(hipStreamSynchronize(s->stream()));
    *volume = s->hbuf[1];
    return SWE_OK;
}

swe_status swe_state_read_scalars(const swe_state *cs, double *q) {
    swe_state *s = const_cast<swe_state *>(cs);
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (!q || s->ns == 0) return SWE_OK;
    swe_status st = s->read_ctrl();
    if (st) return st;
    const HostMesh &M = s->m->H;
    const int64_t n = M.nc;
    const void *src = s->lvl().cur ? s->Q1 : s->Q0;
    auto rd = [&](auto tag) -> swe_status {
        using T = decltype(tag);
        std::vector<T> v((size_t)s->ns * n);
        HIP_TRY(hipMemcpyAsync(v.data(), src, v.size() * sizeof(T), hipMemcpyDeviceToHost, s->stream()));
        HIP_TRY(hipStreamSynchronize(s->stream()));
        for (int c = 0; c < s->ns; c++)
            for (int64_t i = 0; i < n; i++) q[(size_t)c * n + i] = double(v[(size_t)c * n + M.inv[i]]);
        return SWE_OK;
    };
    return s->prec == SWE_FP32 ? rd(float()) : rd(double());
}

swe_status swe_scalar_mass(const swe_state *cs, double *mass, double *bnd_flux, double *clipped) {
    swe_state *s = const_cast<swe_state *>(cs);
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (s->ns == 0) return SWE_OK;
    hipStream_t q = s->stream();
    for (int c = 0; c < s->ns; c++) {
        if (s->prec == SWE_FP32)
            HIP_TRY(launch_species_mass<float>(s->inst32, c, s->partials, s->mass_out, s->nslots, s->phase, q));
        else
            HIP_TRY(launch_species_mass<double>(s->inst64, c, s->partials, s->mass_out, s->nslots, s->phase, q));
        HIP_TRY(hipMemcpyAsync(s->hbuf + 1, s->mass_out, 2 * sizeof(double), hipMemcpyDeviceToHost, q));
        HIP_TRY(hipStreamSynchronize(q));
        if (mass) mass[c] = s->hbuf[1];
        if (bnd_flux) bnd_flux[c] = s->hbuf[2];
    }
    if (clipped) {
        const int ng = std::max(s->ngroups, 1);
        for (int c = 0; c < s->ns; c++) {
            HIP_TRY(launch_pair_sum(s->sclip_acc + (size_t)2 * c * ng, ng, s->mass_out, q));
            HIP_TRY(hipMemcpyAsync(s->hbuf + 1, s->mass_out, sizeof(double), hipMemcpyDeviceToHost, q));
            HIP_TRY(hipStreamSynchronize(q));
            clipped[c] = s->hbuf[1];
        }
    }
    return SWE_OK;
}

swe_status swe_autotune(swe_state *s, int32_t k, int32_t *block_size) {
    if (!s) return fail(SWE_EINVAL, "state is NULL");
    if (s->ns > 0 || s->nsrc > 0 || s->morpho) {
        // the species and Exner steps have one tile size; a state with
        // sources keeps its tile (its source tally is kept per tile)
        if (block_size) *block_size = s->tile;
        return SWE_OK;
    }
    if (k < 1) k = 8;
    swe_status st = s->read_ctrl();
    if (st) return st;
    const Ctrl saved = *s->hctrl;
    const int saved_phase = s->phase;
    // the boundary records too: a trial step may lower a dynamic wall's
    // collapse time (its collapse depth reached)
    std::vector<BCdev> keepB((size_t)std::max(s->n_bc, 1));
    HIP_TRY(hipMemcpyAsync(keepB.data(), s->bcs, sizeof(BCdev) * keepB.size(), hipMemcpyDeviceToHost, s->stream()));
    HIP_TRY(hipStreamSynchronize(s->stream()));
    const int64_t n = s->m->H.nc;
    const size_t ub = (size_t)n * vec4_bytes(s->prec);
    const size_t ab = 2 * sizeof(double) * std::max(s->nslots, 1);
    const size_t cb = 2 * sizeof(double) * std::max(s->ngroups, 1);
    const size_t lb = s->prec == SWE_FP32 ? (size_t)n * sizeof(int16_t) : 0;
    void *keepU = s->mem.alloc(ub + lb);  // the state, then (FP32) the low parts of the surface
    void *keepA = s->mem.alloc(ab);
    void *keepC = s->mem.alloc(cb);
    if (!keepU || !keepA || !keepC) {
        s->mem.release(keepU);
        s->mem.release(keepA);
        s->mem.release(keepC);
        return fail(SWE_ENOMEM, "device allocation failed (autotune)");
    }
    void *cur = saved.s[saved_phase].cur ? s->U1 : s->U0;
    void *curL = saved.s[saved_phase].cur ? (void *)s->L1 : (void *)s->L0;
    hipStream_t q = s->stream();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        s->mem.release(keepU);
        s->mem.release(keepA);
        s->mem.release(keepC);
    };
    auto restore = [&]() -> swe_status {
        *s->hctrl = saved;
        s->phase = saved_phase;
        HIP_TRY(hipMemcpyAsync(cur, keepU, ub, hipMemcpyDeviceToDevice, q));
        if (lb) HIP_TRY(hipMemcpyAsync(curL, (char *)keepU + ub, lb, hipMemcpyDeviceToDevice, q));
        HIP_TRY(hipMemcpyAsync(s->slot_acc, keepA, ab, hipMemcpyDeviceToDevice, q));
        HIP_TRY(hipMemcpyAsync(s->clip_acc, keepC, cb, hipMemcpyDeviceToDevice, q));
        HIP_TRY(hipMemcpyAsync(s->ctrl, s->hctrl, sizeof(Ctrl), hipMemcpyHostToDevice, q));
        HIP_TRY(hipMemcpyAsync(s->bcs, keepB.data(), sizeof(BCdev) * keepB.size(), hipMemcpyHostToDevice, q));
        HIP_TRY(hipStreamSynchronize(q));
        return SWE_OK;
    };
    st = [&]() -> swe_status {
        HIP_TRY(hipMemcpyAsync(keepU, cur, ub, hipMemcpyDeviceToDevice, q));
        if (lb) HIP_TRY(hipMemcpyAsync((char *)keepU + ub, curL, lb, hipMemcpyDeviceToDevice, q));
        HIP_TRY(hipMemcpyAsync(keepA, s->slot_acc, ab, hipMemcpyDeviceToDevice, q));
        HIP_TRY(hipMemcpyAsync(keepC, s->clip_acc, cb, hipMemcpyDeviceToDevice, q));
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        // each tile size timed in AUTOTUNE_ROUNDS interleaved rounds (so a
        // drift of the clock or of the other work on the device hits every
        // size alike); a size's figure is its fastest round
        float tbest[3] = {std::numeric_limits<float>::infinity(), std::numeric_limits<float>::infinity(),
                          std::numeric_limits<float>::infinity()};
        for (int round = 0; round < AUTOTUNE_ROUNDS; round++)
            for (int ti = 0; ti < 3; ti++) {
                const int b = TILES[ti];
                swe_status r = restore();
                if (r) return r;
                r = s->set_tile(b);
                if (r) return r;
                r = s->set_t_end(std::numeric_limits<double>::infinity());
                if (r) return r;
                HIP_TRY(s->launch_one());
                HIP_TRY(hipEventRecord(e0, q));
                for (int i = 0; i < k; i++) HIP_TRY(s->launch_one());
                HIP_TRY(hipEventRecord(e1, q));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                r = s->read_ctrl();
                if (r) return r;
                if (s->hctrl->flags == 0 && ms < tbest[ti]) tbest[ti] = ms;
            }
        float best = std::numeric_limits<float>::infinity();
        int bb = s->tile;
        for (int ti = 0; ti < 3; ti++)
            if (tbest[ti] < best) {
                best = tbest[ti];
                bb = TILES[ti];
            }
        swe_status r = s->set_tile(bb);
        if (r) return r;
        return restore();
    }();
    cleanup();
    if (st) return st;
    if (block_size) *block_size = s->tile;
    return SWE_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
struct swe_batch {
    DevMem mem;
    int prec = SWE_FP32;
    int64_t budget = 0;
    std::vector<swe_state *> members;
    std::vector<double> t_end;
    std::vector<char> finished;  // members known to be done (excluded from the work list)
    void *insts = nullptr;
    size_t insts_cap = 0;
    int2 *tiles = nullptr;
    size_t tiles_cap = 0;
    int ntiles = 0;
    int tile = 256, grid = 0;
    int phase = 0;  // launches so far mod 3; every member is aligned to it
    bool dirty = true;
    bool iw = false;  // some running member has internal walls
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
    int g_k = 0;
    ~swe_batch() {
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        mem.release(insts);
        mem.release(tiles);
    }
    void drop_graphs() {
        for (auto &g : gexec)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    }
    hipStream_t stream() const { return mem.stream(); }
    int64_t footprint() const {
        int64_t f = 0;
        for (auto *s : members)
            if (s) f += swe_state_footprint(s->m, s->prec);
        return f;
    }
    hipError_t launch(hipStream_t s, int ph) {
        return prec == SWE_FP32
                   ? launch_step_batched<float>((const Inst<float> *)insts, tiles, ntiles, grid, tile, iw, ph, s)
                   : launch_step_batched<double>((const Inst<double> *)insts, tiles, ntiles, grid, tile, iw, ph, s);
    }
    // work list of the members that are still running
    swe_status rebuild() {
        std::vector<Inst<float>> i32;
        std::vector<Inst<double>> i64;
        std::vector<int2> tl;
        bool any_iw = false;
        for (size_t m = 0; m < members.size(); m++) {
            swe_state *s = members[m];
            if (!s || finished[m]) continue;
            any_iw = any_iw || s->inst32.iw_on;
            const int idx = prec == SWE_FP32 ? (int)i32.size() : (int)i64.size();
            swe_status st = prec == SWE_FP32 ? s->m->ensure_tiles<float>(prec, tile)
                                             : s->m->ensure_tiles<double>(prec, tile);
            if (st) return st;
            const TileGeom &tg = s->m->geom[prec][tile_index(tile)];
            const int nt = tg.ntiles;
            if (prec == SWE_FP32) {
                Inst<float> I = s->inst32;
                tg.bind(I);
                i32.push_back(I);
            } else {
                Inst<double> I = s->inst64;
                tg.bind(I);
                i64.push_back(I);
            }
            for (int t = 0; t < nt; t++) tl.push_back(make_int2(idx, t));
        }
        const size_t nb = prec == SWE_FP32 ? i32.size() * sizeof(Inst<float>) : i64.size() * sizeof(Inst<double>);
        if (nb > insts_cap) {
            mem.release(insts);
            insts_cap = std::max(nb, insts_cap * 2);
            insts = mem.alloc(insts_cap);
            if (!insts) return fail(SWE_ENOMEM, "device allocation failed (batch)");
        }
        if (tl.size() * sizeof(int2) > tiles_cap) {
            mem.release(tiles);
            tiles_cap = std::max(tl.size() * sizeof(int2), tiles_cap * 2);
            tiles = (int2 *)mem.alloc(tiles_cap);
            if (!tiles) return fail(SWE_ENOMEM, "device allocation failed (batch)");
        }
        if (nb)
            HIP_TRY(hipMemcpyAsync(insts, prec == SWE_FP32 ? (const void *)i32.data() : (const void *)i64.data(), nb,
                                   hipMemcpyHostToDevice, stream()));
        if (!tl.empty())
            HIP_TRY(hipMemcpyAsync(tiles, tl.data(), tl.size() * sizeof(int2), hipMemcpyHostToDevice, stream()));
        HIP_TRY(hipStreamSynchronize(stream()));
        ntiles = (int)tl.size();
        iw = any_iw;
        grid = prec == SWE_FP32 ? batched_grid<float>(tile, iw) : batched_grid<double>(tile, iw);
        if (grid < 1) grid = 1;
        drop_graphs();
        dirty = false;
        return SWE_OK;
    }
    // k persistent launches starting at the current phase, captured once
    swe_status graph(int k) {
        if (g_k != k) {
            drop_graphs();
            g_k = k;
        }
        if (gexec[phase] || ntiles == 0) return SWE_OK;
        if (!cap) HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t gr = nullptr;
        HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < k; i++) {
            hipError_t e = launch(cap, (phase + i) % 3);
            if (e != hipSuccess) {
                hipGraph_t dummy = nullptr;
                (void)hipStreamEndCapture(cap, &dummy);
                if (dummy) (void)hipGraphDestroy(dummy);
                return fail(SWE_EDEVICE, std::string("batch capture: ") + hipGetErrorString(e));
            }
        }
        HIP_TRY(hipStreamEndCapture(cap, &gr));
        hipError_t e = hipGraphInstantiate(&gexec[phase], gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return fail(SWE_EDEVICE, std::string("batch graph: ") + hipGetErrorString(e));
        return SWE_OK;
    }
};

extern "C" {

swe_status swe_batch_create(int32_t precision, int64_t budget_bytes, const swe_device *dev, swe_batch **out) {
    if (!out) return fail(SWE_EINVAL, "out is NULL");
    *out = nullptr;
    if (precision != SWE_FP32 && precision != SWE_FP64) return fail(SWE_EINVAL, "unknown precision");
    if (budget_bytes < 0) return fail(SWE_EINVAL, "negative budget");
    swe_batch *b = new (std::nothrow) swe_batch();
    if (!b) return fail(SWE_ENOMEM, "out of host memory");
    b->mem.set(dev);
    b->prec = precision;
    b->budget = budget_bytes;
    *out = b;
    return SWE_OK;
}

void swe_batch_destroy(swe_batch *b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream());
    delete b;
}

int64_t swe_batch_footprint(const swe_batch *b) { return b ? b->footprint() : 0; }

swe_status swe_batch_add(swe_batch *b, swe_state *s, double t_end, int32_t *slot) {
    if (!b || !s) return fail(SWE_EINVAL, "batch or state is NULL");
    if (s->prec != b->prec) return fail(SWE_EINVAL, "state precision differs from the batch");
    if (s->ns > 0) return fail(SWE_EINVAL, "states with passive species are not batched");
    if (s->nsrc > 0) return fail(SWE_EINVAL, "states with sources are not batched");
    if (s->morpho) return fail(SWE_EINVAL, "states with a moving bed are not batched");
    if (s->p.limiter == SWE_LIMIT_DRAIN) return fail(SWE_EINVAL, "states with the draining-time limiter are not batched");
    if (s->stream() != b->stream()) return fail(SWE_EINVAL, "state and batch must use the same stream");
    if (std::isnan(t_end)) return fail(SWE_EINVAL, "t_end is NaN");
    for (auto *x : b->members)
        if (x == s) return fail(SWE_EINVAL, "state already in the batch");
    const int64_t f = swe_state_footprint(s->m, s->prec);
    if (b->budget > 0 && b->footprint() + f > b->budget) return fail(SWE_EBUDGET, "batch footprint budget exceeded");
    swe_status st = s->realign(b->phase);
    if (st) return st;
    st = s->set_t_end(t_end);
    if (st) return st;
    st = s->read_ctrl();
    if (st) return st;
    int idx = -1;
    for (size_t i = 0; i < b->members.size(); i++)
        if (!b->members[i]) {
            idx = (int)i;
            break;
        }
    if (idx < 0) {
        idx = (int)b->members.size();
        b->members.push_back(nullptr);
        b->t_end.push_back(0);
        b->finished.push_back(0);
    }
    b->members[idx] = s;
    b->t_end[idx] = t_end;
    b->finished[idx] = !(s->lvl().t < t_end) || s->hctrl->flags != 0;
    b->dirty = true;
    if (slot) *slot = idx;
    return SWE_OK;
}

swe_status swe_batch_remove(swe_batch *b, int32_t slot) {
    if (!b || slot < 0 || slot >= (int32_t)b->members.size() || !b->members[slot])
        return fail(SWE_EINVAL, "no such batch member");
    (void)hipStreamSynchronize(b->stream());
    b->members[slot] = nullptr;
    b->finished[slot] = 0;
    b->dirty = true;
    return SWE_OK;
}

swe_status swe_batch_launch(swe_batch *b, int32_t k) {
    if (!b || k < 1) return fail(SWE_EINVAL, "bad batch launch");
    if (b->dirty) {
        swe_status st = b->rebuild();
        if (st) return st;
    }
    if (b->ntiles == 0) return SWE_OK;
    swe_status st = b->graph(k);
    if (st) return st;
    HIP_TRY(hipGraphLaunch(b->gexec[b->phase], b->stream()));
    b->phase = (b->phase + k) % 3;
    // every member in the work list stepped (or carried its level) k times
    for (size_t i = 0; i < b->members.size(); i++)
        if (b->members[i] && !b->finished[i]) b->members[i]->phase = b->phase;
    return SWE_OK;
}

swe_status swe_batch_step(swe_batch *b, int32_t k, int32_t *n_active) {
    swe_status st = swe_batch_launch(b, k);
    if (st) return st;
    int active = 0;
    for (size_t i = 0; i < b->members.size(); i++) {
        swe_state *s = b->members[i];
        if (!s) continue;
        HIP_TRY(hipMemcpyAsync(s->hctrl, s->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, b->stream()));
    }
    HIP_TRY(hipStreamSynchronize(b->stream()));
    for (size_t i = 0; i < b->members.size(); i++) {
        swe_state *s = b->members[i];
        if (!s) continue;
        const bool done = !(s->lvl().t < b->t_end[i]) || s->hctrl->flags != 0;
        if (done && !b->finished[i]) {
            b->finished[i] = 1;
            b->dirty = true;
        }
        if (!done) active++;
    }
    if (n_active) *n_active = active;
    return SWE_OK;
}

swe_status swe_batch_step_noalloc(swe_state *const *states, const double *t_end, int32_t n, int32_t k,
                                  int32_t *n_active) {
    if (n < 1 || n > NOALLOC_MAX_STATES) return fail(SWE_EINVAL, "between 1 and 64 states");
    if (!states || !t_end) return fail(SWE_EINVAL, "states or t_end is NULL");
    if (k < 1) return fail(SWE_EINVAL, "k must be positive");
    swe_state *s0 = states[0];
    if (!s0) return fail(SWE_EINVAL, "state is NULL");
    const int prec = s0->prec, tile = s0->tile;
    const int ti = tile_index(tile);
    int64_t total = 0;
    for (int32_t i = 0; i < n; i++) {
        swe_state *s = states[i];
        if (!s) return fail(SWE_EINVAL, "state is NULL");
        if (s->prec != prec) return fail(SWE_EINVAL, "states of one call share their precision");
        if (s->tile != tile) return fail(SWE_EINVAL, "states of one call share their tile size");
        if (s->stream() != s0->stream()) return fail(SWE_EINVAL, "states of one call share their stream");
        if (s->ns > 0 || s->nsrc > 0 || s->morpho || s->p.limiter == SWE_LIMIT_DRAIN)
            return fail(SWE_EINVAL, "states with species, sources, a moving bed or the limiter are not batched");
        if (std::isnan(t_end[i])) return fail(SWE_EINVAL, "t_end is NaN");
        for (int32_t j = 0; j < i; j++)
            if (states[j] == s) return fail(SWE_EINVAL, "a state is given twice");
        total += s->m->geom[prec][ti].ntiles;
    }
    if (total > NOALLOC_MAX_TILES) return fail(SWE_EINVAL, "more than 262144 tiles in one call");
    void *scr = nullptr;
    HIP_TRY(noalloc_scratch(&scr));
    hipStream_t q = s0->stream();
    const int phase = s0->phase;
    for (int32_t i = 0; i < n; i++) {
        swe_status st = states[i]->realign(phase);
        if (st) return st;
        st = states[i]->set_t_end(t_end[i]);
        if (st) return st;
    }
    // the work list, staged in host arrays of the scratch's fixed size
    static std::mutex mu;
    static Inst<float> h32[NOALLOC_MAX_STATES];
    static Inst<double> h64[NOALLOC_MAX_STATES];
    static int2 htiles[NOALLOC_MAX_TILES];
    int ntiles = 0;
    bool iw = false;
    {
        std::lock_guard<std::mutex> lock(mu);
        for (int32_t i = 0; i < n; i++) {
            iw = iw || states[i]->inst32.iw_on;
            h32[i] = states[i]->inst32;
            h64[i] = states[i]->inst64;
            const int nt = states[i]->m->geom[prec][ti].ntiles;
            for (int t = 0; t < nt; t++) htiles[ntiles++] = make_int2(i, t);
        }
        char *base = (char *)scr;
        if (prec == SWE_FP32)
            HIP_TRY(hipMemcpyAsync(base, h32, n * sizeof(Inst<float>), hipMemcpyHostToDevice, q));
        else
            HIP_TRY(hipMemcpyAsync(base, h64, n * sizeof(Inst<double>), hipMemcpyHostToDevice, q));
        if (ntiles)
            HIP_TRY(hipMemcpyAsync(base + NOALLOC_INST_BYTES, htiles, ntiles * sizeof(int2), hipMemcpyHostToDevice, q));
        HIP_TRY(hipStreamSynchronize(q));
    }
    const int2 *dtiles = (const int2 *)((char *)scr + NOALLOC_INST_BYTES);
    int grid = prec == SWE_FP32 ? batched_grid<float>(tile, iw) : batched_grid<double>(tile, iw);
    if (grid < 1) grid = 1;
    for (int32_t i = 0; i < k; i++) {
        const int ph = (phase + i) % 3;
        if (prec == SWE_FP32)
            HIP_TRY(launch_step_batched<float>((const Inst<float> *)scr, dtiles, ntiles, grid, tile, iw, ph, q));
        else
            HIP_TRY(launch_step_batched<double>((const Inst<double> *)scr, dtiles, ntiles, grid, tile, iw, ph, q));
    }
    const int after = (phase + k) % 3;
    for (int32_t i = 0; i < n; i++) {
        states[i]->phase = after;
        HIP_TRY(hipMemcpyAsync(states[i]->hctrl, states[i]->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, q));
    }
    HIP_TRY(hipStreamSynchronize(q));
    int active = 0;
    swe_status err = SWE_OK;
    for (int32_t i = 0; i < n; i++) {
        const int flags = states[i]->hctrl->flags;
        if (flags && !err) err = check_flags(flags);
        if (!flags && states[i]->lvl().t < t_end[i]) active++;
    }
    if (n_active) *n_active = active;
    return err;
}

swe_status swe_batch_autotune(swe_batch *b, int32_t k, int32_t *block_size) {
    if (!b) return fail(SWE_EINVAL, "batch is NULL");
    if (k < 1) k = 4;
    if (b->dirty) {
        swe_status st = b->rebuild();
        if (st) return st;
    }
    // every running member's current state vector, boundary accumulators,
    // boundary records (a trial step may lower a dynamic wall's collapse
    // time), control block and launch phase, restored after each trial
    struct Saved {
        swe_state *s;
        void *U = nullptr, *A = nullptr, *C = nullptr, *cur = nullptr, *curL = nullptr;
        size_t ub = 0, ab = 0, cb = 0, lb = 0;
        Ctrl c{};
        int phase = 0;
        std::vector<BCdev> B;
    };
    std::vector<Saved> sv;
    hipStream_t q = b->stream();
    const int bphase = b->phase;
    auto release = [&]() {
        for (auto &x : sv) {
            x.s->mem.release(x.U);
            x.s->mem.release(x.A);
            x.s->mem.release(x.C);
        }
    };
    for (size_t i = 0; i < b->members.size(); i++) {
        swe_state *s = b->members[i];
        if (!s || b->finished[i]) continue;
        swe_status st = s->read_ctrl();
        if (st) {
            release();
            return st;
        }
        Saved x;
        x.s = s;
        x.c = *s->hctrl;
        x.phase = s->phase;
        x.cur = x.c.s[s->phase].cur ? s->U1 : s->U0;
        x.curL = x.c.s[s->phase].cur ? (void *)s->L1 : (void *)s->L0;
        x.lb = s->prec == SWE_FP32 ? (size_t)s->m->H.nc * sizeof(int16_t) : 0;
        x.ub = (size_t)s->m->H.nc * vec4_bytes(s->prec);
        x.ab = 2 * sizeof(double) * std::max(s->nslots, 1);
        x.cb = 2 * sizeof(double) * std::max(s->ngroups, 1);
        x.U = s->mem.alloc(x.ub + x.lb);
        x.A = s->mem.alloc(x.ab);
        x.C = s->mem.alloc(x.cb);
        sv.push_back(x);
        if (!x.U || !x.A || !x.C) {
            release();
            return fail(SWE_ENOMEM, "device allocation failed (batch autotune)");
        }
        HIP_TRY(hipMemcpyAsync(x.U, x.cur, x.ub, hipMemcpyDeviceToDevice, q));
        if (x.lb) HIP_TRY(hipMemcpyAsync((char *)x.U + x.ub, x.curL, x.lb, hipMemcpyDeviceToDevice, q));
        HIP_TRY(hipMemcpyAsync(x.A, s->slot_acc, x.ab, hipMemcpyDeviceToDevice, q));
        HIP_TRY(hipMemcpyAsync(x.C, s->clip_acc, x.cb, hipMemcpyDeviceToDevice, q));
        sv.back().B.resize((size_t)std::max(s->n_bc, 1));
        HIP_TRY(hipMemcpyAsync(sv.back().B.data(), s->bcs, sizeof(BCdev) * sv.back().B.size(), hipMemcpyDeviceToHost, q));
    }
    HIP_TRY(hipStreamSynchronize(q));
    auto restore = [&]() -> swe_status {
        for (auto &x : sv) {
            *x.s->hctrl = x.c;
            x.s->phase = x.phase;
            HIP_TRY(hipMemcpyAsync(x.cur, x.U, x.ub, hipMemcpyDeviceToDevice, q));
            if (x.lb) HIP_TRY(hipMemcpyAsync(x.curL, (char *)x.U + x.ub, x.lb, hipMemcpyDeviceToDevice, q));
            HIP_TRY(hipMemcpyAsync(x.s->slot_acc, x.A, x.ab, hipMemcpyDeviceToDevice, q));
            HIP_TRY(hipMemcpyAsync(x.s->clip_acc, x.C, x.cb, hipMemcpyDeviceToDevice, q));
            HIP_TRY(hipMemcpyAsync(x.s->ctrl, x.s->hctrl, sizeof(Ctrl), hipMemcpyHostToDevice, q));
            HIP_TRY(hipMemcpyAsync(x.s->bcs, x.B.data(), sizeof(BCdev) * x.B.size(), hipMemcpyHostToDevice, q));
        }
        HIP_TRY(hipStreamSynchronize(q));
        b->phase = bphase;
        return SWE_OK;
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const int tile0 = b->tile;
    swe_status st = [&]() -> swe_status {
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        float tbest[3] = {std::numeric_limits<float>::infinity(), std::numeric_limits<float>::infinity(),
                          std::numeric_limits<float>::infinity()};
        for (int round = 0; round < AUTOTUNE_ROUNDS; round++)
        for (int ti = 0; ti < 3; ti++) {
            const int t = TILES[ti];
            swe_status r = restore();
            if (r) return r;
            b->tile = t;
            r = b->rebuild();
            if (r) return r;
            if (b->ntiles == 0) break;
            HIP_TRY(b->launch(q, b->phase));
            b->phase = (b->phase + 1) % 3;
            HIP_TRY(hipEventRecord(e0, q));
            for (int i = 0; i < k; i++) {
                HIP_TRY(b->launch(q, b->phase));
                b->phase = (b->phase + 1) % 3;
            }
            HIP_TRY(hipEventRecord(e1, q));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            bool ok = true;
            for (auto &x : sv) {
                r = x.s->read_ctrl();
                if (r) return r;
                ok = ok && x.s->hctrl->flags == 0;
            }
            if (ok && ms < tbest[ti]) tbest[ti] = ms;
        }
        float best = std::numeric_limits<float>::infinity();
        int bt = tile0;
        for (int ti = 0; ti < 3; ti++)
            if (tbest[ti] < best) {
                best = tbest[ti];
                bt = TILES[ti];
            }
        swe_status r = restore();
        if (r) return r;
        b->tile = bt;
        return b->rebuild();
    }();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    release();
    if (st) {
        b->tile = tile0;
        b->dirty = true;
        return st;
    }
    if (block_size) *block_size = b->tile;
    return SWE_OK;
}

swe_status swe_batch_poll(swe_batch *b, int32_t slot, int32_t *done, int32_t *error, double *t, int64_t *steps) {
    if (!b || slot < 0 || slot >= (int32_t)b->members.size() || !b->members[slot])
        return fail(SWE_EINVAL, "no such batch member");
    swe_state *s = b->members[slot];
    const CtrlSlot &c = s->lvl();
    const int flags = s->hctrl->flags;
    if (done) *done = !(c.t < b->t_end[slot]) || flags != 0;
    if (error) *error = flags ? check_flags(flags) : 0;
    if (t) *t = c.t;
    if (steps) *steps = c.steps;
    return SWE_OK;
}

}  // extern "C"
