// HIP kernels of the shallow-water step for gfx950 (CDNA4, wave64).
//
// One thread updates one cell (or `CPT` cells) of a Hilbert-ordered mesh: it
// gathers its three neighbours' (H, qx, qy, z), evaluates the three edge
// fluxes itself (cell-centric: no atomics, no edge buffers, every thread
// writes only its own cell), applies the conservative update (paper:
// eq. hydrodynamicupdateformula), the Manning friction split (eq.
// friction_closure, Table friction_closure) and the positivity clip, and
// computes the CFL candidate of its new state (eq. CFL_condition).  A wave64
// shuffle, an LDS pass and one 64-bit atomic min per block give the grid-wide
// minimum; the last block to arrive advances time on the device, so a run of
// steps needs no host round trip and can be captured in one hipGraph.
//
// Interior edges are evaluated by both adjacent cells.  Both evaluate the
// flux in the edge's canonical orientation (left = the cell with the smaller
// original index) from bitwise-identical inputs, so the mass flux one cell
// loses is exactly the flux the other gains.
#include "swe_internal.h"

#include <math.h>

namespace swe {

namespace {

constexpr double H_DRY = 1e-12;  // reconstructed depths below this are dry

template <typename T> __device__ __forceinline__ V4<T> make4(T a, T b, T c, T d);
template <> __device__ __forceinline__ float4 make4<float>(float a, float b, float c, float d) {
    return make_float4(a, b, c, d);
}
template <> __device__ __forceinline__ double4 make4<double>(double a, double b, double c, double d) {
    return make_double4(a, b, c, d);
}

template <typename T> __device__ __forceinline__ T pow73(T h);
template <> __device__ __forceinline__ double pow73<double>(double h) { return pow(h, 7.0 / 3.0); }
template <> __device__ __forceinline__ float pow73<float>(float h) { return exp2f((7.0f / 3.0f) * log2f(h)); }

// Division and square root.  FP64 uses IEEE-correct operations so that every
// wet/dry decision matches an FP64 reference bit for bit; FP32 uses the
// hardware reciprocal and square root (about 1 ulp), which is far inside the
// single-precision error budget of the method.
__device__ __forceinline__ double qdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double qsqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float qsqrt(float a) { return __builtin_amdgcn_sqrtf(a); }

// Edge length and unit normal from l*n.  FP64: the IEEE square root and two
// divisions (matching the oracle); FP32: one reciprocal square root.
__device__ __forceinline__ void edge_normal(double lx, double ly, double &l, double &nx, double &ny) {
    l = sqrt(lx * lx + ly * ly);
    nx = lx / l;
    ny = ly / l;
}
__device__ __forceinline__ void edge_normal(float lx, float ly, float &l, float &nx, float &ny) {
    const float s = lx * lx + ly * ly;
    const float r = __builtin_amdgcn_rsqf(s);
    l = s * r;
    nx = lx * r;
    ny = ly * r;
}

// HLLC flux (Toro 1994) in the frame of the edge normal, for reconstructed
// depths hL, hR >= 0.  Wave speeds: two-rarefaction estimates with c* >= 0
// when both sides are wet, dry-bed speeds u -+ 2c when one side is dry.  The
// flux is F_K + S_K (U*_K - U_K) on the side K the contact speed S* selects,
// with U*_K = h_K (S_K - u_K)/(S_K - S*) (1, S*, ut_K), or the physical flux
// F_K when all waves move one way (or the states are identical); two dry
// sides give zero.  The side is chosen first and the formulas evaluated once,
// so neighbouring edges with opposite flow directions do not diverge.
template <typename T>
__device__ __forceinline__ void hllc(T hL, T unL, T utL, T hR, T unR, T utR, T g, T &F0, T &F1, T &F2) {
    const T zero = T(0), half = T(0.5);
    if (!(hL > zero) && !(hR > zero)) {
        F0 = zero; F1 = zero; F2 = zero;
        return;
    }
    const bool ident = hL == hR && unL == unR && utL == utR;
    const T cL = qsqrt(g * hL), cR = qsqrt(g * hR);
    const bool dryL = !(hL > zero), dryR = !(hR > zero);
    const T a = half * (cL + cR) + T(0.25) * (unL - unR);
    const T us = half * (unL + unR) + cL - cR;
    const T cs = a > zero ? a : zero;
    const T SL = dryL ? unR - T(2) * cR : (dryR ? unL - cL : fmin(unL - cL, us - cs));
    const T SR = dryL ? unR + cR : (dryR ? unL + T(2) * cL : fmax(unR + cR, us + cs));
    const T Ss = qdiv(SL * hR * (unR - SR) - SR * hL * (unL - SL), hR * (unR - SR) - hL * (unL - SL));
    // side K whose flux (and star state) is used
    const bool left = ident || zero <= SL || (!(SR <= zero) && zero <= Ss);
    const bool star = !ident && !(zero <= SL) && !(SR <= zero);
    const T hK = left ? hL : hR, unK = left ? unL : unR, utK = left ? utL : utR, SK = left ? SL : SR;
    F0 = hK * unK;
    F1 = hK * unK * unK + half * g * hK * hK;
    F2 = hK * unK * utK;
    if (star) {
        const T f = qdiv(hK * (SK - unK), SK - Ss);
        F0 = F0 + SK * (f - hK);
        F1 = F1 + SK * (f * Ss - hK * unK);
        F2 = F2 + SK * (f * utK - hK * utK);
    }
}

// Hydrograph value at time t (linear, held constant past the ends).
__device__ __forceinline__ double hydrograph(const BCdev &b, double t) {
    const double *ts = b.t, *Qs = b.Q;
    int n = b.npts;
    if (t <= ts[0]) return Qs[0];
    if (t >= ts[n - 1]) return Qs[n - 1];
    int k = 0;
    while (ts[k + 1] < t) k++;
    double w = (t - ts[k]) / (ts[k + 1] - ts[k]);
    return Qs[k] + w * (Qs[k + 1] - Qs[k]);
}

// Inflow uniform(Q, S): unit discharge q = Q / length entering with the
// Manning normal depth (n q / sqrt(S))^(3/5) of the adjacent cell's n.
// Returns false when Q <= 0 (the edge then behaves as a wall).
__device__ __forceinline__ bool inflow_ghost(const BCdev &b, double t, double gn2, double g, double &hg,
                                             double &ung) {
    double Q = hydrograph(b, t);
    if (!(Q > 0.0)) return false;
    double q = Q / b.length;
    double n = sqrt(gn2 / g);
    hg = pow(n * q / sqrt(b.slope), 0.6);
    ung = -q / hg;
    return true;
}

__device__ __forceinline__ void neumaier(double &s, double &c, double v) {
    double t = s + v;
    if (fabs(s) >= fabs(v))
        c += (s - t) + v;
    else
        c += (v - t) + s;
    s = t;
}

// rho_k / lambda_k of one edge (eq. CFL_condition: rho is twice the
// centroid-edge distance, 4|cell| / (3 l)).  FP64 evaluates it exactly as
// written, edge by edge; FP32 folds the three edges into one division.
template <typename T> struct CflMin;
template <> struct CflMin<double> {
    double best = INFINITY;
    double area;
    __device__ explicit CflMin(double a) : area(a) {}
    __device__ void add(double l, double lam) {
        const double r = 4.0 * area / (3.0 * l) / lam;
        best = r < best ? r : best;
    }
    __device__ double value() const { return best; }
};
template <> struct CflMin<float> {
    float lmax = 0.0f;
    float area;
    __device__ explicit CflMin(float a) : area(a) {}
    __device__ void add(double l, double lam) { lmax = fmaxf(lmax, float(l * lam)); }
    __device__ double value() const {
        return lmax > 0.0f ? 4.0 * double(area) / (3.0 * double(lmax)) : INFINITY;
    }
};

// Updates cell i from U[cur] into U[cur ^ 1] and returns the CFL candidate
// min_k rho_k / lambda_k of the new state (+inf when nothing constrains it).
template <typename T>
__device__ __forceinline__ double cell_update(const Inst<T> &I, int i, int cur, double t, double dt,
                                              double t_next) {
    const V4<T> *__restrict__ src = cur ? I.U1 : I.U0;
    V4<T> *__restrict__ dst = cur ? I.U0 : I.U1;
    const T g = T(I.g);
    const double h_min = I.h_min;
    const V4<T> s = src[i];
    const V4<T> g0 = I.geo0[i];
    const V4<T> g1 = I.geo1[i];
    const int nb[3] = {I.nbr[i], I.nbr[I.n + i], I.nbr[2 * I.n + i]};
    const T lx[3] = {g0.x, g0.z, g1.x};
    const T ly[3] = {g0.y, g0.w, g1.y};
    const T area = g1.z, gn2 = g1.w;

    // primitive variables: velocity only above the minimum depth
    const double hsd = double(s.x) - double(s.w);
    const T hs = T(hsd);
    const bool wet = hsd > h_min;
    const T u = wet ? qdiv(s.y, hs) : T(0);
    const T v = wet ? qdiv(s.z, hs) : T(0);

    T R0 = T(0), R1 = T(0), R2 = T(0);
    T el[3], enx[3], eny[3];
    int inflow_bc[3] = {-1, -1, -1};
#pragma unroll
    for (int k = 0; k < 3; k++) {
        T l, nx, ny;
        edge_normal(lx[k], ly[k], l, nx, ny);
        el[k] = l;
        enx[k] = nx;
        eny[k] = ny;
        // this cell's velocity in the frame (n, t), t = (-ny, nx)
        const T uns = u * nx + v * ny;
        const T uts = v * nx - u * ny;
        const int e = nb[k];
        T F0, F1, F2, hself;
        if (e >= 0) {
            const int j = e & NBR_MASK;
            const bool flip = (e & NBR_FLIP) != 0;
            const V4<T> o = src[j];
            const double hod = double(o.x) - double(o.w);
            const T ho = T(hod);
            const bool owet = hod > h_min;
            const T uo = owet ? qdiv(o.y, ho) : T(0);
            const T vo = owet ? qdiv(o.z, ho) : T(0);
            const T uno = uo * nx + vo * ny;
            const T uto = vo * nx - uo * ny;
            // hydrostatic reconstruction of the two modified states
            const double zs = double(s.w > o.w ? s.w : o.w);
            const double a = double(s.x) - zs, b = double(o.x) - zs;
            const T hs_s = a < H_DRY ? T(0) : T(a);
            const T hs_o = b < H_DRY ? T(0) : T(b);
            // canonical orientation (left = smaller original index); the
            // normal of the canonical frame is -n when this cell is the right
            const T hL = flip ? hs_o : hs_s, hR = flip ? hs_s : hs_o;
            const T unL = flip ? -uno : uns, utL = flip ? -uto : uts;
            const T unR = flip ? -uns : uno, utR = flip ? -uts : uto;
            hllc<T>(hL, unL, utL, hR, unR, utR, g, F0, F1, F2);
            if (flip) F0 = -F0;  // mass leaving this cell through edge k
            hself = hs_s;
        } else {
            const int slot = -1 - e;
            const int kb = I.slot_kbc[slot];
            const int kind = kb & 15;
            const int bi = kb >> 4;
            // the ghost shares this cell's bed, so z* = z and h* = H - z
            const T hs_s = hsd < H_DRY ? T(0) : T(hsd);
            double hg, ung;
            bool open = false;
            if (kind == BC_OUTFLOW) {
                // transmissive: the ghost repeats the interior state
                hllc<T>(hs_s, uns, uts, hs_s, uns, uts, g, F0, F1, F2);
                open = true;
            } else if (kind == BC_INFLOW && inflow_ghost(I.bcs[bi], t, double(gn2), double(g), hg, ung)) {
                const double b = (double(s.w) + hg) - double(s.w);
                const T hs_g = b < H_DRY ? T(0) : T(b);
                hllc<T>(hs_s, uns, uts, hs_g, T(ung), T(0), g, F0, F1, F2);
                open = true;
            } else {
                // reflective, impermeable wall: mirrored normal velocity
                hllc<T>(hs_s, uns, uts, hs_s, -uns, uts, g, F0, F1, F2);
                F0 = T(0);
            }
            if (kind == BC_INFLOW) inflow_bc[k] = bi;
            if (open) {
                double *acc = I.slot_acc + 2 * slot;
                double sm = acc[0], cp = acc[1];
                neumaier(sm, cp, dt * double(l * F0));
                acc[0] = sm;
                acc[1] = cp;
            }
            hself = hs_s;
        }
        // fluctuation of this side: the flux minus its own reconstructed
        // pressure (bed slope in well-balanced form), rotated back
        const T Dn = F1 - T(0.5) * g * hself * hself;
        R0 += l * F0;
        R1 += l * (Dn * nx - F2 * ny);
        R2 += l * (Dn * ny + F2 * nx);
    }

    // conservative update (eq. hydrodynamicupdateformula)
    const T w = T(dt) * qdiv(T(1), area);
    T Hn = s.x - w * R0;
    T qx = s.y - w * R1;
    T qy = s.z - w * R2;
    const double hn = double(Hn) - double(s.w);
    // friction split: exact solution of dq/dt = -g n^2 |q| q / h^(7/3)
    T f;
    if (hn > h_min) {
        if (gn2 > T(0)) {
            const T qa = qsqrt(qx * qx + qy * qy);
            f = qdiv(T(1), T(1) + qdiv(T(dt) * gn2 * qa, pow73<T>(T(hn))));
        } else {
            f = T(1);
        }
    } else {
        f = T(0);
    }
    qx = qx * f;
    qy = qy * f;
    if (hn < 0.0) {
        // positivity: clip and account for the added volume
        atomicAdd(&I.ctrl->clipped, -hn * I.area[i]);
        atomicAdd(&I.ctrl->nclip, 1ull);
        if (I.neg_policy) atomicOr(&I.ctrl->flags, FLAG_NEGDEPTH);
        Hn = s.w;
        qx = T(0);
        qy = T(0);
    }
    if (!isfinite(Hn) || !isfinite(qx) || !isfinite(qy)) atomicOr(&I.ctrl->flags, FLAG_NONFINITE);
    dst[i] = make4<T>(Hn, qx, qy, s.w);

    // CFL candidate of the new state over wet cells and inflow ghosts
    CflMin<T> cfl(area);
    const double h2 = double(Hn) - double(s.w);
    if (h2 > h_min) {
        const T hh = T(h2);
        const T u2 = qdiv(qx, hh), v2 = qdiv(qy, hh);
        const T c = qsqrt(g * hh);
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const T lam = fabs(u2 * enx[k] + v2 * eny[k]) + c;
            cfl.add(double(el[k]), double(lam));
        }
    }
#pragma unroll
    for (int k = 0; k < 3; k++) {
        if (inflow_bc[k] >= 0) {
            double hg, ung;
            if (inflow_ghost(I.bcs[inflow_bc[k]], t_next, double(gn2), double(g), hg, ung))
                cfl.add(double(el[k]), fabs(ung) + sqrt(double(g) * hg));
        }
    }
    return cfl.value();
}

// CFL candidate of the current state (first step after an initialisation);
// the same arithmetic as the epilogue of cell_update.
template <typename T>
__device__ __forceinline__ double cell_candidate(const Inst<T> &I, int i, int cur, double t) {
    const V4<T> *__restrict__ src = cur ? I.U1 : I.U0;
    const T g = T(I.g);
    const V4<T> s = src[i];
    const V4<T> g0 = I.geo0[i];
    const V4<T> g1 = I.geo1[i];
    const int nb[3] = {I.nbr[i], I.nbr[I.n + i], I.nbr[2 * I.n + i]};
    const T lx[3] = {g0.x, g0.z, g1.x};
    const T ly[3] = {g0.y, g0.w, g1.y};
    CflMin<T> cfl(g1.z);
    const double hd = double(s.x) - double(s.w);
    const T hh = T(hd);
    const bool wet = hd > I.h_min;
    const T u = wet ? qdiv(s.y, hh) : T(0), v = wet ? qdiv(s.z, hh) : T(0);
    const T c = wet ? qsqrt(g * hh) : T(0);
#pragma unroll
    for (int k = 0; k < 3; k++) {
        T l, nx, ny;
        edge_normal(lx[k], ly[k], l, nx, ny);
        if (wet) {
            const T lam = fabs(u * nx + v * ny) + c;
            cfl.add(double(l), double(lam));
        }
        if (nb[k] < 0) {
            const int kb = I.slot_kbc[-1 - nb[k]];
            double hg, ung;
            if ((kb & 15) == BC_INFLOW && inflow_ghost(I.bcs[kb >> 4], t, double(g1.w), double(g), hg, ung))
                cfl.add(double(l), fabs(ung) + sqrt(double(g) * hg));
        }
    }
    return cfl.value();
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ unsigned long long load_agent(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename V> __device__ __forceinline__ void store_agent(V *p, V v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Time level of phase p as this step sees it.
struct Level {
    double t, dt, rawmin;
    long long steps;
    int cur;
    bool run;
};

// Reads time level `phase` and decides this step's dt: min(CFL * min
// rho/lambda, dt_max, t_end - t).  A finished or failed state does not step;
// block `lead` then carries the level forward unchanged, so phases stay
// aligned with the launch count.
__device__ __forceinline__ Level step_setup(Ctrl *c, int phase, double cfl, double dt_max, bool lead) {
    const int pin = phase, pout = phase == 2 ? 0 : phase + 1, pclr = phase == 0 ? 2 : phase - 1;
    Level L;
    L.t = c->s[pin].t;
    L.steps = c->s[pin].steps;
    L.cur = c->s[pin].cur;
    L.rawmin = __longlong_as_double((long long)c->m[pin].bits);
    L.dt = 0.0;
    const double t_end = c->t_end;
    L.run = L.t < t_end && c->flags == 0;
    if (L.run) {
        L.dt = fmin(fmin(cfl * L.rawmin, dt_max), t_end - L.t);
        if (!(L.dt > 0.0) || !(L.dt < INFINITY)) {
            L.run = false;
            if (lead && threadIdx.x == 0) atomicOr(&c->flags, FLAG_NODT);
        }
    }
    if (!L.run && lead && threadIdx.x == 0) {
        store_agent(&c->s[pout].t, L.t);
        store_agent(&c->s[pout].dt, c->s[pin].dt);
        store_agent(&c->s[pout].steps, L.steps);
        store_agent(&c->s[pout].cur, L.cur);
        store_agent(&c->m[pout].bits, c->m[pin].bits);
        store_agent(&c->m[pclr].bits, INF_BITS);
    }
    return L;
}

// Block minimum of the CFL candidates -> at most one atomic min on the next
// level's slot (skipped when it cannot lower the running value); block `lead`
// publishes the next time level and clears the slot two phases ahead.
__device__ __forceinline__ void block_finish(Ctrl *c, int phase, double cand, const Level &L, bool lead,
                                             bool advance) {
    __shared__ double wmin[16];
    const int pout = phase == 2 ? 0 : phase + 1, pclr = phase == 0 ? 2 : phase - 1;
    cand = wave_min(cand);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wmin[w] = cand;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wmin[0];
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 1; k < nw; k++) m = fmin(m, wmin[k]);
        const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
        unsigned long long *slot = advance ? &c->m[pout].bits : &c->m[phase].bits;
        if (mb < load_agent(slot)) atomicMin(slot, mb);
        if (lead && advance) {
            store_agent(&c->s[pout].t, L.t + L.dt);
            store_agent(&c->s[pout].dt, L.dt);
            store_agent(&c->s[pout].steps, L.steps + 1);
            store_agent(&c->s[pout].cur, L.cur ^ 1);
            store_agent(&c->m[pclr].bits, INF_BITS);
        }
    }
    __syncthreads();  // wmin may be reused by a following tile
}

template <typename T, int CPT>
__global__ void __launch_bounds__(1024) k_step(Inst<T> I, int phase) {
    const bool lead = blockIdx.x == 0;
    const Level L = step_setup(I.ctrl, phase, I.cfl, I.dt_max, lead);
    if (!L.run) return;
    const double t_next = L.t + L.dt;
    double cand = INFINITY;
#pragma unroll
    for (int r = 0; r < CPT; r++) {
        const int i = (blockIdx.x * CPT + r) * blockDim.x + threadIdx.x;
        if (i < I.n) cand = fmin(cand, cell_update<T>(I, i, L.cur, L.t, L.dt, t_next));
    }
    block_finish(I.ctrl, phase, cand, L, lead, true);
}

// CFL minimum of the state of level `phase` (after an initialisation); the
// host clears the slot first.
template <typename T>
__global__ void __launch_bounds__(256) k_dt_init(Inst<T> I, int phase) {
    const Ctrl *c = I.ctrl;
    Level L;
    L.t = c->s[phase].t;
    L.cur = c->s[phase].cur;
    L.dt = 0.0;
    L.steps = 0;
    L.rawmin = 0.0;
    L.run = true;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double cand = INFINITY;
    if (i < I.n) cand = cell_candidate<T>(I, i, L.cur, L.t);
    block_finish(I.ctrl, phase, cand, L, false, false);
}

// Persistent batched step: blocks stride over a list of (member, tile)
// pairs; each member keeps its own control block, so members step with their
// own dt and finished members cost one control-block read per tile.
template <typename T, int CPT>
__global__ void __launch_bounds__(256) k_step_batched(const Inst<T> *__restrict__ insts,
                                                       const int2 *__restrict__ tiles, int ntiles, int phase) {
    for (int tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
        // the tile is the same for the whole block: keep its record scalar
        const int2 td = make_int2(__builtin_amdgcn_readfirstlane(tiles[tt].x),
                                  __builtin_amdgcn_readfirstlane(tiles[tt].y));
        const Inst<T> I = insts[td.x];
        const bool lead = td.y == 0;
        const Level L = step_setup(I.ctrl, phase, I.cfl, I.dt_max, lead);
        if (!L.run) continue;
        const double t_next = L.t + L.dt;
        double cand = INFINITY;
#pragma unroll
        for (int r = 0; r < CPT; r++) {
            const int i = (td.y * CPT + r) * blockDim.x + threadIdx.x;
            if (i < I.n) cand = fmin(cand, cell_update<T>(I, i, L.cur, L.t, L.dt, t_next));
        }
        block_finish(I.ctrl, phase, cand, L, lead, true);
    }
}

// Error-free sum of two compensated accumulators (TwoSum on the heads).
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
    const double s = a.x + b.x;
    const double bb = s - a.x;
    const double e = (a.x - (s - bb)) + (b.x - bb);
    return make_double2(s, a.y + b.y + e);
}

__device__ __forceinline__ double2 block_csum(double2 v) {
    __shared__ double2 buf[MASS_THREADS];
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int w = MASS_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) buf[threadIdx.x] = cadd(buf[threadIdx.x], buf[threadIdx.x + w]);
        __syncthreads();
    }
    return buf[0];
}

// Volume sum (H - z)|cell| in a fixed order: fixed grid, strided per thread,
// fixed-shape tree per block, then one block over the partials.
template <typename T>
__global__ void __launch_bounds__(MASS_THREADS) k_mass_partial(Inst<T> I, double2 *partials, int phase) {
    const V4<T> *src = I.ctrl->s[phase].cur ? I.U1 : I.U0;
    double s = 0.0, c = 0.0;
    for (int i = blockIdx.x * MASS_THREADS + threadIdx.x; i < I.n; i += MASS_BLOCKS * MASS_THREADS) {
        const V4<T> u = src[i];
        neumaier(s, c, (double(u.x) - double(u.w)) * I.area[i]);
    }
    const double2 r = block_csum(make_double2(s, c));
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

template <typename T>
__global__ void __launch_bounds__(MASS_THREADS) k_mass_final(Inst<T> I, const double2 *partials, int nslots,
                                                             double *out) {
    double2 acc = make_double2(0.0, 0.0);
    for (int k = threadIdx.x; k < MASS_BLOCKS; k += MASS_THREADS) acc = cadd(acc, partials[k]);
    double2 m = block_csum(acc);
    __syncthreads();
    double2 b = make_double2(0.0, 0.0);
    for (int k = threadIdx.x; k < nslots; k += MASS_THREADS)
        b = cadd(b, make_double2(I.slot_acc[2 * k], I.slot_acc[2 * k + 1]));
    double2 bs = block_csum(b);
    if (threadIdx.x == 0) {
        out[0] = m.x + m.y;
        out[1] = bs.x + bs.y;
    }
}

}  // namespace

template <typename T>
hipError_t launch_step(const Inst<T> &I, int block, int cpt, int phase, hipStream_t s) {
    if (I.n <= 0) return hipSuccess;
    const int per = block * cpt;
    const int grid = (I.n + per - 1) / per;
    if (cpt == 2)
        hipLaunchKernelGGL((k_step<T, 2>), dim3(grid), dim3(block), 0, s, I, phase);
    else
        hipLaunchKernelGGL((k_step<T, 1>), dim3(grid), dim3(block), 0, s, I, phase);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dt_init(const Inst<T> &I, int phase, hipStream_t s) {
    if (I.n <= 0) return hipSuccess;
    const int grid = (I.n + 255) / 256;
    hipLaunchKernelGGL((k_dt_init<T>), dim3(grid), dim3(256), 0, s, I, phase);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mass(const Inst<T> &I, double2 *partials, double *out, int nslots, int phase, hipStream_t s) {
    hipLaunchKernelGGL((k_mass_partial<T>), dim3(MASS_BLOCKS), dim3(MASS_THREADS), 0, s, I, partials, phase);
    hipLaunchKernelGGL((k_mass_final<T>), dim3(1), dim3(MASS_THREADS), 0, s, I, (const double2 *)partials, nslots,
                       out);
    return hipGetLastError();
}

template <typename T>
int batched_grid(int block, int cpt) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e;
    if (cpt == 2)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_step_batched<T, 2>, block, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_step_batched<T, 1>, block, 0);
    if (e != hipSuccess || per < 1) per = 1;
    return cus * per;
}

template <typename T>
hipError_t launch_step_batched(const Inst<T> *insts, const int2 *tiles, int ntiles, int grid, int block, int cpt,
                               int phase, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (grid > ntiles) grid = ntiles;
    if (cpt == 2)
        hipLaunchKernelGGL((k_step_batched<T, 2>), dim3(grid), dim3(block), 0, s, insts, tiles, ntiles, phase);
    else
        hipLaunchKernelGGL((k_step_batched<T, 1>), dim3(grid), dim3(block), 0, s, insts, tiles, ntiles, phase);
    return hipGetLastError();
}

#define SWE_INSTANTIATE(T)                                                                                  \
    template hipError_t launch_step<T>(const Inst<T> &, int, int, int, hipStream_t);                        \
    template hipError_t launch_dt_init<T>(const Inst<T> &, int, hipStream_t);                               \
    template hipError_t launch_mass<T>(const Inst<T> &, double2 *, double *, int, int, hipStream_t);        \
    template hipError_t launch_step_batched<T>(const Inst<T> *, const int2 *, int, int, int, int, int,      \
                                               hipStream_t);                                                \
    template int batched_grid<T>(int, int);
SWE_INSTANTIATE(float)
SWE_INSTANTIATE(double)

}  // namespace swe
