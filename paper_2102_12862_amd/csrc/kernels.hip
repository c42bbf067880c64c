// HIP kernels of the shallow-water step for gfx950 (CDNA4, wave64).
//
// A block owns a tile of TILE consecutive cells of the Hilbert-ordered mesh.
// Phase 0 stages the tile's surfaces, velocities and beds in LDS.
// Phase 1 evaluates every edge of the tile once -- hydrostatic reconstruction,
// HLLC flux, the two fluctuations -- and leaves each cell's contribution in
// the LDS slot of its local edge (edges to other tiles are evaluated by both
// tiles, from identical inputs in the edge's canonical orientation, so the
// mass one cell loses is bitwise the mass the other gains).  Phase 2 gives
// each cell to one thread: it sums its three contributions in local edge
// order, applies the conservative update (paper: eq.
// hydrodynamicupdateformula), the friction split (eq. friction_closure, any
// closure of Table friction_closure) and the positivity clip, writes
// its new state and computes its CFL candidate (eq. CFL_condition).  A wave64
// shuffle, an LDS pass and at most one atomic min per block give the next
// time step; block 0 publishes the next time level, so a run of steps needs no
// host round trip and can be captured in one hipGraph.
//
// Precision.  The FP64 instantiation evaluates every formula in the operation
// order of an FP64 reference, so each wet/dry decision matches it bit for bit.
// The FP32 instantiation keeps the state and the flux arithmetic in single
// precision (hardware reciprocal, square root, log2 and exp2; fused
// multiply-adds where they cannot break the exact balance of a lake at rest),
// with the depth differences H - z, the wet/dry tests, the time levels, the
// time step and the mass sums in FP64.  Its water surface is stored as an
// unevaluated sum of two single-precision numbers, H = hi + lo (lo in an
// array of its own): the fluxes see hi, the update adds its increment to the
// whole sum in FP64, so an increment smaller than the single-precision
// spacing of a surface tens of metres above the datum (the first water a
// wetting front brings into a dry cell) is kept in lo instead of rounded
// away, and the volume is conserved at the fronts too.
#include "swe_internal.h"

#include <math.h>

#include <mutex>
#include <type_traits>

namespace swe {

namespace {

constexpr double H_DRY = 1e-12;  // reconstructed depths below this are dry

template <typename T> constexpr bool IS32 = sizeof(T) == 4;

template <typename T> __device__ __forceinline__ V4<T> make4(T a, T b, T c, T d);
template <> __device__ __forceinline__ float4 make4<float>(float a, float b, float c, float d) {
    return make_float4(a, b, c, d);
}
template <> __device__ __forceinline__ double4 make4<double>(double a, double b, double c, double d) {
    return make_double4(a, b, c, d);
}

// The surface of a cell in FP64: FP32 states carry it as hi + lo (exact in
// FP64), FP64 states as hi alone.
__device__ __forceinline__ double surface(double hi, double /*lo*/) { return hi; }
__device__ __forceinline__ double surface(float hi, float lo) { return double(hi) + double(lo); }

// FP32 states store hi = the nearest float to the surface and the rest
// H - hi (at most half an ulp of hi) as a 16-bit integer k in units of
// 2^-16 ulp(hi): ulp(hi) = 2^(e-24) for hi = m 2^e, m in [1/2, 1), so the
// unit is 2^(e-40) and |k| <= 2^15 (the one code past the int16 range,
// +2^15, is clamped).  The surface so resolves to about 2^-40 of itself at
// 2 bytes per cell.  lo_value decodes exactly; lo_code rounds to nearest.
__device__ __forceinline__ int lo_unit_exp(float hi) { return __builtin_amdgcn_frexp_expf(hi) - 40; }
__device__ __forceinline__ float lo_value(float hi, int16_t k) { return ldexpf(float(k), lo_unit_exp(hi)); }
__device__ __forceinline__ int16_t lo_code(float hi, double rest) {
    const double k = rint(ldexp(rest, -lo_unit_exp(hi)));
    return int16_t(fmin(fmax(k, -32768.0), 32767.0));
}
// The decoded low part of cell i's surface (FP64: none).
template <typename T> __device__ __forceinline__ T low_part(gptr<const int16_t> L, int i, T hi) {
    if constexpr (IS32<T>) return lo_value(hi, L[i]);
    else return T(0);
}

// Division and square root.  FP64 uses IEEE-correct operations so that every
// wet/dry decision matches an FP64 reference bit for bit; FP32 uses the
// hardware reciprocal and square root (about 1 ulp), which is far inside the
// single-precision error budget of the method.
__device__ __forceinline__ double qdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double qsqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float qsqrt(float a) { return __builtin_amdgcn_sqrtf(a); }

// Edge length and unit normal from l*n.  FP64: the IEEE square root and two
// divisions (matching the reference); FP32: one reciprocal square root.  Both
// give exactly negated normals for exactly negated l*n.
__device__ __forceinline__ void edge_normal(double lx, double ly, double &l, double &nx, double &ny) {
    l = sqrt(lx * lx + ly * ly);
    nx = lx / l;
    ny = ly / l;
}
__device__ __forceinline__ void edge_normal(float lx, float ly, float &l, float &nx, float &ny) {
    const float s = fmaf(lx, lx, ly * ly);
    const float r = __builtin_amdgcn_rsqf(s);
    l = s * r;
    nx = lx * r;
    ny = ly * r;
}

// Velocity (u, v) in the frame (n, t) of an edge, t = (-ny, nx).  The FP32
// form is odd in n, so the two cells of an edge see exactly opposite values.
__device__ __forceinline__ void rotate(double u, double v, double nx, double ny, double &un, double &ut) {
    un = u * nx + v * ny;
    ut = v * nx - u * ny;
}
__device__ __forceinline__ void rotate(float u, float v, float nx, float ny, float &un, float &ut) {
    un = fmaf(u, nx, v * ny);
    ut = fmaf(v, nx, -(u * ny));
}

// HLLC flux (Toro 1994) in the frame of the edge normal, for reconstructed
// depths hL, hR >= 0.  Wave speeds: two-rarefaction estimates with c* >= 0
// when both sides are wet, dry-bed speeds u -+ 2c when one side is dry.  The
// flux is F_K + S_K (U*_K - U_K) on the side K the contact speed S* selects,
// with U*_K = h_K (S_K - u_K)/(S_K - S*) (1, S*, ut_K), or the physical flux
// F_K when all waves move one way (or the states are identical); two dry
// sides give zero.  The side is chosen first and the formulas evaluated once,
// so neighbouring edges with opposite flow directions do not diverge.  The
// hydrostatic pressure g h^2 / 2 of F1 is formed as (g/2 * h) * h, the same
// product the fluctuations subtract, so a lake at rest balances exactly.
__device__ __forceinline__ void hllc(double hL, double unL, double utL, double hR, double unR, double utR, double g,
                                     double &F0, double &F1, double &F2) {
    const double zero = 0.0, half = 0.5;
    if (!(hL > zero) && !(hR > zero)) {
        F0 = zero; F1 = zero; F2 = zero;
        return;
    }
    const bool ident = hL == hR && unL == unR && utL == utR;
    const double cL = sqrt(g * hL), cR = sqrt(g * hR);
    const bool dryL = !(hL > zero), dryR = !(hR > zero);
    const double a = half * (cL + cR) + 0.25 * (unL - unR);
    const double us = half * (unL + unR) + cL - cR;
    const double cs = a > zero ? a : zero;
    const double SL = dryL ? unR - 2.0 * cR : (dryR ? unL - cL : fmin(unL - cL, us - cs));
    const double SR = dryL ? unR + cR : (dryR ? unL + 2.0 * cL : fmax(unR + cR, us + cs));
    const double Ss = (SL * hR * (unR - SR) - SR * hL * (unL - SL)) / (hR * (unR - SR) - hL * (unL - SL));
    const bool left = ident || zero <= SL || (!(SR <= zero) && zero <= Ss);
    const bool star = !ident && !(zero <= SL) && !(SR <= zero);
    const double hK = left ? hL : hR, unK = left ? unL : unR, utK = left ? utL : utR, SK = left ? SL : SR;
    F0 = hK * unK;
    F1 = hK * unK * unK + half * g * hK * hK;
    F2 = hK * unK * utK;
    if (star) {
        const double f = hK * (SK - unK) / (SK - Ss);
        F0 = F0 + SK * (f - hK);
        F1 = F1 + SK * (f * Ss - hK * unK);
        F2 = F2 + SK * (f * utK - hK * utK);
    }
}
__device__ __forceinline__ void hllc(float hL, float unL, float utL, float hR, float unR, float utR, float g,
                                     float &F0, float &F1, float &F2) {
    if (!(hL > 0.0f) && !(hR > 0.0f)) {
        F0 = 0.0f; F1 = 0.0f; F2 = 0.0f;
        return;
    }
    const bool ident = hL == hR && unL == unR && utL == utR;
    const float cL = qsqrt(g * hL), cR = qsqrt(g * hR);
    const bool dryL = !(hL > 0.0f), dryR = !(hR > 0.0f);
    const float a = fmaf(0.25f, unL - unR, 0.5f * (cL + cR));
    const float us = fmaf(0.5f, unL + unR, cL - cR);
    const float cs = a > 0.0f ? a : 0.0f;
    const float SL = dryL ? fmaf(-2.0f, cR, unR) : (dryR ? unL - cL : fminf(unL - cL, us - cs));
    const float SR = dryL ? unR + cR : (dryR ? fmaf(2.0f, cL, unL) : fmaxf(unR + cR, us + cs));
    const float AR = hR * (unR - SR), AL = hL * (unL - SL);
    const float Ss = qdiv(fmaf(SL, AR, -(SR * AL)), AR - AL);
    const bool left = ident || 0.0f <= SL || (!(SR <= 0.0f) && 0.0f <= Ss);
    const bool star = !ident && !(0.0f <= SL) && !(SR <= 0.0f);
    const float hK = left ? hL : hR, unK = left ? unL : unR, utK = left ? utL : utR, SK = left ? SL : SR;
    const float m = hK * unK;
    F0 = m;
    F1 = fmaf(m, unK, (0.5f * g * hK) * hK);
    F2 = m * utK;
    if (star) {
        const float f = qdiv(hK * (SK - unK), SK - Ss);
        F0 = fmaf(SK, f - hK, F0);
        F1 = fmaf(SK, fmaf(f, Ss, -m), F1);
        F2 = fmaf(SK, (f - hK) * utK, F2);
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

// FP64 power of the boundary branches, kept out of line: inlined, the
// compiler loads the polynomial constants of pow into some forty registers
// before the edge loop and holds them through it, for a call that only
// boundary edges make.
__device__ __noinline__ double bc_pow(double x, double p) { return pow(x, p); }

// Boundary state of the two discharge inflows (kind BC_INFLOW or
// BC_FROUDE): q = Q / length enters at the depth x^p, x = n q / sqrt(S),
// p = 3/5 (uniform) or x = q / (Fr sqrt(g)), p = 2/3 (froude).  One pow
// call serves both.  FP64
// takes sqrt(g) from the host (like sqrt(2 g) of the weir law: formed on the
// device, it would be hoisted into every wave's prologue); FP32 forms its
// single-instruction square root itself.
__device__ __forceinline__ bool discharge_ghost(const BCdev &b, int kind, double t, double gn2, double g,
                                                double sqrtg, double &hg, double &ung, double &qin) {
    double Q = hydrograph(b, t);
    if (!(Q > 0.0)) return false;
    double q = Q / b.length;
    const bool unif = kind == BC_INFLOW;
    double x = unif ? sqrt(gn2 / g) * q / sqrt(b.slope) : q / (b.slope * sqrtg);
    hg = bc_pow(x, unif ? 0.6 : 2.0 / 3.0);
    ung = -q / hg;
    qin = q;
    return true;
}
__device__ __forceinline__ bool discharge_ghost(const BCdev &b, int kind, double t, float gn2, float g,
                                                double /*sqrtg*/, float &hg, float &ung, float &qin) {
    const double Q = hydrograph(b, t);
    if (!(Q > 0.0)) return false;
    const float q = float(Q / b.length);
    const bool unif = kind == BC_INFLOW;
    const float x = unif ? q * qsqrt(qdiv(gn2, g * float(b.slope))) : qdiv(q, float(b.slope) * qsqrt(g));
    hg = __builtin_amdgcn_exp2f((unif ? 0.6f : 2.0f / 3.0f) * __builtin_amdgcn_logf(x));
    ung = -qdiv(q, hg);
    qin = q;
    return true;
}

// Normal depth (n q / sqrt(S))^(3/5) of a unit discharge q >= 0 under the
// cell's power-law coefficient gn2 = g n^2 (uniform outflow).
__device__ __forceinline__ double normal_depth(double gn2, double g, double q, double S) {
    double n = sqrt(gn2 / g);
    return bc_pow(n * q / sqrt(S), 0.6);
}
__device__ __forceinline__ float normal_depth(float gn2, float g, float q, double S) {
    const float x = q * qsqrt(qdiv(gn2, g * float(S)));
    return x > 0.0f ? __builtin_amdgcn_exp2f(0.6f * __builtin_amdgcn_logf(x)) : 0.0f;
}

// Discharge per unit length leaving through a weir (Poleni's free overflow
// (2/3) mu sqrt(2g) d^(3/2), head d over the crest, a crest below the cell's
// bed counting at the bed) or an h-Q relation (Q(H) over the boundary
// length), from the cell's surface H and bed z; zero for a dry cell.  The
// constant sqrt(2 g) comes from the host: formed here, the compiler hoists
// it out of the edge loop into every wave's prologue.
__device__ __forceinline__ double imposed_outflow(const BCdev &b, double H, double z, double sqrt2g) {
    if (!(H - z > 0.0)) return 0.0;
    if (b.kind == BC_WEIR) {
        const double crest = b.slope > z ? b.slope : z;
        const double d = H - crest;
        if (!(d > 0.0)) return 0.0;
        return (2.0 / 3.0) * b.par * sqrt2g * (d * sqrt(d));
    }
    return hydrograph(b, H) / b.length;
}

__device__ __forceinline__ void neumaier(double &s, double &c, double v) {
    double t = s + v;
    if (fabs(s) >= fabs(v))
        c += (s - t) + v;
    else
        c += (v - t) + s;
    s = t;
}

// Volumes a cell's update sets by hand (the water's positivity clip, the
// species' reset in a cell left dry, the non-erodible bed's clip), handed
// from the update to the per-group tallies.
template <int NS> struct Tally {
    double clip = 0.0, bed = 0.0;
    double sp[NS > 0 ? NS : 1] = {};
};

// Adds each lane's v to the compensated accumulator (sum, compensation) of
// its group of 64 consecutive device cells, acc + 2 * (cell / 64): a shuffle
// tree in a fixed order, then lane 0 updates the group's own slot.  No slot
// has two writers and every sum runs in one order, so the tally is the same
// bitwise at any tile size and launch order.  Called by whole waves; a wave
// with nothing to add skips it.
template <typename P>
__device__ __forceinline__ void group_tally(P acc, int cell, double v) {
    if (__ballot(v != 0.0) == 0) return;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) {
        const P a = acc + 2 * (cell >> 6);
        double sm = a[0], cp = a[1];
        neumaier(sm, cp, v);
        a[0] = sm;
        a[1] = cp;
    }
}

// Friction split (eq. friction_closure, Table friction_closure).  With
// S_f = u|u| / (g h c_f^2) the momentum sink is |q| q / (h^2 c_f^2); its exact
// solution over dt (h frozen) scales q by 1 / (1 + dt |q| / (h^2 c_f^2)).  The
// power laws (Manning; Strickler with n = 1/k_str) give
// 1 / (1 + dt g n^2 |q| / h^(7/3)) with par = g n^2; the log types take
// par = K_s (Chezy: c_f = 6.25 + ln(h/K_s) above K_s, else 6.25) or y_R
// (Bezzola, three branches in h/y_R).
__device__ __forceinline__ double friction_cf(int kind, double par, double h) {
    if (kind == FR_CHEZY) return h > par ? 6.25 + log(h / par) : 6.25;
    const double r = h / par;
    if (r > 2.0) return 2.5 * sqrt(1.0 - 1.0 / r) * log(10.9 * r);
    if (r >= 0.5) return 1.25 * sqrt(r) * log(10.9 * r);
    return 1.5;
}
__device__ __forceinline__ double friction_factor(int kind, double dt, double par, double qx, double qy,
                                                  double h) {
    const double qa = sqrt(qx * qx + qy * qy);
    // h^(7/3) as h^2 h^(1/3): the cube root costs a fraction of a general
    // power (within an ulp of it)
    if (kind <= FR_STRICKLER) return 1.0 / (1.0 + dt * par * qa / (h * h * cbrt(h)));
    const double cf = friction_cf(kind, par, h);
    return 1.0 / (1.0 + dt * qa / (h * h * cf * cf));
}
__device__ __forceinline__ float friction_cf(int kind, float par, float h) {
    constexpr float LN2 = 0.693147180559945f;
    if (kind == FR_CHEZY)
        return h > par ? fmaf(LN2, __builtin_amdgcn_logf(h * __builtin_amdgcn_rcpf(par)), 6.25f) : 6.25f;
    const float r = h * __builtin_amdgcn_rcpf(par);
    const float ln = LN2 * __builtin_amdgcn_logf(10.9f * r);
    if (r > 2.0f) return 2.5f * qsqrt(1.0f - __builtin_amdgcn_rcpf(r)) * ln;
    if (r >= 0.5f) return 1.25f * qsqrt(r) * ln;
    return 1.5f;
}
__device__ __forceinline__ float friction_factor(int kind, float dt, float par, float qx, float qy, float h) {
    const float qa = qsqrt(fmaf(qx, qx, qy * qy));
    if (kind <= FR_STRICKLER) {
        const float hp = __builtin_amdgcn_exp2f((-7.0f / 3.0f) * __builtin_amdgcn_logf(h));  // h^(-7/3)
        return __builtin_amdgcn_rcpf(fmaf(dt * par * qa, hp, 1.0f));
    }
    const float cf = friction_cf(kind, par, h);
    return __builtin_amdgcn_rcpf(fmaf(dt * qa, __builtin_amdgcn_rcpf(h * h * cf * cf), 1.0f));
}

// CFL terms (eq. CFL_condition, rho = twice the centroid-edge distance =
// 4|cell| / (3 l)).  FP64 takes min over edges of rho/lambda exactly as
// written.  FP32 takes the cell's max of l * lambda / |cell| in single
// precision; the block turns its maximum m into 4 / (3 m) in FP64.  Inflow
// ghosts do not depend on the new state, so the edge pass folds their terms
// into one LDS word per tile, as the bits of a positive number (a min in
// FP64, a max in FP32), whose integer order is its numeric order.
template <typename T> using CandT = T;  // FP64: min rho/lambda; FP32: max l*lambda/|cell|
template <typename T> using GhostBits = typename std::conditional<IS32<T>, unsigned, unsigned long long>::type;
__device__ __forceinline__ double cfl_term(double area, double l, double lam) { return 4.0 * area / (3.0 * l) / lam; }
__device__ __forceinline__ unsigned long long ghost_init(double) { return INF_BITS; }
__device__ __forceinline__ unsigned ghost_init(float) { return 0u; }
__device__ __forceinline__ double ghost_value(unsigned long long b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ float ghost_value(unsigned b) { return __uint_as_float(b); }

__device__ __forceinline__ double wave_reduce(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
// FP32 terms are non-negative, so their bit patterns (sign cleared) order
// like their values: the max runs on integers, by DPP permutations within
// each row of 16 lanes, then over the four rows' lanes 0, 16, 32, 48.
__device__ __forceinline__ unsigned dpp_max(unsigned v, int ctrl_id) {
    int p;
    switch (ctrl_id) {
        case 0: p = __builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false); break;   // quad_perm 1,0,3,2
        case 1: p = __builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false); break;   // quad_perm 2,3,0,1
        case 2: p = __builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false); break;  // row_half_mirror
        default: p = __builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false); break; // row_mirror
    }
    return max(v, (unsigned)p);
}
__device__ __forceinline__ float wave_reduce(float v) {
    unsigned b = __float_as_uint(v) & 0x7FFFFFFFu;
    b = dpp_max(b, 0);
    b = dpp_max(b, 1);
    b = dpp_max(b, 2);
    b = dpp_max(b, 3);
    const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)b, 0);
    const unsigned r1 = (unsigned)__builtin_amdgcn_readlane((int)b, 16);
    const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)b, 32);
    const unsigned r3 = (unsigned)__builtin_amdgcn_readlane((int)b, 48);
    return __uint_as_float(max(max(r0, r1), max(r2, r3)));
}
__device__ __forceinline__ double combine(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float combine(float a, float b) { return fmaxf(a, b); }
// block value -> min rho/lambda over the block
__device__ __forceinline__ double block_rho_lambda(double m) { return m; }
__device__ __forceinline__ double block_rho_lambda(float m) {
    return m > 0.0f ? 4.0 / (3.0 * double(m)) : INFINITY;
}

__device__ __forceinline__ unsigned long long load_agent(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename V> __device__ __forceinline__ void store_agent(V *p, V v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A dynamic wall (section "Hydrodynamic BCs") with a collapse depth: the
// step that starts with a cell next to it at that depth or deeper lowers the
// wall's collapse time to its own end time t_next (an atomic min on the
// device record), so every block of that step still sees the wall and the
// steps from t_next on do not.
__device__ __forceinline__ void wall_trigger(const BCdev &B, double h, double t_next) {
    if (B.par > 0.0 && h >= B.par) {
        // formed here: hoisted out of the edge loop the value would hold
        // registers through it
        __asm__ volatile("" : "+v"(t_next));
        __hip_atomic_fetch_min(const_cast<double *>(&B.slope), t_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
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

// Work-groups are dealt to the eight XCDs in turn (group b to XCD b mod 8),
// each with its own L2.  Remapping group b to tile x*q + min(x, r) + b/8
// (x = b mod 8, n = 8q + r tiles) gives every XCD one contiguous run of
// Hilbert-ordered tiles, walked in order, so the neighbours a tile gathers
// from other tiles were mostly just read through the same L2.  A bijection
// for any n; results do not depend on the order tiles are processed in.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int q = n >> 3, r = n & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// Slot that a step of launch phase `phase` lowers (advance) or an
// initialisation fills (!advance).
__device__ __forceinline__ unsigned long long *cfl_slot(Ctrl *c, int phase, bool advance) {
    return advance ? &c->m[phase == 2 ? 0 : phase + 1].bits : &c->m[phase].bits;
}

// Block reduction of the CFL terms -> at most one atomic min on the slot,
// skipped when the slot already holds a value no larger.  The slot is read
// here, after every other load of the block: the loads of a wave complete in
// order, so reading this contended line earlier would hold up the update
// phase's own loads.  Block `lead` publishes the next time level and clears
// the slot two phases ahead.
template <typename C>
__device__ __forceinline__ void block_finish(Ctrl *c, int phase, C cand, const Level &L, bool lead, bool advance) {
    __shared__ C wred[16];
    const int pout = phase == 2 ? 0 : phase + 1, pclr = phase == 0 ? 2 : phase - 1;
    cand = wave_reduce(cand);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wred[w] = cand;
    __syncthreads();
    if (threadIdx.x == 0) {
        C r = wred[0];
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 1; k < nw; k++) r = combine(r, wred[k]);
        const double m = block_rho_lambda(r);
        const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
        unsigned long long *slot = cfl_slot(c, phase, advance);
        if (mb < load_agent(slot)) atomicMin(slot, mb);
        if (lead && advance) {
            store_agent(&c->s[pout].t, L.t + L.dt);
            store_agent(&c->s[pout].dt, L.dt);
            store_agent(&c->s[pout].steps, L.steps + 1);
            store_agent(&c->s[pout].cur, L.cur ^ 1);
            store_agent(&c->m[pclr].bits, INF_BITS);
        }
    }
    __syncthreads();  // wred may be reused by a following tile
}

// LDS of one tile: per cell (H, u, v, z) with the velocity zero at or below
// the minimum depth, per (local edge, cell) the three contribution components
// and the edge geometry the CFL candidate needs, and the tile's inflow-ghost
// CFL term.  The update thread of a cell keeps its (H, qx, qy, z) in
// registers.  FP32 keeps l*n of local edges 0 and 1 only (the outward l*n of
// a triangle's three edges add up to zero, so edge 2's is minus their sum)
// and, staged with the state, the low part of the surface; FP64 keeps the
// unit normal and the length of all three (its CFL term follows the oracle's
// operation order).
template <typename T, int TILE> struct TileLds {
    V4<T> huvz[TILE];
    T c[3][3][TILE];   // [component][local edge][cell]
    T gx[IS32<T> ? 2 : 3][TILE], gy[IS32<T> ? 2 : 3][TILE];
    T gl[IS32<T> ? 1 : 3][IS32<T> ? 1 : TILE];
    T lo[IS32<T> ? TILE : 1];
    GhostBits<T> ghost;
};

// Geometry of the three edges of cell c of the tile, from what TileLds keeps:
// FP32 l*n in (gx, gy); FP64 the unit normal in (gx, gy) and the length in gl
// (the normal's sign is the cell's outward one).
template <typename T, int TILE>
__device__ __forceinline__ void cell_geometry(const TileLds<T, TILE> &S, int c, T (&gx)[3], T (&gy)[3],
                                              T (&gl)[3]) {
    if constexpr (IS32<T>) {
        gx[0] = S.gx[0][c];
        gy[0] = S.gy[0][c];
        gx[1] = S.gx[1][c];
        gy[1] = S.gy[1][c];
        gx[2] = -(gx[0] + gx[1]);
        gy[2] = -(gy[0] + gy[1]);
        gl[0] = gl[1] = gl[2] = T(0);
    } else {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            gx[k] = S.gx[k][c];
            gy[k] = S.gy[k][c];
            gl[k] = S.gl[k][c];
        }
    }
}

// LDS of the passive species of one tile (section "Scalar advection-
// diffusion", advective part): per species the concentrations of the tile's
// cells and the advective contribution of each (local edge, cell).
template <typename T, int TILE, int NS> struct ScalarLds {
    T phi[NS][TILE];
    T c[NS][3][TILE];
};

// Concentration phi = q / h of a cell with water (q and h are carried by the
// same mass flux, so thin films keep theirs), 0 in a dry one.
__device__ __forceinline__ double concentration(double q, double h) { return h > 0.0 ? q / h : 0.0; }
__device__ __forceinline__ float concentration(float q, double h) {
    return h > 0.0 ? q * __builtin_amdgcn_rcpf(float(h)) : 0.0f;
}

// LDS of the Exner module for one tile (section "Morphodynamics"): per cell
// the transport magnitude Phi and dPhi/d|u|, per (local edge, cell) the bed
// contribution l q_B.
template <typename T, int TILE> struct MorphoLds {
    T phi[TILE];
    T dphi[TILE];
    T c[3][TILE];
};

// c_f^2 of the cell's friction closure at depth h > 0 (0: frictionless).
__device__ __forceinline__ double cell_cf2(int kind, double par, double h) {
    if (!(par > 0.0)) return 0.0;
    if (kind <= FR_STRICKLER) return cbrt(h) / par;  // h^(1/3) / (g n^2)
    const double cf = friction_cf(kind, par, h);
    return cf * cf;
}
__device__ __forceinline__ float cell_cf2(int kind, float par, float h) {
    if (!(par > 0.0f)) return 0.0f;
    if (kind <= FR_STRICKLER)
        return __builtin_amdgcn_exp2f((1.0f / 3.0f) * __builtin_amdgcn_logf(h)) * __builtin_amdgcn_rcpf(par);
    const float cf = friction_cf(kind, par, h);
    return cf * cf;
}

__device__ __forceinline__ double spow(double x, double p) { return pow(x, p); }
__device__ __forceinline__ float spow(float x, float p) {
    return __builtin_amdgcn_exp2f(p * __builtin_amdgcn_logf(x));
}

// Transport magnitude Phi(|u|) and dPhi/d|u| at fixed depth (Table
// sedtransport_closure): MPM alpha (theta - theta_cr)^m K, Grass alpha
// (|u| - u_cr)^m, Engelund-Hansen 0.05 c_f^2 theta^(5/2) K, with the Shields
// number theta = |u|^2 / (c_f^2 (s - 1) g d) and K = sqrt((s - 1) g d^3).
template <typename T>
__device__ __forceinline__ void sed_mag(const Inst<T> &I, T umag, T cf2, T &phi, T &dphi) {
    phi = T(0);
    dphi = T(0);
    if (!(umag > T(0))) return;
    const T alpha = T(I.salpha), m = T(I.sm), thr = T(I.sthr);
    if (I.sclos == SED_GRASS) {
        const T e = umag - thr;
        if (e > T(0)) {
            phi = alpha * spow(e, m);
            dphi = alpha * m * spow(e, m - T(1));
        }
        return;
    }
    if (!(cf2 > T(0))) return;
    const T theta = umag * umag / (cf2 * T(I.srgd));
    const T Kc = T(I.sK);
    if (I.sclos == SED_MPM) {
        const T e = theta - thr;
        if (e > T(0)) {
            phi = alpha * spow(e, m) * Kc;
            dphi = alpha * m * spow(e, m - T(1)) * Kc * (T(2) * theta / umag);
        }
    } else {
        phi = T(0.05) * cf2 * spow(theta, T(2.5)) * Kc;
        dphi = T(5) * phi / umag;
    }
}

// Phi and dPhi of a cell from its state: no transport when dry (h <= h_min),
// frictionless, or at its non-erodible bed.
template <typename T>
__device__ __forceinline__ void cell_sediment(const Inst<T> &I, double hd, T u, T v, T z, T gn2, int cell, T &phi,
                                              T &dphi) {
    phi = T(0);
    dphi = T(0);
    if (!(hd > I.h_min)) return;
    if (I.zfix && z <= I.zfix[cell]) return;
    const T cf2 = cell_cf2(I.friction, gn2, T(hd));
    sed_mag(I, T(qsqrt(u * u + v * v)), cf2, phi, dphi);
}

// Normal transport q_B.n and the speeds lambda_1, lambda_2 of one side of an
// edge (eq. exner_wave_estimation), with dq_B,n/dq_n at fixed depth and
// tangential velocity: (Phi' cos^2 a + Phi / |u| sin^2 a) / h.
template <typename T>
__device__ __forceinline__ void sed_side(T phi, T dphi, T u, T v, T un, T h, T g, T &qn, T &l1, T &l2) {
    T dd = T(0);
    qn = T(0);
    if (phi > T(0) && h > T(0)) {
        const T umag = qsqrt(u * u + v * v);
        const T ca = un / umag;
        qn = phi * ca;
        dd = (dphi * (ca * ca) + (phi / umag) * (T(1) - ca * ca)) / h;
    }
    const T c = qsqrt(g * (h > T(0) ? h : T(0)));
    const T a = un - c;
    const T r = qsqrt(a * a + T(4) * dd * (c * c));
    l1 = T(0.5) * (a - r);
    l2 = T(0.5) * (a + r);
}

// CFL term of an inflow ghost (depth hg, normal velocity ung) on an edge of
// length l of a cell with ap = |cell| (FP64) or 1/|cell| (FP32), merged into
// the tile's LDS word.
template <typename T, int TILE>
__device__ __forceinline__ void ghost_cfl(TileLds<T, TILE> &S, T l, T hg, T ung, T g, T ap) {
    if constexpr (IS32<T>) {
        atomicMax(&S.ghost, __float_as_uint(l * (fabsf(ung) + qsqrt(g * hg)) * ap));
    } else {
        const double r = cfl_term(ap, l, fabs(ung) + sqrt(g * hg));
        atomicMin(&S.ghost, (unsigned long long)__double_as_longlong(r));
    }
}

// Forces all four components of a gathered state to be loaded together (one
// 16 B load in FP32) instead of a partial load plus a conditional one.
template <typename V> __device__ __forceinline__ void whole(V &s) {
    asm volatile("" : "+v"(s.x), "+v"(s.y), "+v"(s.z), "+v"(s.w));
}

// Phases 0 and 1 for tile `tile`: fluxes at time t (UPDATE = false: geometry
// only) and the inflow ghosts' CFL terms at time t_cand.  `own` receives the
// state (H, qx, qy, z) of this thread's cell.  NS > 0: NS passive species
// ride on the pass (SS, and qown for the cell's specific masses); each edge's
// advective flux is the HLLC mass flux times the concentration of the cell
// the water leaves.
// DRAIN: 0 none; DRAIN_MEASURE: fluxes into LDS only, without the
// boundary tallies (the draining-time pass); DRAIN_APPLY: each flux scaled by
// the draining factor of the cell its water leaves.
enum : int { DRAIN_NONE = 0, DRAIN_MEASURE = 1, DRAIN_APPLY = 2 };

// IW: the mesh has internal walls (tagged interior edges); the check is
// compiled only where it is needed, as it costs the plain step registers.
template <typename T, int TILE, bool UPDATE, int NS = 0, bool MORPHO = false, int DRAIN = DRAIN_NONE, bool IW = true>
__device__ __forceinline__ void tile_edges(const Inst<T> &I, TileLds<T, TILE> &S, int tile, int cur, double t,
                                           double dt, double t_cand, V4<T> &own,
                                           ScalarLds<T, TILE, (NS > 0 ? NS : 1)> *SS = nullptr,
                                           T *qown = nullptr, MorphoLds<T, TILE> *MS = nullptr) {
    const gptr<const V4<T>> __restrict__ src = cur ? I.U1 : I.U0;
    const gptr<const T> __restrict__ qsrc = cur ? I.Q1 : I.Q0;
    const T g = T(I.g);
    const T hg2 = T(0.5) * g;  // g/2 of the hydrostatic pressure (g/2 h) h
    const double h_min = I.h_min;
    const int c = threadIdx.x;
    const int i = tile * TILE + c;
    // the edge records do not depend on the state: the first one is loaded
    // before phase 0 and each next one an iteration ahead (unconditionally:
    // lanes past the end re-read the tile's last record, which every tile
    // has, so the loads need no branch)
    const int e1 = I.eoff[tile + 1];
    int e = I.eoff[tile] + c;
    Edge<T> En = I.edges[min(e, e1 - 1)];
    own = make4<T>(T(0), T(0), T(0), T(0));
    if (i < I.n) {
        const V4<T> s = src[i];
        own = s;
        if constexpr (IS32<T>) S.lo[c] = low_part<T>(cur ? I.L1 : I.L0, i, s.x);
        // velocity only above the minimum depth (the fluxes see the surface's
        // high part)
        const double hd = double(s.x) - double(s.w);
        const bool wet = hd > h_min;
        const T h = T(hd);
        S.huvz[c] = make4<T>(s.x, wet ? qdiv(s.y, h) : T(0), wet ? qdiv(s.z, h) : T(0), s.w);
        if constexpr (NS > 0) {
#pragma unroll
            for (int sp = 0; sp < NS; sp++) {
                const T q = qsrc[(size_t)sp * I.n + i];
                qown[sp] = q;
                SS->phi[sp][c] = concentration(q, hd);
            }
        }
        if constexpr (MORPHO) {
            T phi, dphi;
            cell_sediment(I, hd, S.huvz[c].y, S.huvz[c].z, s.w, I.cellp[i].y, i, phi, dphi);
            MS->phi[c] = phi;
            MS->dphi[c] = dphi;
        }
    }
    if (c == 0) S.ghost = ghost_init(T(0));
    __syncthreads();
    for (; e < e1; e += TILE) {
        const Edge<T> E = En;
        En = I.edges[min(e + TILE, e1 - 1)];
        const int a = E.w0 & 1023, ka = (E.w0 >> 10) & 3, kb = (E.w0 >> 12) & 3, kind = (E.w0 >> 14) & 3;
        bool flip = (E.w0 >> 16) & 1;
        T l, nx, ny;
        edge_normal(E.lx, E.ly, l, nx, ny);  // n: outward of a
        if constexpr (IS32<T>) {
            if (ka < 2) {
                S.gx[ka][a] = E.lx;
                S.gy[ka][a] = E.ly;
            }
        } else {
            S.gl[ka][a] = l;
            S.gx[ka][a] = nx;
            S.gy[ka][a] = ny;
        }
        if (kind == EK_LOCAL) {
            const int b = (E.w0 >> 17) & 1023;
            if constexpr (IS32<T>) {
                if (kb < 2) {
                    S.gx[kb][b] = -E.lx;
                    S.gy[kb][b] = -E.ly;
                }
            } else {
                S.gl[kb][b] = l;
                S.gx[kb][b] = -nx;
                S.gy[kb][b] = -ny;
            }
        }
        if (!UPDATE) {
            if (kind == EK_BOUNDARY) {
                const int kbc = I.slot_kbc[I.ew1[e]];
                if ((kbc & 15) == BC_INFLOW || (kbc & 15) == BC_FROUDE) {
                    const V2<T> cp = I.cellp[tile * TILE + a];
                    T hg, ung, qg;
                    if (discharge_ghost(I.bcs[kbc >> 4], kbc & 15, t_cand, cp.y, g, I.sqrtg, hg, ung, qg))
                        ghost_cfl<T, TILE>(S, l, hg, ung, g, cp.x);
                } else if ((kbc & 15) == BC_ZHYDRO) {
                    const double dg = hydrograph(I.bcs[kbc >> 4], t_cand) - double(S.huvz[a].w);
                    if (!(dg < H_DRY)) ghost_cfl<T, TILE>(S, l, T(dg), T(0), g, I.cellp[tile * TILE + a].x);
                }
            }
            continue;
        }
        const V4<T> sa = S.huvz[a];
        const double Ha = double(sa.x);
        // a's velocity in the frame (n, t)
        T una, uta;
        rotate(sa.y, sa.z, nx, ny, una, uta);
        T F0, F1, F2, ha, hb = T(0);
        T phib[NS > 0 ? NS : 1];  // other side's concentrations (edges leaving the tile)
        // the two states handed to the Riemann solver (one call for every
        // kind of edge keeps a single copy of the solver in the kernel)
        T hL, unL, utL, hR, unR, utR;
        int slot = 0, bi = 0;
        // the other cell's sediment state (Exner): Phi, dPhi, velocity, depth, bed
        T mphi = T(0), mdphi = T(0), mub = T(0), mvb = T(0), mhb = T(0), mzb = T(0);
        bool open = false, inflow_on = false, imposed = false, walled = false;
        int ihq = 0;  // internal rating curve: 1 this side upstream, -1 downstream
        T qimp = T(0);  // weir or h-Q discharge, or an active inflow's unit discharge
        if (kind != EK_BOUNDARY) {
            V4<T> sb;
            T ub, vb;
            double Hb;
            if (kind == EK_LOCAL) {
                const int b = (E.w0 >> 17) & 1023;
                sb = S.huvz[b];
                Hb = double(sb.x);
                ub = sb.y;
                vb = sb.z;
            } else {
                sb = src[I.ew1[e]];
                whole(sb);
                Hb = double(sb.x);
                const double hbd = Hb - double(sb.w);
                if constexpr (NS > 0) {
#pragma unroll
                    for (int sp = 0; sp < NS; sp++) phib[sp] = concentration(qsrc[(size_t)sp * I.n + I.ew1[e]], hbd);
                }
                const bool bwet = hbd > h_min;
                const T hh = T(hbd);
                ub = bwet ? qdiv(sb.y, hh) : T(0);
                vb = bwet ? qdiv(sb.z, hh) : T(0);
                if constexpr (MORPHO) {
                    const int jb = I.ew1[e];
                    cell_sediment(I, hbd, ub, vb, sb.w, I.cellp[jb].y, jb, mphi, mdphi);
                    mhb = hh;
                }
            }
            if constexpr (MORPHO) {
                if (kind == EK_LOCAL) {
                    const int b = (E.w0 >> 17) & 1023;
                    mphi = MS->phi[b];
                    mdphi = MS->dphi[b];
                    mhb = T(Hb - double(sb.w));
                }
                mub = ub;
                mvb = vb;
                mzb = sb.w;
            }
            T unb, utb;
            rotate(ub, vb, nx, ny, unb, utb);
            // hydrostatic reconstruction of the two modified states
            const double zs = double(sa.w > sb.w ? sa.w : sb.w);
            const double da = Ha - zs, db = Hb - zs;
            ha = da < H_DRY ? T(0) : T(da);
            hb = db < H_DRY ? T(0) : T(db);
            // canonical orientation (left = smaller original index); the
            // canonical normal is -n when a is the right cell
            hL = flip ? hb : ha;
            hR = flip ? ha : hb;
            unL = flip ? -unb : una;
            utL = flip ? -utb : uta;
            unR = flip ? -una : unb;
            utR = flip ? -uta : utb;
            // a standing internal wall (static, or dynamic before its
            // collapse time): this side sees its own reflected state.  An
            // internal rating curve is a wall for the momentum too, while
            // the discharge of its table at the upstream cell's surface
            // crosses from the side left of the tag's segment (bit 17) to
            // the other
            const int iw = IW ? (E.w0 >> 27) & 31 : 0;
            if (iw) {
                const int bc = I.iw_bc[iw - 1];
                const int bk = bc >= 0 ? I.bcs[bc].kind : -1;
                if (bk == BC_WALL || (bk == BC_DYNWALL && t < I.bcs[bc].slope) || bk == BC_HQ) {
                    const double dw = Ha - double(sa.w);
                    if (bk == BC_DYNWALL) wall_trigger(I.bcs[bc], dw, t_cand);
                    ha = dw < H_DRY ? T(0) : T(dw);
                    hL = hR = ha;
                    unL = una;
                    utL = utR = uta;
                    unR = -una;
                    flip = false;
                    walled = true;
                    if (bk == BC_HQ) {
                        const bool up = (E.w0 >> 17) & 1;
                        qimp = T(up ? imposed_outflow(I.bcs[bc], Ha, double(sa.w), I.sqrt2g)
                                    : imposed_outflow(I.bcs[bc], Hb, double(sb.w), I.sqrt2g));
                        ihq = up ? 1 : -1;
                    }
                }
            }
        } else {
            slot = I.ew1[e];
            const int kbc = I.slot_kbc[slot];
            const int bkind = kbc & 15;
            bi = kbc >> 4;
            // the ghost shares a's bed, so z* = z and h* = H - z
            const double zc = double(sa.w);
            const double da = Ha - zc;
            ha = da < H_DRY ? T(0) : T(da);
            // by default a reflective, impermeable wall: mirrored normal velocity
            hL = ha;
            unL = una;
            utL = uta;
            hR = ha;
            unR = -una;
            utR = uta;
            T hg, ung;
            if (bkind == BC_OUTFLOW || (bkind == BC_DYNWALL && t >= I.bcs[bi].slope)) {
                // transmissive (a dynamic wall after its collapse time too)
                unR = una;
                open = true;
            } else if (bkind == BC_DYNWALL) {
                wall_trigger(I.bcs[bi], da, t_cand);
            } else if (bkind == BC_INFLOW || bkind == BC_FROUDE) {
                const V2<T> cp = I.cellp[tile * TILE + a];
                const BCdev &B = I.bcs[bi];
                const bool on = discharge_ghost(B, bkind, t, cp.y, g, I.sqrtg, hg, ung, qimp);
                if (on) {
                    const double dg = (zc + double(hg)) - zc;
                    hR = dg < H_DRY ? T(0) : T(dg);
                    unR = ung;
                    utR = T(0);
                    open = inflow_on = true;
                }
                T qg;
                const bool onc = discharge_ghost(B, bkind, t_cand, cp.y, g, I.sqrtg, hg, ung, qg);
                if (onc) ghost_cfl<T, TILE>(S, l, hg, ung, g, cp.x);
            } else if (bkind == BC_UNIFORM_OUT) {
                // the normal depth of the cell's outflowing unit discharge,
                // with the cell's velocity
                const T qn = T(da) * una;
                hg = normal_depth(I.cellp[tile * TILE + a].y, g, qn > T(0) ? qn : T(0), I.bcs[bi].slope);
                const double dg = (zc + double(hg)) - zc;
                hR = dg < H_DRY ? T(0) : T(dg);
                unR = una;
                open = true;
            } else if (bkind == BC_WEIR || bkind == BC_HQ) {
                open = imposed = true;
                qimp = T(imposed_outflow(I.bcs[bi], Ha, zc, I.sqrt2g));
            } else if (bkind == BC_ZHYDRO) {
                // still water at the prescribed surface over a's bed
                const double dg = hydrograph(I.bcs[bi], t) - zc;
                hR = dg < H_DRY ? T(0) : T(dg);
                unR = T(0);
                utR = T(0);
                open = true;
                const double dc = hydrograph(I.bcs[bi], t_cand) - zc;
                if (!(dc < H_DRY)) ghost_cfl<T, TILE>(S, l, T(dc), T(0), g, I.cellp[tile * TILE + a].x);
            }
        }
        hllc(hL, unL, utL, hR, unR, utR, g, F0, F1, F2);
        if (kind != EK_BOUNDARY) {
            if (flip) F0 = -F0;  // mass leaving a
            if (walled) F0 = T(0);
            if (ihq > 0) {
                // the rating curve's discharge leaves carrying a's state
                F0 = qimp;
                F1 = (ha > T(0) ? qimp * qdiv(qimp, ha) : T(0)) + hg2 * ha * ha;
                F2 = qimp * uta;
            } else if (ihq < 0) {
                F0 = -qimp;  // and enters the downstream cell
            }
        } else {
            if (!open) F0 = T(0);  // no mass crosses a wall
            if (imposed) {
                // weir or h-Q: the boundary discharge leaves carrying the cell's state
                const T q = qimp;
                F0 = q;
                F1 = (ha > T(0) ? q * qdiv(q, ha) : T(0)) + hg2 * ha * ha;
                F2 = q * uta;
            } else if (inflow_on) {
                // an inflow imposes its discharge as the mass flux (the
                // momentum flux is the Riemann solver's), so the volume that
                // enters is the hydrograph's in any flow regime
                F0 = -qimp;
            }
        }
        if constexpr (DRAIN == DRAIN_APPLY) {
            // the flux acts only for the draining time of the cell it leaves
            T th = T(1);
            if (F0 > T(0))
                th = I.theta[tile * TILE + a];
            else if (F0 < T(0) && kind != EK_BOUNDARY)
                th = I.theta[kind == EK_LOCAL ? tile * TILE + ((E.w0 >> 17) & 1023) : I.ew1[e]];
            F0 = F0 * th;
            F1 = F1 * th;
            F2 = F2 * th;
        }
        if (kind == EK_BOUNDARY && DRAIN != DRAIN_MEASURE) {
            if (open) {
                const gptr<double> acc = I.slot_acc + 2 * slot;
                double sm = acc[0], cp = acc[1];
                neumaier(sm, cp, dt * double(l * F0));
                acc[0] = sm;
                acc[1] = cp;
            }
            if constexpr (NS > 0) {
                // the ghost repeats a's concentration, except at an active inflow
#pragma unroll
                for (int sp = 0; sp < NS; sp++) {
                    phib[sp] = inflow_on ? I.phi_in[bi * NS + sp] : SS->phi[sp][a];
                    if (open) {
                        const T A = F0 * (F0 >= T(0) ? SS->phi[sp][a] : phib[sp]);
                        double *acc = I.sslot_acc + 2 * ((size_t)slot * NS + sp);
                        double sm = acc[0], cp = acc[1];
                        neumaier(sm, cp, dt * double(l * A));
                        acc[0] = sm;
                        acc[1] = cp;
                    }
                }
            }
        }
        // fluctuations: the flux minus each side's reconstructed pressure
        // (bed slope in well-balanced form), rotated back
        const T Da = F1 - hg2 * ha * ha;
        S.c[0][ka][a] = l * F0;
        if constexpr (IS32<T>) {
            S.c[1][ka][a] = l * fmaf(Da, nx, -(F2 * ny));
            S.c[2][ka][a] = l * fmaf(Da, ny, F2 * nx);
        } else {
            S.c[1][ka][a] = l * (Da * nx - F2 * ny);
            S.c[2][ka][a] = l * (Da * ny + F2 * nx);
        }
        if constexpr (NS > 0) {
            // advective species fluxes (F0 is the mass leaving a)
            const int b = (E.w0 >> 17) & 1023;
#pragma unroll
            for (int sp = 0; sp < NS; sp++) {
                const T pa = SS->phi[sp][a], pb = kind == EK_LOCAL ? SS->phi[sp][b] : phib[sp];
                const T A = F0 * (F0 >= T(0) ? pa : pb);
                SS->c[sp][ka][a] = l * A;
                if (kind == EK_LOCAL) SS->c[sp][kb][b] = -(l * A);
            }
        }
        if constexpr (MORPHO) {
            // HLL sediment flux (eq. exner_hll, speeds eq. exner_wave_assign)
            // in the edge's canonical orientation, like the water's
            const T ua = sa.y, va = sa.z;
            const T ha_raw = T(Ha - double(sa.w));
            T cq;  // l q_B as leaving a
            if (walled) {
                cq = T(0);
            } else if (kind != EK_BOUNDARY) {
                // canonical normal n_c = flip ? -n : n; both sides' normal components with it
                const T unb_c = mub * (flip ? -nx : nx) + mvb * (flip ? -ny : ny);
                const T una_c = flip ? -una : una;
                T qa_c, l1a_c, l2a_c, qb_c, l1b_c, l2b_c;
                sed_side(MS->phi[a], MS->dphi[a], ua, va, una_c, ha_raw, g, qa_c, l1a_c, l2a_c);
                sed_side(mphi, mdphi, mub, mvb, unb_c, mhb, g, qb_c, l1b_c, l2b_c);
                // left = a unless flipped
                const T qLs = flip ? qb_c : qa_c, qRs = flip ? qa_c : qb_c;
                const T l1L = flip ? l1b_c : l1a_c, l1R = flip ? l1a_c : l1b_c;
                const T l2L = flip ? l2b_c : l2a_c, l2R = flip ? l2a_c : l2b_c;
                const T zL = flip ? mzb : sa.w, zR = flip ? sa.w : mzb;
                const T lm = l1L < l1R ? l1L : l1R;
                const T lp = l2L > l2R ? l2L : l2R;
                T q;
                if (lp > lm)
                    q = (lp * qLs - lm * qRs + lp * lm * (zR - zL)) / (lp - lm);
                else
                    q = T(0.5) * (qLs + qRs);
                cq = flip ? -(l * q) : l * q;
            } else {
                // open edges carry the cell's own normal transport, walls none
                T qa, l1a, l2a;
                sed_side(MS->phi[a], MS->dphi[a], ua, va, una, ha_raw, g, qa, l1a, l2a);
                cq = open ? l * qa : T(0);
                if (open) {
                    double *acc = I.bslot_acc + 2 * slot;
                    double sm = acc[0], cp = acc[1];
                    neumaier(sm, cp, dt * double(cq));
                    acc[0] = sm;
                    acc[1] = cp;
                }
            }
            MS->c[ka][a] = cq;
            if (kind == EK_LOCAL) MS->c[kb][(E.w0 >> 17) & 1023] = -cq;
        }
        if (kind == EK_LOCAL) {
            const int b = (E.w0 >> 17) & 1023;
            const T Db = F1 - hg2 * hb * hb;
            S.c[0][kb][b] = -(l * F0);
            if constexpr (IS32<T>) {
                S.c[1][kb][b] = -(l * fmaf(Db, nx, -(F2 * ny)));
                S.c[2][kb][b] = -(l * fmaf(Db, ny, F2 * nx));
            } else {
                S.c[1][kb][b] = -(l * (Db * nx - F2 * ny));
                S.c[2][kb][b] = -(l * (Db * ny + F2 * nx));
            }
        }
    }
    __syncthreads();
}

// CFL term of cell c of the tile with state (H, qx, qy, z), H in FP64, from
// the edge geometry left in LDS.  ap is |cell| (FP64) or 1/|cell| (FP32).  A
// dry cell contributes nothing (its inflow ghosts are in the tile's ghost
// term).
template <typename T, int TILE>
__device__ __forceinline__ CandT<T> tile_candidate(const Inst<T> &I, const TileLds<T, TILE> &S, int c, T ap,
                                                   double H, T qx, T qy, T z) {
    const T g = T(I.g);
    const double h2 = H - double(z);
    if constexpr (IS32<T>) {
        float lmax = 0.0f;
        if (h2 > I.h_min) {
            const float hh = float(h2);
            const float rh = __builtin_amdgcn_rcpf(hh);
            const float u2 = qx * rh, v2 = qy * rh;
            const float cc = qsqrt(g * hh);
            float gx[3], gy[3], gl[3];
            cell_geometry(S, c, gx, gy, gl);
#pragma unroll
            for (int k = 0; k < 3; k++)
            {
                const float lx = gx[k], ly = gy[k];
                const float lk = qsqrt(fmaf(lx, lx, ly * ly));
                lmax = fmaxf(lmax, fmaf(cc, lk, fabsf(fmaf(u2, lx, v2 * ly))));
            }
        }
        return lmax * ap;
    } else {
        double best = INFINITY;
        if (h2 > I.h_min) {
            const double hh = h2;
            const double u2 = qx / hh, v2 = qy / hh;
            const double cc = sqrt(g * hh);
            double gx[3], gy[3], gl[3];
            cell_geometry(S, c, gx, gy, gl);
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const double lam = fabs(u2 * gx[k] + v2 * gy[k]) + cc;
                const double r = cfl_term(ap, gl[k], lam);
                best = r < best ? r : best;
            }
        }
        return best;
    }
}

// Phase 2 for cell c of tile `tile`: update, friction, clip, write; returns
// the CFL term of the new state.  NS > 0: the species' specific masses get
// the same update from their advective contributions, and a cell the step
// leaves without water keeps none (the change is tallied per species).
// SRC: external sources and sinks add dt S_h to the continuity equation
// (taken at time t) before the friction split; dvol receives the volume the
// cell's source added (negative: removed), and a sink's removal leaves the
// species' concentrations unchanged (added water carries none).
template <typename T, int TILE, int NS = 0, bool SRC = false, bool MORPHO = false>
__device__ __forceinline__ CandT<T> tile_update(const Inst<T> &I, const TileLds<T, TILE> &S, int tile, int cur,
                                                double dt, const V4<T> &s, Tally<NS> &tl,
                                                const ScalarLds<T, TILE, (NS > 0 ? NS : 1)> *SS = nullptr,
                                                const T *qown = nullptr, double t = 0.0,
                                                double *dvol = nullptr,
                                                const MorphoLds<T, TILE> *MS = nullptr) {
    const int c = threadIdx.x;
    const int i = tile * TILE + c;
    if (i >= I.n) return IS32<T> ? T(0) : T(INFINITY);
    const gptr<V4<T>> __restrict__ dst = cur ? I.U0 : I.U1;
    const gptr<int16_t> __restrict__ ldst = cur ? I.L0 : I.L1;
    // FP32: the low part of the cell's surface (staged in LDS with the state)
    const T slo = IS32<T> ? S.lo[c] : T(0);
    const double h_min = I.h_min;
    const V2<T> cp = I.cellp[i];
    const T gn2 = cp.y;
    // residual in local edge order, then the conservative update
    const T R0 = S.c[0][0][c] + S.c[0][1][c] + S.c[0][2][c];
    const T R1 = S.c[1][0][c] + S.c[1][1][c] + S.c[1][2][c];
    const T R2 = S.c[2][0][c] + S.c[2][1][c] + S.c[2][2][c];
    // the new surface in FP64 (FP32: hi + lo minus the single-precision
    // increment, so no increment is lost to the spacing of the surface)
    double Hn;
    T qx, qy;
    if constexpr (IS32<T>) {
        const float w = float(dt) * cp.x;  // cp.x = 1/|cell|
        Hn = surface(s.x, slo) - double(w * R0);
        qx = fmaf(-w, R1, s.y);
        qy = fmaf(-w, R2, s.z);
    } else {
        const double w = dt * (1.0 / cp.x);
        Hn = s.x - w * R0;
        qx = s.y - w * R1;
        qy = s.z - w * R2;
    }
    double sfac = 1.0;  // fraction of the cell's water a sink left
    bool has_src = false;
    if constexpr (SRC) {
        const int r = I.src_cell[i];
        if (r >= 0) {
            has_src = true;
            const BCdev &B = I.srcs[r];
            const double hf = Hn - double(s.w);
            const double avail = hf > 0.0 ? hf : 0.0;
            double dh;
            bool empty = false;
            if (B.kind == SRC_INFINITY) {
                dh = -avail;
                empty = true;
            } else {
                dh = dt * (hydrograph(B, t) * B.length);
                if (dh < -avail) {
                    if (B.kind == SRC_AVAILABLE) {
                        dh = -avail;
                        empty = true;
                    } else {
                        atomicOr(&I.ctrl->flags, FLAG_SINK);
                    }
                }
            }
            if (empty) {
                if (avail > 0.0) Hn = double(s.w);
            } else {
                Hn = Hn + dh;
            }
            *dvol = dh * I.area[i];
            const double h2 = Hn - double(s.w);
            sfac = (dh < 0.0 && hf > 0.0) ? (h2 > 0.0 ? h2 / hf : 0.0) : 1.0;
        }
    }
    const double hn = Hn - double(s.w);
    // friction split
    T f;
    if (hn > h_min)
        f = gn2 > T(0) ? friction_factor(I.friction, T(dt), gn2, qx, qy, T(hn)) : T(1);
    else
        f = T(0);
    qx = qx * f;
    qy = qy * f;
    if (hn < 0.0) {
        // positivity: clip and account for the added volume
        tl.clip = -hn * I.area[i];
        if (I.neg_policy) atomicOr(&I.ctrl->flags, FLAG_NEGDEPTH);
        Hn = double(s.w);
        qx = T(0);
        qy = T(0);
    }
    T zn = s.w;
    if constexpr (MORPHO) {
        // eq. exnerupdateformula; the water depth is kept as the bed moves
        const T Rz = MS->c[0][c] + MS->c[1][c] + MS->c[2][c];
        double znd;
        if constexpr (IS32<T>) {
            znd = double(s.w) - double((float(dt) * cp.x) * Rz) / (1.0 - I.spor);
        } else {
            const double w = dt * (1.0 / cp.x);
            znd = s.w - (w * Rz) / (1.0 - I.spor);
        }
        if (I.zfix && znd < double(I.zfix[i])) {
            tl.bed = (1.0 - I.spor) * (double(I.zfix[i]) - znd) * I.area[i];
            znd = double(I.zfix[i]);
        }
        zn = T(znd);
        Hn = Hn + (znd - double(s.w));
    }
    if (!isfinite(Hn) || !isfinite(qx) || !isfinite(qy) || !isfinite(zn)) atomicOr(&I.ctrl->flags, FLAG_NONFINITE);
    // FP32: hi = the nearest float, the rest in the 16-bit low part
    const T Hhi = T(Hn);
    dst[i] = make4<T>(Hhi, qx, qy, zn);
    if constexpr (IS32<T>) ldst[i] = lo_code(Hhi, Hn - double(Hhi));
    if constexpr (NS > 0) {
        const gptr<T> __restrict__ qdst = cur ? I.Q0 : I.Q1;
        const bool dry = !(Hn - double(s.w) > 0.0);
#pragma unroll
        for (int sp = 0; sp < NS; sp++) {
            const T R = SS->c[sp][0][c] + SS->c[sp][1][c] + SS->c[sp][2][c];
            T q;
            if constexpr (IS32<T>) {
                q = fmaf(-(float(dt) * cp.x), R, qown[sp]);
            } else {
                q = qown[sp] - dt * (1.0 / cp.x) * R;
            }
            if (SRC && has_src) q = T(double(q) * sfac);
            if (dry) {
                tl.sp[sp] = -double(q) * I.area[i];
                q = T(0);
            }
            if (!isfinite(q)) atomicOr(&I.ctrl->flags, FLAG_NONFINITE);
            qdst[(size_t)sp * I.n + i] = q;
        }
    }
    return tile_candidate<T, TILE>(I, S, c, cp.x, Hn, qx, qy, zn);
}

// Occupancy hint (minimum waves per SIMD): what the tile's LDS allows (FP32:
// eight waves per SIMD, the most a SIMD holds; FP64: three, two at 512
// cells), so the register budget matches it.  The persistent batched kernel
// needs more registers (its member parameters and every boundary kind) and
// asks for six FP32 waves, the most it runs without spilling.
template <typename T, int TILE>
constexpr int WAVES_PER_SIMD = IS32<T> ? 8 : (TILE >= 512 ? 2 : 3);
template <typename T, int TILE, bool IW>
constexpr int WAVES_PER_SIMD_BATCHED = IS32<T> ? 6 : (TILE >= 512 ? 2 : 3);

// Adds the tile's source volume (one value per thread) to the tile's
// compensated accumulator: shuffle tree per wave, then the waves in order.
template <int TILE>
__device__ __forceinline__ void tile_source_tally(double *acc, double v) {
    __shared__ double part[TILE / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sm = acc[0], cp = acc[1];
        for (int w = 0; w < TILE / 64; w++) neumaier(sm, cp, part[w]);
        acc[0] = sm;
        acc[1] = cp;
    }
}

// The limited step (draining factors gathered per edge) and the step with
// internal walls need a few more registers: seven FP32 waves per SIMD keep
// them spill-free.
template <typename T, int TILE, bool MORE>
constexpr int WAVES_PER_SIMD_STEP = (MORE && IS32<T>) ? 7 : WAVES_PER_SIMD<T, TILE>;

template <typename T, int TILE, bool SRC = false, bool DRAIN = false, bool IW = false>
__global__ void __launch_bounds__(TILE, (WAVES_PER_SIMD_STEP<T, TILE, (DRAIN || IW)>)) k_step(Inst<T> I, int phase) {
    __shared__ TileLds<T, TILE> S;
    const bool lead = blockIdx.x == 0;
    const Level L = step_setup(I.ctrl, phase, I.cfl, I.dt_max, lead);
    if (!L.run) return;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    V4<T> own;
    tile_edges<T, TILE, true, 0, false, (DRAIN ? DRAIN_APPLY : DRAIN_NONE), IW>(I, S, tile, L.cur, L.t, L.dt,
                                                                                 L.t + L.dt, own);
    double dvol = 0.0;
    Tally<0> tl;
    CandT<T> cand = tile_update<T, TILE, 0, SRC>(I, S, tile, L.cur, L.dt, own, tl, nullptr, nullptr, L.t, &dvol);
    if constexpr (SRC) tile_source_tally<TILE>(I.src_acc + 2 * tile, dvol);
    group_tally(I.clip_acc, tile * TILE + threadIdx.x, tl.clip);
    if (threadIdx.x == 0) cand = combine(cand, ghost_value(S.ghost));
    block_finish(I.ctrl, phase, cand, L, lead, true);
}

// Draining-time pass (before a limited step, same time level): each cell's
// outgoing mass over the step, summed in local edge order, against the water
// it holds gives theta = min(1, draining time / dt), stored per cell.
template <typename T, int TILE, bool IW>
__global__ void __launch_bounds__(TILE, (WAVES_PER_SIMD<T, TILE>)) k_drain(Inst<T> I, int phase) {
    __shared__ TileLds<T, TILE> S;
    const Level L = step_setup(I.ctrl, phase, I.cfl, I.dt_max, false);
    if (!L.run) return;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    V4<T> own;
    tile_edges<T, TILE, true, 0, false, DRAIN_MEASURE, IW>(I, S, tile, L.cur, L.t, L.dt, L.t + L.dt, own);
    const int c = threadIdx.x, i = tile * TILE + c;
    if (i >= I.n) return;
    const double o0 = double(S.c[0][0][c]), o1 = double(S.c[0][1][c]), o2 = double(S.c[0][2][c]);
    const double out = (o0 > 0.0 ? o0 : 0.0) + (o1 > 0.0 ? o1 : 0.0) + (o2 > 0.0 ? o2 : 0.0);
    const double h = surface(own.x, low_part<T>(L.cur ? I.L1 : I.L0, i, own.x)) - double(own.w);
    const double vol = (h > 0.0 ? h : 0.0) * I.area[i];
    const double leave = out * L.dt;
    I.theta[i] = T(leave > vol ? vol / leave : 1.0);
}

// The step with NS passive species riding on the edge pass (tile of 256
// cells; the species' LDS lowers the occupancy, so it is a kernel of its own).
template <typename T, int TILE, int NS, bool SRC>
__global__ void __launch_bounds__(TILE) k_step_species(Inst<T> I, int phase) {
    __shared__ TileLds<T, TILE> S;
    __shared__ ScalarLds<T, TILE, NS> SS;
    const bool lead = blockIdx.x == 0;
    const Level L = step_setup(I.ctrl, phase, I.cfl, I.dt_max, lead);
    if (!L.run) return;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    V4<T> own;
    T qown[NS];
    tile_edges<T, TILE, true, NS>(I, S, tile, L.cur, L.t, L.dt, L.t + L.dt, own, &SS, qown);
    double dvol = 0.0;
    Tally<NS> tl;
    CandT<T> cand = tile_update<T, TILE, NS, SRC>(I, S, tile, L.cur, L.dt, own, tl, &SS, qown, L.t, &dvol);
    if constexpr (SRC) tile_source_tally<TILE>(I.src_acc + 2 * tile, dvol);
    const int cell = tile * TILE + threadIdx.x;
    group_tally(I.clip_acc, cell, tl.clip);
#pragma unroll
    for (int sp = 0; sp < NS; sp++) group_tally(I.sclip_acc + (size_t)2 * sp * I.ngroups, cell, tl.sp[sp]);
    if (threadIdx.x == 0) cand = combine(cand, ghost_value(S.ghost));
    block_finish(I.ctrl, phase, cand, L, lead, true);
}

// The step with the Exner module: the bed moves with the same dt from the
// state at t^n (synchronous-decoupled), its HLL sediment fluxes evaluated in
// the same edge pass (tile of 256 cells, a kernel of its own for its LDS).
template <typename T, int TILE>
__global__ void __launch_bounds__(TILE) k_step_morpho(Inst<T> I, int phase) {
    __shared__ TileLds<T, TILE> S;
    __shared__ MorphoLds<T, TILE> MS;
    const bool lead = blockIdx.x == 0;
    const Level L = step_setup(I.ctrl, phase, I.cfl, I.dt_max, lead);
    if (!L.run) return;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    V4<T> own;
    tile_edges<T, TILE, true, 0, true>(I, S, tile, L.cur, L.t, L.dt, L.t + L.dt, own, nullptr, nullptr, &MS);
    Tally<0> tl;
    CandT<T> cand = tile_update<T, TILE, 0, false, true>(I, S, tile, L.cur, L.dt, own, tl, nullptr, nullptr, L.t,
                                                          nullptr, &MS);
    group_tally(I.clip_acc, tile * TILE + threadIdx.x, tl.clip);
    group_tally(I.bclip_acc, tile * TILE + threadIdx.x, tl.bed);
    if (threadIdx.x == 0) cand = combine(cand, ghost_value(S.ghost));
    block_finish(I.ctrl, phase, cand, L, lead, true);
}

// Smallest squared speed for which a cell gets a turbulent dispersion
// tensor: zero in FP64; in FP32 1e-30 (m/s)^2, below which the single-
// precision reciprocal of |u|^2 overflows (and the tensor, of order h |u|,
// is far below anything FP32 resolves beside the molecular part).
template <typename T> __device__ __forceinline__ constexpr T speed2_floor() { return IS32<T> ? T(1e-30) : T(0); }

// CFL term of the relaxation waves of the diffusing species in one cell of
// depth h2: lambda = |u.n| + sqrt((K^m_max + K^t_nn) / zeta) over its three
// edges (geometry per local edge as the tile LDS keeps it: l*n in FP32, the
// unit normal and l in FP64); no term at or below h_min.
template <typename T>
__device__ __forceinline__ CandT<T> relax_candidate(const Inst<T> &I, const T (&gx)[3], const T (&gy)[3],
                                                    const T (&gl)[3], const V2<T> &cp, double h2, T qx, T qy) {
    CandT<T> cand = IS32<T> ? T(0) : T(INFINITY);
    if (!(h2 > I.h_min)) return cand;
    const T u2 = qdiv(qx, T(h2)), v2 = qdiv(qy, T(h2));
    const T um2 = u2 * u2 + v2 * v2;
    const T cf2 = cell_cf2(I.friction, cp.y, T(h2));
    const bool turb = um2 > speed2_floor<T>() && cf2 > T(0);
    const T at = turb ? T(h2) * qsqrt(qdiv(um2, cf2)) : T(0);
    const T dd = turb ? qdiv(T(I.daL) - T(I.daT), um2) : T(0);
    if constexpr (IS32<T>) {
        float lmax = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const float lx = gx[k], ly = gy[k];
            const float lk = qsqrt(fmaf(lx, lx, ly * ly));
            const float rl = __builtin_amdgcn_rcpf(lk);
            const float un = (u2 * lx + v2 * ly) * rl;
            const float kt = turb ? at * (float(I.daT) + dd * un * un) : 0.0f;
            const float lam = fabsf(un) + qsqrt((float(I.dKmax) + kt) / float(I.dzeta));
            lmax = fmaxf(lmax, lk * lam);
        }
        cand = lmax * cp.x;
    } else {
        double best = INFINITY;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const double un = u2 * gx[k] + v2 * gy[k];
            const double kt = turb ? at * (I.daT + dd * un * un) : 0.0;
            const double lam = fabs(un) + sqrt((I.dKmax + kt) / I.dzeta);
            const double r = cfl_term(cp.x, gl[k], lam);
            best = r < best ? r : best;
        }
        cand = best;
    }
    return cand;
}

// CFL minimum of the state of level `phase` (after an initialisation); the
// host clears the slot first.
template <typename T, int TILE>
__global__ void __launch_bounds__(TILE) k_dt_init(Inst<T> I, int phase) {
    __shared__ TileLds<T, TILE> S;
    const Ctrl *c = I.ctrl;
    Level L;
    L.t = c->s[phase].t;
    L.cur = c->s[phase].cur;
    L.dt = 0.0;
    L.steps = 0;
    L.rawmin = 0.0;
    L.run = true;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    V4<T> s;
    tile_edges<T, TILE, false>(I, S, tile, L.cur, L.t, 0.0, L.t, s);
    CandT<T> cand = IS32<T> ? T(0) : T(INFINITY);
    const int i = tile * TILE + threadIdx.x;
    if (i < I.n) {
        const V2<T> cp = I.cellp[i];
        const T slo = low_part<T>(L.cur ? I.L1 : I.L0, i, s.x);
        cand = tile_candidate<T, TILE>(I, S, threadIdx.x, cp.x, surface(s.x, slo), s.y, s.z, s.w);
        if (I.diff) {
            T gx[3], gy[3], gl[3];
            cell_geometry(S, threadIdx.x, gx, gy, gl);
            cand = combine(cand, relax_candidate(I, gx, gy, gl, cp, surface(s.x, slo) - double(s.w), s.y, s.z));
        }
    }
    if (threadIdx.x == 0) cand = combine(cand, ghost_value(S.ghost));
    block_finish(I.ctrl, phase, cand, L, false, false);
}

// ---------------------------------------------------------------------
// Species diffusion (section "Scalar advection-diffusion": the Cattaneo-type
// relaxation of eq. relaxation_terms adds per species the auxiliary
// variables psi = (psi_x, psi_y); the relaxed flux of eq. vecform_scalar2 is
// solved at each edge as the exact two-wave Riemann problem of the linear
// system in the edge's normal direction; eq. scl:updateformula with the stiff
// relaxation source -psi/zeta by the locally implicit Euler step).  A kernel
// of its own, launched after the species step on the same time level: it
// reads the state of t^n (U[cur], Q[cur], P[cur]), adds its contributions to
// the advected specific masses the species step wrote (Q[1-cur]), writes the
// auxiliary variables of t^{n+1} (P[1-cur]), resets both in cells the step
// left dry, and lowers the next time step's CFL slot by the relaxation waves
// of the new state.

// Depth and turbulent dispersion tensor (h, Kxx, Kxy, Kyy) of a cell: the
// Elder form h u_* (alpha_T I + (alpha_L - alpha_T) u u^T / |u|^2) with
// u_* = |u| / c_f (the cell's friction closure); h = 0 marks a cell at or
// below h_min, which takes part in no diffusive exchange.
template <typename T>
__device__ __forceinline__ void dispersion(const Inst<T> &I, double hd, T qx, T qy, T par, T &h, T &kxx, T &kxy,
                                           T &kyy) {
    h = kxx = kxy = kyy = T(0);
    if (!(hd > I.h_min)) return;
    h = T(hd);
    const T u = qdiv(qx, h), v = qdiv(qy, h);
    const T um2 = u * u + v * v;
    const T cf2 = cell_cf2(I.friction, par, h);
    if (!(um2 > speed2_floor<T>()) || !(cf2 > T(0))) return;
    const T us = qsqrt(qdiv(um2, cf2));
    const T a = h * us;
    const T d = qdiv(T(I.daL) - T(I.daT), um2);
    kxx = a * (T(I.daT) + d * u * u);
    kxy = a * (d * u * v);
    kyy = a * (T(I.daT) + d * v * v);
}

template <typename T, int TILE, int NS> struct DiffLds {
    T hk[4][TILE];               // per cell at t^n: depth (0: no exchange), Kxx, Kxy, Kyy
    T H[TILE], z[TILE];          // surface (high part) and bed, for the reconstructed depths
    T phi[NS][TILE];
    T psx[NS][TILE], psy[NS][TILE];
    T c[NS][3][3][TILE];         // [species][q, psi_x, psi_y][local edge][cell]
    T gx[3][TILE], gy[3][TILE];  // l*n (FP32) or the unit normal (FP64) per (local edge, cell)
    T gl[IS32<T> ? 1 : 3][IS32<T> ? 1 : TILE];
};

// The mirrored side of an edge without diffusive exchange (a boundary, a
// standing internal wall, or a neighbour at or below h_min) for cell c of
// the tile with outward normal (nx, ny): psi_n* = 0, so the species flux
// vanishes, and psi receives -(phi*/zeta) n with phi* = phi - sqrt(K_nn zeta)
// psi_n.
template <typename T, int TILE, int NS>
__device__ __forceinline__ void diff_mirror(const Inst<T> &I, DiffLds<T, TILE, NS> &S, int c, int k, T l, T nx,
                                            T ny) {
    if (!(S.hk[0][c] > T(0))) return;
    const T zeta = T(I.dzeta);
#pragma unroll
    for (int sp = 0; sp < NS; sp++) {
        const T knn = T(I.dKm[sp]) + (S.hk[1][c] * nx * nx + T(2) * S.hk[2][c] * nx * ny + S.hk[3][c] * ny * ny);
        const T psn = S.psx[sp][c] * nx + S.psy[sp][c] * ny;
        const T phs = S.phi[sp][c] - qsqrt(knn * zeta) * psn;
        S.c[sp][0][k][c] = T(0);
        S.c[sp][1][k][c] = l * (-qdiv(phs, zeta) * nx);
        S.c[sp][2][k][c] = l * (-qdiv(phs, zeta) * ny);
    }
}

template <typename T, int TILE, int NS>
__global__ void __launch_bounds__(TILE) k_diffuse(Inst<T> I, int phase) {
    __shared__ DiffLds<T, TILE, NS> S;
    const Level L = step_setup(I.ctrl, phase, I.cfl, I.dt_max, false);
    if (!L.run) return;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int c = threadIdx.x, i = tile * TILE + c;
    const gptr<const V4<T>> __restrict__ src = L.cur ? I.U1 : I.U0;
    const gptr<const T> __restrict__ qsrc = L.cur ? I.Q1 : I.Q0;
    const gptr<const V2<T>> __restrict__ psrc = (gptr<const V2<T>>)(L.cur ? I.P1 : I.P0);
    const int e1 = I.eoff[tile + 1];
    int e = I.eoff[tile] + c;
    const T zeta = T(I.dzeta);
    // phase 0: the tile's cells at t^n
    if (i < I.n) {
        const V4<T> s = src[i];
        const double hd = double(s.x) - double(s.w);
        T h, kxx, kxy, kyy;
        dispersion(I, hd, s.y, s.z, I.cellp[i].y, h, kxx, kxy, kyy);
        S.hk[0][c] = h;
        S.hk[1][c] = kxx;
        S.hk[2][c] = kxy;
        S.hk[3][c] = kyy;
        S.H[c] = s.x;
        S.z[c] = s.w;
#pragma unroll
        for (int sp = 0; sp < NS; sp++) {
            S.phi[sp][c] = concentration(qsrc[(size_t)sp * I.n + i], hd);
            const V2<T> p = psrc[(size_t)sp * I.n + i];
            S.psx[sp][c] = p.x;
            S.psy[sp][c] = p.y;
#pragma unroll
            for (int k = 0; k < 3; k++) {
                S.c[sp][0][k][c] = T(0);
                S.c[sp][1][k][c] = T(0);
                S.c[sp][2][k][c] = T(0);
            }
        }
    }
    __syncthreads();
    // phase 1: every edge of the tile once
    for (; e < e1; e += TILE) {
        const Edge<T> E = I.edges[e];
        const int a = E.w0 & 1023, ka = (E.w0 >> 10) & 3, kb = (E.w0 >> 12) & 3, kind = (E.w0 >> 14) & 3;
        const bool flip = (E.w0 >> 16) & 1;
        const int b = (E.w0 >> 17) & 1023;
        T l, nx, ny;
        edge_normal(E.lx, E.ly, l, nx, ny);  // outward of a
        if constexpr (IS32<T>) {
            S.gx[ka][a] = E.lx;
            S.gy[ka][a] = E.ly;
            if (kind == EK_LOCAL) {
                S.gx[kb][b] = -E.lx;
                S.gy[kb][b] = -E.ly;
            }
        } else {
            S.gl[ka][a] = l;
            S.gx[ka][a] = nx;
            S.gy[ka][a] = ny;
            if (kind == EK_LOCAL) {
                S.gl[kb][b] = l;
                S.gx[kb][b] = -nx;
                S.gy[kb][b] = -ny;
            }
        }
        bool closed = kind == EK_BOUNDARY;
        const int iw = (E.w0 >> 27) & 31;
        if (iw && !closed) {
            // standing walls and rating curves exchange nothing by diffusion
            const int bc = I.iw_bc[iw - 1];
            const int bk = bc >= 0 ? I.bcs[bc].kind : -1;
            if (bk == BC_WALL || (bk == BC_DYNWALL && L.t < I.bcs[bc].slope) || bk == BC_HQ) closed = true;
        }
        if (closed) {
            diff_mirror<T, TILE, NS>(I, S, a, ka, l, nx, ny);
            continue;
        }
        // the other cell's state at t^n
        T hb, kbxx, kbxy, kbyy, Hb, zb;
        T phb[NS], pxb[NS], pyb[NS];
        if (kind == EK_LOCAL) {
            hb = S.hk[0][b];
            kbxx = S.hk[1][b];
            kbxy = S.hk[2][b];
            kbyy = S.hk[3][b];
            Hb = S.H[b];
            zb = S.z[b];
#pragma unroll
            for (int sp = 0; sp < NS; sp++) {
                phb[sp] = S.phi[sp][b];
                pxb[sp] = S.psx[sp][b];
                pyb[sp] = S.psy[sp][b];
            }
        } else {
            const int j = I.ew1[e];
            const V4<T> s = src[j];
            const double hbd = double(s.x) - double(s.w);
            dispersion(I, hbd, s.y, s.z, I.cellp[j].y, hb, kbxx, kbxy, kbyy);
            Hb = s.x;
            zb = s.w;
#pragma unroll
            for (int sp = 0; sp < NS; sp++) {
                phb[sp] = concentration(qsrc[(size_t)sp * I.n + j], hbd);
                const V2<T> p = psrc[(size_t)sp * I.n + j];
                pxb[sp] = p.x;
                pyb[sp] = p.y;
            }
        }
        // the wetted cross-section both share: the smaller reconstructed depth
        const double zs = double(S.z[a] > zb ? S.z[a] : zb);
        double da = double(S.H[a]) - zs, db = double(Hb) - zs;
        if (da < H_DRY) da = 0.0;
        if (db < H_DRY) db = 0.0;
        const T hi = T(da < db ? da : db);
        if (!(S.hk[0][a] > T(0)) || !(hb > T(0)) || !(hi > T(0))) {
            diff_mirror<T, TILE, NS>(I, S, a, ka, l, nx, ny);
            if (kind == EK_LOCAL) diff_mirror<T, TILE, NS>(I, S, b, kb, l, -nx, -ny);
            continue;
        }
        // canonical orientation (left = smaller original index), n_c = flip ? -n : n
        const T cnx = flip ? -nx : nx, cny = flip ? -ny : ny;
        const T KL1 = flip ? kbxx : S.hk[1][a], KR1 = flip ? S.hk[1][a] : kbxx;
        const T KL2 = flip ? kbxy : S.hk[2][a], KR2 = flip ? S.hk[2][a] : kbxy;
        const T KL3 = flip ? kbyy : S.hk[3][a], KR3 = flip ? S.hk[3][a] : kbyy;
#pragma unroll
        for (int sp = 0; sp < NS; sp++) {
            const T kxx = T(I.dKm[sp]) + T(0.5) * (KL1 + KR1);
            const T kxy = T(0.5) * (KL2 + KR2);
            const T kyy = T(I.dKm[sp]) + T(0.5) * (KL3 + KR3);
            const T knn = kxx * cnx * cnx + T(2) * kxy * cnx * cny + kyy * cny * cny;
            const T knt = -kxx * cnx * cny + kxy * (cnx * cnx - cny * cny) + kyy * cnx * cny;
            const T pxL = flip ? pxb[sp] : S.psx[sp][a], pyL = flip ? pyb[sp] : S.psy[sp][a];
            const T pxR = flip ? S.psx[sp][a] : pxb[sp], pyR = flip ? S.psy[sp][a] : pyb[sp];
            const T fL = flip ? phb[sp] : S.phi[sp][a], fR = flip ? S.phi[sp][a] : phb[sp];
            const T pnL = pxL * cnx + pyL * cny, pnR = pxR * cnx + pyR * cny;
            const T ptL = -pxL * cny + pyL * cnx, ptR = -pxR * cny + pyR * cnx;
            T Dq, fs;
            if (knn > T(0)) {
                const T r = qsqrt(knn * zeta);
                const T pns = T(0.5) * (pnL + pnR) + qdiv(fR - fL, T(2) * r);
                fs = T(0.5) * (fL + fR) + T(0.5) * r * (pnR - pnL);
                Dq = -hi * (knn * pns + knt * (T(0.5) * (ptL + ptR)));
            } else {
                fs = T(0.5) * (fL + fR);
                Dq = T(0);
            }
            const T Dx = -qdiv(fs, zeta) * cnx, Dy = -qdiv(fs, zeta) * cny;
            // leaving the canonical left cell: +l D; a gets it with its sign
            const T sg = flip ? T(-1) : T(1);
            S.c[sp][0][ka][a] = sg * (l * Dq);
            S.c[sp][1][ka][a] = sg * (l * Dx);
            S.c[sp][2][ka][a] = sg * (l * Dy);
            if (kind == EK_LOCAL) {
                S.c[sp][0][kb][b] = -(sg * (l * Dq));
                S.c[sp][1][kb][b] = -(sg * (l * Dx));
                S.c[sp][2][kb][b] = -(sg * (l * Dy));
            }
        }
    }
    __syncthreads();
    // phase 2: update, dry reset, CFL term of the relaxation waves of the new state
    CandT<T> cand = IS32<T> ? T(0) : T(INFINITY);
    Tally<NS> tl;
    if (i < I.n) {
        const V2<T> cp = I.cellp[i];
        const gptr<V4<T>> __restrict__ udst = L.cur ? I.U0 : I.U1;
        const gptr<T> __restrict__ qdst = L.cur ? I.Q0 : I.Q1;
        const gptr<V2<T>> __restrict__ pdst = (gptr<V2<T>>)(L.cur ? I.P0 : I.P1);
        const V4<T> sn = udst[i];
        const T lon = low_part<T>(L.cur ? I.L0 : I.L1, i, sn.x);
        const double Hn = surface(sn.x, lon);
        const bool dry = !(Hn - double(sn.w) > 0.0);
        const bool active = S.hk[0][c] > T(0);
        const T rel = T(1.0 + L.dt / I.dzeta);
#pragma unroll
        for (int sp = 0; sp < NS; sp++) {
            const T Rq = S.c[sp][0][0][c] + S.c[sp][0][1][c] + S.c[sp][0][2][c];
            const T Rx = S.c[sp][1][0][c] + S.c[sp][1][1][c] + S.c[sp][1][2][c];
            const T Ry = S.c[sp][2][0][c] + S.c[sp][2][1][c] + S.c[sp][2][2][c];
            T q = qdst[(size_t)sp * I.n + i];
            T px, py;
            if constexpr (IS32<T>) {
                const float w = float(L.dt) * cp.x;
                q = fmaf(-w, Rq, q);
                px = fmaf(-w, Rx, S.psx[sp][c]) / rel;
                py = fmaf(-w, Ry, S.psy[sp][c]) / rel;
            } else {
                const double w = L.dt * (1.0 / cp.x);
                q = q - w * Rq;
                px = (S.psx[sp][c] - w * Rx) / rel;
                py = (S.psy[sp][c] - w * Ry) / rel;
            }
            if (!active || dry) {
                px = T(0);
                py = T(0);
            }
            if (dry) {
                tl.sp[sp] = -double(q) * I.area[i];
                q = T(0);
            }
            if (!isfinite(q) || !isfinite(px) || !isfinite(py)) atomicOr(&I.ctrl->flags, FLAG_NONFINITE);
            qdst[(size_t)sp * I.n + i] = q;
            V2<T> pv;
            pv.x = px;
            pv.y = py;
            pdst[(size_t)sp * I.n + i] = pv;
        }
        // relaxation waves of the new state
        T gx[3], gy[3], gl[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            gx[k] = S.gx[k][c];
            gy[k] = S.gy[k][c];
            if constexpr (IS32<T>)
                gl[k] = T(0);
            else
                gl[k] = S.gl[k][c];
        }
        cand = relax_candidate(I, gx, gy, gl, cp, Hn - double(sn.w), sn.y, sn.z);
    }
#pragma unroll
    for (int sp = 0; sp < NS; sp++) group_tally(I.sclip_acc + (size_t)2 * sp * I.ngroups, i, tl.sp[sp]);
    block_finish(I.ctrl, phase, cand, L, false, true);
}

// Persistent batched step: blocks stride over a list of (member, tile)
// pairs; each member keeps its own control block, so members step with their
// own dt and finished members cost one control-block read per tile.  IW: some
// member has internal walls (the check costs registers, so a batch without
// them runs the kernel compiled without it).
template <typename T, int TILE, bool IW>
__global__ void __launch_bounds__(TILE, (WAVES_PER_SIMD_BATCHED<T, TILE, IW>)) k_step_batched(
    const Inst<T> *__restrict__ insts, const int2 *__restrict__ tiles, int ntiles, int phase) {
    __shared__ TileLds<T, TILE> S;
    // a member's time level does not change during the launch: it is read
    // once per run of the member's tiles (and by each member's lead tile,
    // which also publishes the next level)
    int mlast = -1;
    Level L;
    for (int tt = blockIdx.x; tt < ntiles; tt += gridDim.x) {
        const int2 td = tiles[xcd_tile(tt, ntiles)];
        const Inst<T> I = insts[td.x];
        const bool lead = td.y == 0;
        if (lead || td.x != mlast) {
            L = step_setup(I.ctrl, phase, I.cfl, I.dt_max, lead);
            mlast = td.x;
        }
        if (!L.run) continue;
        V4<T> own;
        tile_edges<T, TILE, true, 0, false, DRAIN_NONE, IW>(I, S, td.y, L.cur, L.t, L.dt, L.t + L.dt, own);
        Tally<0> tl;
        CandT<T> cand = tile_update<T, TILE>(I, S, td.y, L.cur, L.dt, own, tl);
        group_tally(I.clip_acc, td.y * TILE + threadIdx.x, tl.clip);
        if (threadIdx.x == 0) cand = combine(cand, ghost_value(S.ghost));
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
    const int cur = I.ctrl->s[phase].cur;
    const gptr<const V4<T>> src = cur ? I.U1 : I.U0;
    const gptr<const int16_t> lsrc = cur ? I.L1 : I.L0;
    double s = 0.0, c = 0.0;
    for (int i = blockIdx.x * MASS_THREADS + threadIdx.x; i < I.n; i += MASS_BLOCKS * MASS_THREADS) {
        const V4<T> u = src[i];
        neumaier(s, c, (surface(u.x, low_part<T>(lsrc, i, u.x)) - double(u.w)) * I.area[i]);
    }
    const double2 r = block_csum(make_double2(s, c));
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// Sum of n compensated pairs in a fixed order (one block).
__global__ void __launch_bounds__(MASS_THREADS) k_pair_sum(const double *acc, int n, double *out) {
    double2 a = make_double2(0.0, 0.0);
    for (int k = threadIdx.x; k < n; k += MASS_THREADS) a = cadd(a, make_double2(acc[2 * k], acc[2 * k + 1]));
    const double2 r = block_csum(a);
    if (threadIdx.x == 0) out[0] = r.x + r.y;
}

// Sediment volume (1 - p) z |cell| in the same fixed order as the water volume.
template <typename T>
__global__ void __launch_bounds__(MASS_THREADS) k_bed_partial(Inst<T> I, double2 *partials, int phase) {
    const gptr<const V4<T>> src = I.ctrl->s[phase].cur ? I.U1 : I.U0;
    double s = 0.0, c = 0.0;
    for (int i = blockIdx.x * MASS_THREADS + threadIdx.x; i < I.n; i += MASS_BLOCKS * MASS_THREADS)
        neumaier(s, c, (1.0 - I.spor) * double(src[i].w) * I.area[i]);
    const double2 r = block_csum(make_double2(s, c));
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// Species mass sum q |cell| in the same fixed order as the water volume.
template <typename T>
__global__ void __launch_bounds__(MASS_THREADS) k_species_mass_partial(Inst<T> I, int sp, double2 *partials,
                                                                        int phase) {
    const gptr<const T> q = (I.ctrl->s[phase].cur ? I.Q1 : I.Q0) + (size_t)sp * I.n;
    double s = 0.0, c = 0.0;
    for (int i = blockIdx.x * MASS_THREADS + threadIdx.x; i < I.n; i += MASS_BLOCKS * MASS_THREADS)
        neumaier(s, c, double(q[i]) * I.area[i]);
    const double2 r = block_csum(make_double2(s, c));
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

template <typename T>
__global__ void __launch_bounds__(MASS_THREADS) k_species_mass_final(Inst<T> I, int sp, const double2 *partials,
                                                                      int nslots, double *out) {
    double2 acc = make_double2(0.0, 0.0);
    for (int k = threadIdx.x; k < MASS_BLOCKS; k += MASS_THREADS) acc = cadd(acc, partials[k]);
    double2 m = block_csum(acc);
    __syncthreads();
    double2 b = make_double2(0.0, 0.0);
    for (int k = threadIdx.x; k < nslots; k += MASS_THREADS) {
        const double *a = I.sslot_acc + 2 * ((size_t)k * I.ns + sp);
        b = cadd(b, make_double2(a[0], a[1]));
    }
    double2 bs = block_csum(b);
    if (threadIdx.x == 0) {
        out[0] = m.x + m.y;
        out[1] = bs.x + bs.y;
    }
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

#define SWE_TILE_DISPATCH(tile, KERNEL, ...)                                               \
    switch (tile) {                                                                        \
        case 128: hipLaunchKernelGGL((KERNEL<T, 128>), __VA_ARGS__); break;                \
        case 256: hipLaunchKernelGGL((KERNEL<T, 256>), __VA_ARGS__); break;                \
        case 512: hipLaunchKernelGGL((KERNEL<T, 512>), __VA_ARGS__); break;                \
        default: return hipErrorInvalidValue;                                              \
    }

template <typename T, bool SRC>
hipError_t launch_species(const Inst<T> &I, int phase, hipStream_t s) {
    const dim3 grid(I.ntiles), block(SPECIES_TILE);
    switch (I.ns) {
        case 1: hipLaunchKernelGGL((k_step_species<T, SPECIES_TILE, 1, SRC>), grid, block, 0, s, I, phase); break;
        case 2: hipLaunchKernelGGL((k_step_species<T, SPECIES_TILE, 2, SRC>), grid, block, 0, s, I, phase); break;
        case 3: hipLaunchKernelGGL((k_step_species<T, SPECIES_TILE, 3, SRC>), grid, block, 0, s, I, phase); break;
        case 4: hipLaunchKernelGGL((k_step_species<T, SPECIES_TILE, 4, SRC>), grid, block, 0, s, I, phase); break;
        case 5: hipLaunchKernelGGL((k_step_species<T, SPECIES_TILE, 5, SRC>), grid, block, 0, s, I, phase); break;
        default: return hipErrorInvalidValue;
    }
    if (I.diff) {
        // the diffusion of the species, on the same time level (same phase)
        switch (I.ns) {
            case 1: hipLaunchKernelGGL((k_diffuse<T, SPECIES_TILE, 1>), grid, block, 0, s, I, phase); break;
            case 2: hipLaunchKernelGGL((k_diffuse<T, SPECIES_TILE, 2>), grid, block, 0, s, I, phase); break;
            case 3: hipLaunchKernelGGL((k_diffuse<T, SPECIES_TILE, 3>), grid, block, 0, s, I, phase); break;
            case 4: hipLaunchKernelGGL((k_diffuse<T, SPECIES_TILE, 4>), grid, block, 0, s, I, phase); break;
            case 5: hipLaunchKernelGGL((k_diffuse<T, SPECIES_TILE, 5>), grid, block, 0, s, I, phase); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

// The plain step with its compiled-in options: external sources, the
// draining-time limiter (a measuring pass first), internal walls.
template <typename T, int TL, bool SRC, bool DRAIN>
hipError_t launch_plain_opts(const Inst<T> &I, int phase, hipStream_t s) {
    const dim3 grid(I.ntiles), block(TL);
    if (DRAIN) {
        if (I.iw_on)
            hipLaunchKernelGGL((k_drain<T, TL, true>), grid, block, 0, s, I, phase);
        else
            hipLaunchKernelGGL((k_drain<T, TL, false>), grid, block, 0, s, I, phase);
    }
    if (I.iw_on)
        hipLaunchKernelGGL((k_step<T, TL, SRC, DRAIN, true>), grid, block, 0, s, I, phase);
    else
        hipLaunchKernelGGL((k_step<T, TL, SRC, DRAIN, false>), grid, block, 0, s, I, phase);
    return hipGetLastError();
}
template <typename T, int TL>
hipError_t launch_plain_step(const Inst<T> &I, int phase, hipStream_t s) {
    if (I.nsrc > 0)
        return I.drain ? launch_plain_opts<T, TL, true, true>(I, phase, s) : launch_plain_opts<T, TL, true, false>(I, phase, s);
    return I.drain ? launch_plain_opts<T, TL, false, true>(I, phase, s) : launch_plain_opts<T, TL, false, false>(I, phase, s);
}

template <typename T>
hipError_t launch_step(const Inst<T> &I, int tile, int phase, hipStream_t s) {
    if (I.n <= 0) return hipSuccess;
    if (I.morpho) {
        if (tile != SPECIES_TILE || I.ns > 0 || I.nsrc > 0 || I.drain) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_step_morpho<T, SPECIES_TILE>), dim3(I.ntiles), dim3(SPECIES_TILE), 0, s, I, phase);
        return hipGetLastError();
    }
    if (I.ns > 0) {
        if (tile != SPECIES_TILE) return hipErrorInvalidValue;
        return I.nsrc > 0 ? launch_species<T, true>(I, phase, s) : launch_species<T, false>(I, phase, s);
    }
    switch (tile) {
        case 128: return launch_plain_step<T, 128>(I, phase, s);
        case 256: return launch_plain_step<T, 256>(I, phase, s);
        case 512: return launch_plain_step<T, 512>(I, phase, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_dt_init(const Inst<T> &I, int tile, int phase, hipStream_t s) {
    if (I.n <= 0) return hipSuccess;
    SWE_TILE_DISPATCH(tile, k_dt_init, dim3(I.ntiles), dim3(tile), 0, s, I, phase)
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
hipError_t launch_species_mass(const Inst<T> &I, int sp, double2 *partials, double *out, int nslots, int phase,
                               hipStream_t s) {
    if (sp < 0 || sp >= I.ns) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_species_mass_partial<T>), dim3(MASS_BLOCKS), dim3(MASS_THREADS), 0, s, I, sp, partials,
                       phase);
    hipLaunchKernelGGL((k_species_mass_final<T>), dim3(1), dim3(MASS_THREADS), 0, s, I, sp,
                       (const double2 *)partials, nslots, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bed_volume(const Inst<T> &I, double2 *partials, double *out, int phase, hipStream_t s) {
    hipLaunchKernelGGL((k_bed_partial<T>), dim3(MASS_BLOCKS), dim3(MASS_THREADS), 0, s, I, partials, phase);
    hipLaunchKernelGGL(k_pair_sum, dim3(1), dim3(MASS_THREADS), 0, s, (const double *)partials, MASS_BLOCKS, out);
    return hipGetLastError();
}

hipError_t launch_pair_sum(const double *acc, int n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_pair_sum, dim3(1), dim3(MASS_THREADS), 0, s, acc, n, out);
    return hipGetLastError();
}

template <typename T, bool IW>
hipError_t batched_occupancy(int *per, int tile) {
    switch (tile) {
        case 128: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, (const void *)k_step_batched<T, 128, IW>, 128, 0);
        case 256: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, (const void *)k_step_batched<T, 256, IW>, 256, 0);
        case 512: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per, (const void *)k_step_batched<T, 512, IW>, 512, 0);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
int batched_grid(int tile, bool iw) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const hipError_t e = iw ? batched_occupancy<T, true>(&per, tile) : batched_occupancy<T, false>(&per, tile);
    if (e == hipErrorInvalidValue) return 0;
    if (e != hipSuccess || per < 1) per = 1;
    return cus * per;
}

template <typename T>
hipError_t launch_step_batched(const Inst<T> *insts, const int2 *tiles, int ntiles, int grid, int tile, bool iw,
                               int phase, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    if (grid > ntiles) grid = ntiles;
    const dim3 g(grid), b(tile);
    switch (tile * 2 + (iw ? 1 : 0)) {
        case 256: hipLaunchKernelGGL((k_step_batched<T, 128, false>), g, b, 0, s, insts, tiles, ntiles, phase); break;
        case 257: hipLaunchKernelGGL((k_step_batched<T, 128, true>), g, b, 0, s, insts, tiles, ntiles, phase); break;
        case 512: hipLaunchKernelGGL((k_step_batched<T, 256, false>), g, b, 0, s, insts, tiles, ntiles, phase); break;
        case 513: hipLaunchKernelGGL((k_step_batched<T, 256, true>), g, b, 0, s, insts, tiles, ntiles, phase); break;
        case 1024: hipLaunchKernelGGL((k_step_batched<T, 512, false>), g, b, 0, s, insts, tiles, ntiles, phase); break;
        case 1025: hipLaunchKernelGGL((k_step_batched<T, 512, true>), g, b, 0, s, insts, tiles, ntiles, phase); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Scratch of the allocation-free batched step (swe_batch_step_noalloc): the
// work list of one call.  Each device holds its own copy until the process
// ends; host code reaches it only through the address noalloc_scratch looks
// up for the current device, never through this name.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(void **out) {
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void *addr[MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

#define SWE_INSTANTIATE(T)                                                                                  \
    template hipError_t launch_step<T>(const Inst<T> &, int, int, hipStream_t);                             \
    template hipError_t launch_dt_init<T>(const Inst<T> &, int, int, hipStream_t);                          \
    template hipError_t launch_mass<T>(const Inst<T> &, double2 *, double *, int, int, hipStream_t);        \
    template hipError_t launch_species_mass<T>(const Inst<T> &, int, double2 *, double *, int, int, hipStream_t); \
    template hipError_t launch_bed_volume<T>(const Inst<T> &, double2 *, double *, int, hipStream_t);        \
    template hipError_t launch_step_batched<T>(const Inst<T> *, const int2 *, int, int, int, bool, int, hipStream_t); \
    template int batched_grid<T>(int, bool);
SWE_INSTANTIATE(float)
SWE_INSTANTIATE(double)

}  // namespace swe
