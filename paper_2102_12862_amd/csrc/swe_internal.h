// Internal device layout and launch interface of the shallow-water library.
// Shared by kernels.hip (device code) and the host sources; not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swe {

// Device layout (cells renumbered along a Hilbert curve of their centroids):
//   U[2][n]   vec4 (H, qx, qy, z)  ping-pong state; z rides along so a cell's
//             whole state is one vector load
//   L[2][n]   FP32 only: the low part of the surface (H = U.x + L exactly in
//             FP64), ping-pong with U
//   cellp[n]  vec2 (|cell| in FP64, 1/|cell| in FP32; friction coefficient:
//             g n^2 for Manning and Strickler, K_s for Chezy, y_R for Bezzola)
//   edges     per tile of TILE consecutive cells, every edge touching the tile
//             once (see TileEdge in meshprep.h): packed indices and l*n
//             (12 B in FP32, 24 B in FP64)
//   ew1       per edge: the other cell's device id (edge to another tile) or
//             the boundary slot, read only by such edges
//   eoff      first edge of each tile
// A block owns one tile: it stages the tile's states in LDS, evaluates each of
// the tile's edges once, then updates its cells.
constexpr int NBR_FLIP = 1 << 30;

// The arrays the kernels touch on their hot paths are typed as global memory
// in the device pass (the host pass sees plain pointers of the same size).
// A parameter block that a kernel reads out of memory -- a batched member's
// -- otherwise leaves the compiler generic pointers, and the flat accesses it
// then emits wait on the LDS counter as well, so every LDS wait of the edge
// loop would also wait for the prefetched edge record.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename X> using gptr = __attribute__((address_space(1))) X *;
#else
template <typename X> using gptr = X *;
#endif
template <typename X> __host__ __device__ inline gptr<X> dev_ptr(X *p) { return (gptr<X>)p; }
constexpr int NBR_MASK = NBR_FLIP - 1;

template <typename T> struct V4T;
template <> struct V4T<float> { using type = float4; };
template <> struct V4T<double> { using type = double4; };
template <typename T> using V4 = typename V4T<T>::type;
template <typename T> struct V2T;
template <> struct V2T<float> { using type = float2; };
template <> struct V2T<double> { using type = double2; };
template <typename T> using V2 = typename V2T<T>::type;

// Edge record on the device: the host TileEdge's packed indices w0 and l*n
// in precision T; its w1 lives in the separate array ew1.
template <typename T> struct alignas(sizeof(T)) Edge {
    int w0;
    T lx, ly;
};
static_assert(sizeof(Edge<float>) == 12 && sizeof(Edge<double>) == 24, "edge record size");
enum : int { EK_LOCAL = 0, EK_REMOTE = 1, EK_BOUNDARY = 2 };

enum : int {
    BC_WALL = 0,
    BC_INFLOW = 1,
    BC_OUTFLOW = 2,
    BC_ZHYDRO = 3,
    BC_FROUDE = 4,
    BC_UNIFORM_OUT = 5,
    BC_WEIR = 6,
    BC_HQ = 7,
    BC_DYNWALL = 8
};
enum : int { FLAG_NONFINITE = 1, FLAG_NEGDEPTH = 2, FLAG_NODT = 4, FLAG_SINK = 8 };
// sediment transport closures, numbered as SWE_SED_* in swe.h
enum : int { SED_MPM = 0, SED_GRASS = 1, SED_EH = 2 };
// external source modes, numbered as SWE_SRC_* in swe.h
enum : int { SRC_EXACT = 0, SRC_AVAILABLE = 1, SRC_INFINITY = 2 };
// friction closures, numbered as SWE_FRICTION_* in swe.h
enum : int { FR_MANNING = 0, FR_STRICKLER = 1, FR_CHEZY = 2, FR_BEZZOLA = 3 };
constexpr int MAX_BC = 64;

// Boundary condition record on the device.
struct BCdev {
    int kind;
    int npts;
    double slope;    // energy slope, Froude number, crest elevation or collapse time (a
                     // dynamic wall's is lowered on the device when its collapse depth is reached)
    double length;   // summed length of the edges carrying this condition
    const double *t; // series times (surface elevations of an h-Q table)
    const double *Q; // discharge, or surface elevation (zhydrograph)
    double par;      // Poleni factor (weir) or collapse depth (dynamic wall; 0: none)
};

// Per-state control block, triple-buffered by step phase p = step % 3.
// A step launched with phase p reads the time level of slot p (time, CFL
// minimum of its state, buffer index), accumulates the CFL minimum of the
// state it writes into min slot p+1 with at most one atomic min per block,
// and block 0 publishes time level p+1 and clears min slot p+2 (the input of
// the previous step).  No block waits for another and no fence is needed:
// the next launch reads what this one wrote after the kernel boundary.
struct alignas(128) CtrlSlot {
    double t;         // time of this level
    double dt;        // step that produced it
    long long steps;  // steps taken to reach it
    int cur;          // U[cur] holds this level's state
    int pad0;
    double pad1[12];
};
struct alignas(128) MinSlot {
    unsigned long long bits;  // min rho/lambda of this level's state (double bits)
    unsigned long long pad[15];
};
struct alignas(128) Ctrl {
    CtrlSlot s[3];
    MinSlot m[3];
    double t_end;             // steps are capped to land on t_end
    int flags;                // FLAG_* bits
    int pad0;
    double pad1[14];
};
static_assert(sizeof(Ctrl) == 7 * 128, "Ctrl layout");

constexpr unsigned long long INF_BITS = 0x7FF0000000000000ull;

// Everything one kernel needs about one state.
template <typename T> struct Inst {
    gptr<V4<T>> U0;
    gptr<V4<T>> U1;
    // FP32: the low part of each cell's surface as a 16-bit multiple of
    // 2^-16 ulp(hi), ping-pong with U0/U1 (the surface is hi + lo); unused
    // in FP64
    gptr<int16_t> L0;
    gptr<int16_t> L1;
    gptr<const V2<T>> cellp;    // (|cell| in FP64, 1/|cell| in FP32; friction coefficient)
    gptr<const Edge<T>> edges;  // tile edge lists
    gptr<const int> ew1;        // per edge: other cell's device id or boundary slot
    gptr<const int> eoff;       // first edge of each tile (ntiles + 1)
    gptr<const int> slot_kbc;   // per boundary slot: kind | (bc index << 4)
    gptr<double> slot_acc;      // per boundary slot: Neumaier (sum, compensation)
    const BCdev *bcs;
    gptr<const double> area;    // |cell| in FP64, for the mass sum
    Ctrl *ctrl;
    // per group of 64 consecutive device cells a compensated accumulator
    // (sum, compensation) of the volume the positivity clip added
    gptr<double> clip_acc;
    int ngroups;           // ceil(n / 64)
    int n;
    int ntiles;            // tiles of this state's mesh
    double g, cfl, h_min, dt_max;
    double sqrtg, sqrt2g;  // sqrt(g) (froude inflow) and sqrt(2 g) (weir law), formed on the host
    int neg_policy;
    int friction;          // SWE_FRICTION_* closure
    // passive species (ns = 0: none): specific masses q = h phi, [ns][n] per
    // buffer (ping-pong with U), inflow concentrations [bc][ns], per boundary
    // slot and species a Neumaier accumulator, per species and cell group
    // (as clip_acc) the dry-reset tally
    gptr<T> Q0;
    gptr<T> Q1;
    const T *phi_in;
    double *sslot_acc;
    double *sclip_acc;
    int ns;
    // diffusion of the species (diff = 0: advection only): per species and
    // cell the auxiliary variables (psi_x, psi_y) [ns][n] pairs, ping-pong
    // with U; per species the molecular diffusivity, their maximum, the
    // dispersion coefficients and the relaxation time
    gptr<T> P0;
    gptr<T> P1;
    int diff;
    double dKm[5];
    double dKmax, daL, daT, dzeta;
    // external water sources and sinks (nsrc = 0: none): per cell the
    // region or -1, per region its record (kind = mode, length = factor from
    // the series value to m/s), per tile a Neumaier accumulator of the volume
    // they added
    int nsrc;
    gptr<const int> src_cell;
    const BCdev *srcs;
    double *src_acc;
    // morphodynamics (morpho = 0: off): closure, its alpha / exponent /
    // threshold, (s - 1) g d and sqrt((s - 1) g d^3), porosity; per cell the
    // non-erodible bed (or null), per boundary slot a Neumaier accumulator of
    // the sediment that left, and per cell group (as clip_acc) the fixed-bed
    // clip tally
    int morpho;
    int sclos;
    double salpha, sm, sthr, srgd, sK, spor;
    gptr<const T> zfix;
    double *bslot_acc;
    double *bclip_acc;
    // draining-time limiter (drain = 0: the bare clip): per cell the factor
    // min(1, draining time / dt) of the step being taken
    int drain;
    gptr<T> theta;
    // internal conditions: per interior-tag index the boundary condition (a
    // wall or a dynamic wall) or -1
    const int *iw_bc;
    int iw_on;  // some interior tag carries a wall
};
constexpr int MAX_SPECIES = 5;
constexpr int SPECIES_TILE = 256;  // tile size of the species-carrying step

// Launch wrappers (kernels.hip).
template <typename T>
hipError_t launch_step(const Inst<T> &I, int tile, int phase, hipStream_t s);
template <typename T>
hipError_t launch_dt_init(const Inst<T> &I, int tile, int phase, hipStream_t s);
template <typename T>
hipError_t launch_mass(const Inst<T> &I, double2 *partials, double *out, int nslots, int phase, hipStream_t s);
// sum of n compensated pairs (sum, compensation) in a fixed order -> *out
hipError_t launch_pair_sum(const double *acc, int n, double *out, hipStream_t s);
// sediment volume (1 - p) sum z |cell| in a fixed order -> out[0]
template <typename T>
hipError_t launch_bed_volume(const Inst<T> &I, double2 *partials, double *out, int phase, hipStream_t s);
// species sp: out[0] = sum q |cell| (compensated, fixed order), out[1] = mass
// that left through open boundaries
template <typename T>
hipError_t launch_species_mass(const Inst<T> &I, int sp, double2 *partials, double *out, int nslots, int phase,
                               hipStream_t s);
// iw: some member has internal walls
template <typename T>
hipError_t launch_step_batched(const Inst<T> *insts, const int2 *tiles, int ntiles, int grid, int tile, bool iw,
                               int phase, hipStream_t s);
template <typename T>
int batched_grid(int tile, bool iw);

// Allocation-free batched step: its work list lives in a file-scope device
// array (kernels.hip) of a fixed size, one per device: the kernel parameter
// blocks of at most NOALLOC_MAX_STATES states, then at most NOALLOC_MAX_TILES
// (state, tile) pairs.
constexpr int NOALLOC_MAX_STATES = 64;
constexpr int NOALLOC_MAX_TILES = 1 << 18;
constexpr size_t NOALLOC_INST_BYTES = (size_t)NOALLOC_MAX_STATES * 512;
constexpr size_t NOALLOC_SCRATCH_BYTES = NOALLOC_INST_BYTES + (size_t)NOALLOC_MAX_TILES * sizeof(int2);
static_assert(sizeof(Inst<double>) <= 512 && sizeof(Inst<float>) <= 512, "parameter block slot");
// Device address of the current device's copy of that array (looked up with
// hipGetSymbolAddress on the first call on each device).
hipError_t noalloc_scratch(void **out);
constexpr int MASS_BLOCKS = 1024;
constexpr int MASS_THREADS = 256;

}  // namespace swe
