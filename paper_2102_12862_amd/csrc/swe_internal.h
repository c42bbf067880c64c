// Internal device layout and launch interface of the shallow-water library.
// Shared by kernels.hip (device code) and the host sources; not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swe {

// Per-cell device layout (Hilbert-renumbered cells, structure of vec4s):
//   U[2][n]  vec4: (H, qx, qy, z)          ping-pong state, z carried for gathers
//   geo0[n]  vec4: (lx0, ly0, lx1, ly1)    l_k * n_k (outward) of local edges 0,1
//   geo1[n]  vec4: (lx2, ly2, 1/|cell|, g n^2)
//   nbr[3][n] int: neighbour of local edge k (bit 30 set when this cell is the
//                  right-hand cell of the edge's canonical orientation), or
//                  -1 - slot for a boundary edge
// The l*n pair of an interior edge is stored exactly negated in its two cells,
// so both cells recover bitwise opposite unit normals.
constexpr int NBR_FLIP = 1 << 30;
constexpr int NBR_MASK = NBR_FLIP - 1;

template <typename T> struct V4T;
template <> struct V4T<float> { using type = float4; };
template <> struct V4T<double> { using type = double4; };
template <typename T> using V4 = typename V4T<T>::type;

enum : int { BC_WALL = 0, BC_INFLOW = 1, BC_OUTFLOW = 2 };
enum : int { FLAG_NONFINITE = 1, FLAG_NEGDEPTH = 2, FLAG_NODT = 4 };
constexpr int MAX_BC = 64;

// Boundary condition record on the device.
struct BCdev {
    int kind;
    int npts;
    double slope;    // inflow energy slope
    double length;   // summed length of the edges carrying this condition
    const double *t; // hydrograph
    const double *Q;
};

// Per-state control block: time, the CFL minimum of the current state, the
// buffer holding it, the grid-wide arrival counter of the step in flight.
// The last block of a step to arrive advances it, so no host round trip is
// needed between steps.
struct alignas(128) Ctrl {
    double t;                     // current time t^n
    double t_end;                 // steps are capped to land on t_end
    double rawmin;                // min over cells/edges of rho / lambda for U^n
    double dt_last;               // last step taken
    unsigned long long next_min;  // running min (bit pattern) for U^{n+1}
    unsigned int arrive;          // blocks that finished the step in flight
    int cur;                      // U[cur] holds U^n
    int flags;                    // FLAG_* bits
    int pad0;
    long long steps;
    double clipped;               // volume added by positivity clips
    unsigned long long nclip;
    double pad1[4];
};
static_assert(sizeof(Ctrl) == 128, "Ctrl layout");

constexpr unsigned long long INF_BITS = 0x7FF0000000000000ull;

// Arrival groups of the grid-wide step reduction: block b reports to group
// b % NGROUPS (one cache line each), the last block of a group reports to
// the control block.  Spreading the per-block atomics over many lines keeps
// them from serialising on one address.
constexpr int NGROUPS = 64;
struct alignas(128) Group {
    unsigned long long min_bits;
    unsigned int count;
    unsigned int pad[29];
};
static_assert(sizeof(Group) == 128, "Group layout");

// Everything one kernel needs about one state.
template <typename T> struct Inst {
    V4<T> *U0;
    V4<T> *U1;
    const V4<T> *geo0;
    const V4<T> *geo1;
    const int *nbr;        // 3 arrays of n ints, back to back
    const int *slot_kbc;   // per boundary slot: kind | (bc index << 4)
    double *slot_acc;      // per boundary slot: Neumaier (sum, compensation)
    const BCdev *bcs;
    const double *area;    // |cell|, for clip volume and mass
    Ctrl *ctrl;
    Group *groups;         // NGROUPS arrival groups of this state
    int n;
    int ntiles;            // blocks of one step (batched kernel)
    double g, cfl, h_min, dt_max;
    int neg_policy;
    int pad;
};

// Launch wrappers (kernels.hip).
template <typename T>
hipError_t launch_step(const Inst<T> &I, int block, int cpt, hipStream_t s);
template <typename T>
hipError_t launch_dt_init(const Inst<T> &I, hipStream_t s);
template <typename T>
hipError_t launch_mass(const Inst<T> &I, double2 *partials, double *out, int nslots, hipStream_t s);
template <typename T>
hipError_t launch_step_batched(const Inst<T> *insts, const int2 *tiles, int ntiles, int grid, int block,
                               int cpt, hipStream_t s);
template <typename T>
int batched_grid(int block, int cpt);
constexpr int MASS_BLOCKS = 1024;
constexpr int MASS_THREADS = 256;

}  // namespace swe
