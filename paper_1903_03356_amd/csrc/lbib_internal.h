// Internal declarations shared by the HIP kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbib {

// Force field: one 64-cell row segment per wavefront of the grid kernel.
constexpr int kSegW = 64;
constexpr double kPlainStoreMaxBytes = 384.0 * (1 << 20);  // single pass: plain stores up to here
constexpr int kGridRowsPerThread = 1;  // grid kernel: nodes per thread, 4 rows apart
constexpr int kNumXcd = 8;       // MI355X: workgroups are dealt round-robin to 8 XCDs
constexpr int kIBThreads = 512;  // IB kernel block (one block per capsule)
// per-node arrays in the IB kernel's LDS: positions (4), node state (8) and
// work arrays (kNodeScratch)
constexpr int kNodeScratch = 22;
constexpr int kNodeLdsArrays = 12 + kNodeScratch;
// contact kernel: at most this many thread groups share one capsule's pairs;
// its LDS holds eight FP64 node arrays and two FP64 partial sums per thread
constexpr int kContactGroups = 8;
constexpr int kContactChunk = 128;  // capsule records staged per round in the contact kernel
constexpr size_t contact_lds_bytes(int max_nv)
{
    return sizeof(double) * (8 * (size_t)max_nv + 2 * (size_t)kIBThreads);
}

// The spread force is accumulated as a signed 64-bit fixed-point number with
// 48 fractional bits.  Integer addition is associative, so the sum of
// contributions from many nodes and capsules is bit-identical whatever order
// the atomics land in.
constexpr double kFixScale = 281474976710656.0;        // 2^48
constexpr double kFixInv = 1.0 / 281474976710656.0;
constexpr double kFixLimit = 16384.0;                  // |contribution| bound, 2^14

// Per-node arrays of BUF_NODES, each max_nodes_total long, element type real.
enum NodeField {
    NF_HX = 0, NF_HY,   // position relative to the capsule reference point (high part)
    NF_LX, NF_LY,       // low part (compensated sum)
    NF_DX, NF_DY,       // last displacement d^n = x^n - x^{n-1}
    NF_UX, NF_UY,       // node velocity u_v^n (Eq. 24)
    NF_L0,              // stress-free length of element l (node l -> l+1)
    NF_TH0,             // stress-free turning angle at node v
    NF_KS,              // stretching constant of element l
    NF_FX, NF_FY,       // last nodal force (total Dynamic / internal Kinematic)
    NF_EX, NF_EY,       // last hydrodynamic nodal force (Dynamic)
    NF_L0L,             // low part of the stress-free length (l0 = NF_L0 + NF_L0L)
    NF_CX, NF_CY,       // contact force (Eq. 27) of the current positions
    NF_R0X, NF_R0Y,     // rigid particle: body-frame offset of the node from the centroid
    NF_COUNT
};

// One lattice of a context.  A context holds a single lattice (lbib_create) or
// an ensemble of independent lattices (lbib_create_batch) that share the
// buffers, one after the other, and step in lockstep.
struct InstDev {
    int32_t nx, ny, nxp, nseg;
    int32_t periodic_y, pad0;
    int32_t periodic_x, pad1;    // periodic_x = 0: velocity inlet x = 0, pressure outlet x = nx-1
    int64_t pop_off;   // offset of the lattice's planes in a population buffer (elements)
    int64_t fib_off;   // offset in one time level of the force field (long long elements)
    int64_t flag_off;  // offset in one time level of the segment flags (ints)
    double uref_c;     // reference profile of the stored populations (GridArgs)
    double omega, gx, u_bot, u_top;
    double u_in, rho_out;        // inlet peak speed, outlet density (open channel)
};
static_assert(sizeof(InstDev) == 112, "InstDev layout");

struct CapsuleDev {
    int32_t node_offset;
    int32_t nv;
    int32_t primed;
    int32_t inst;         // lattice the capsule lives in
    double ref_x, ref_y;  // integer-valued reference point (world coordinates)
    double kb, ka, mv, A0, P0;
    // the capsule's lattice, copied from its InstDev so that the IB kernel
    // needs no second dependent load
    int32_t nx, ny, nxp, nseg;
    int32_t periodic_y, periodic_x;
    int64_t pop_off, fib_off, flag_off;
    double gx, nu;
    double uref_c;  // reference profile of the lattice's stored populations (GridArgs)
    // rigid particle (Sec. 2.3.1): nodes x_v = X + R(theta) r0_v
    int32_t rigid, pad2;
    double rX, rY, rth;        // centroid (world coordinates) and angle
    double ru[2], rum1[2];     // velocity at n and n-1 (Eq. 19)
    double rw, rwm1;           // angular velocity at n and n-1 (Eq. 20)
    double rI, rm;             // moment of inertia about the centroid, mass
    double rF[2], rM;          // last hydrodynamic (+ contact) force and torque (Eqs. 17-18)
    double pad3;
};
static_assert(sizeof(CapsuleDev) == 272, "CapsuleDev layout");

constexpr int kDiagStride = 16;  // doubles per capsule in BUF_DIAG

enum StatusBits {
    ST_WALL = 1, ST_NONFINITE = 2, ST_PATCH = 4, ST_OVERFLOW = 8, ST_MOVE = 16, ST_NEAR = 32,
    ST_SYNC = 64, ST_EDGE = 128, ST_AREA = 256
};

// Bounded wait of the far pass for the IB launch of its step (overlapped
// schedule): iterations of about 1 us before a block gives up with ST_SYNC
// (the other blocks then stop waiting as well).
constexpr int kSyncSpinLimit = 50000;

// Near region of one capsule for the overlapped grid step: world cells,
// inclusive, x unwrapped (taken modulo nx), y clamped to the lattice or
// wrapped when y is periodic.
struct NearRect {
    int x0, y0, x1, y1;
};

enum Phase { PH_PRIME = 1, PH_B = 2, PH_A = 4, PH_DIAG = 8 };

struct GridArgs {
    int nx, ny, nxp, nseg, periodic_y;
    int periodic_x;  // 0: Zou-He velocity inlet at x = 0, pressure outlet at x = nx - 1
    double omega;    // 1 / tau
    double gx;       // uniform body force
    double u_bot, u_top;
    double u_in, rho_out;  // inlet peak speed (parabolic profile), outlet density
    // reference profile of the stored populations: u_ref(y) = uref_c y (ny - 1 - y)
    // along x (the Poiseuille start of a periodic channel; 0 otherwise)
    double uref_c;
};

// Buffer bases of an IB launch; each block adds its capsule's lattice offsets.
template <typename T>
struct IBArgs {
    const T* pops;              // f*^{n-1} (the stream source of the next step)
    const long long* fib_prev;  // F^{n-1} - g, fixed point, [ny][nxp][2] per lattice
    long long* fib_next;        // F^n - g accumulator, [ny][nxp][2] per lattice
    int* flags_next;            // [ny][nseg] per lattice
    T* nodes;                   // [NF_COUNT][node_stride]
    CapsuleDev* caps;
    double* diag;               // [max_capsules][kDiagStride]
    int* status;
    int node_stride;
    int phase, dynamic;
    int patch_cap, max_nv;
    T* tape_nodes;     // if not NULL: node state written here at the end ([8][node_stride])
    double* tape_ref;  // and the reference points ([max_capsules][2])
    NearRect* rects;   // if not NULL: near region of this step, one per capsule,
    int* near_map;     // its (row, segment) units stamped with `stamp` ([ny][nseg])
    int stamp;
    int contact;       // add the contact force NF_CX/NF_CY (Dynamic B, Kinematic A)
    int4* hints;       // per capsule: the patch box (ox, oy, W, H) of its last launch, W = 0 none
    // overlapped schedule: each block adds 1 here once all its stores are
    // visible device-wide, so that the far pass can tell the launch is over
    unsigned long long* done_count;
    // membrane checks of the force pass, 0 = off: longest element length and
    // largest |A / A0 - 1| before ST_EDGE / ST_AREA
    float max_edge, max_dA;
};

// Node tape of the gradient runs: per time level, the fields NF_HX .. NF_UY
// of every node, then the force c_v F_v the node spread in that step.
constexpr int kTapeFX = 8, kTapeFY = 9;
constexpr int kTapeFields = 10;

// Spreading of a taped step (recomputed segments of the gradient runs).
template <typename T>
struct SpreadTapeArgs {
    long long* fib;         // force level of the step (accumulated), [ny][nxp][2] per lattice
    int* flags;             // its segment flags
    const T* tape;          // node tape of the step, [kTapeFields][node_stride]
    const double* ref;      // reference points of the step, [max_capsules][2]
    const CapsuleDev* caps;
    int* status;
    int node_stride;
};

// Contact forces (Eq. 27) of the current node positions.
template <typename T>
struct ContactArgs {
    T* nodes;                 // reads positions, writes NF_CX / NF_CY
    const CapsuleDev* caps;
    float4* bounds;           // per capsule: world bounding box (x0, y0, x1, y1)
    int node_stride, ncap, max_nv;
    double cutoff;
};

// ---- launchers (lbib_kernels.hip) ----
template <typename T>
hipError_t launch_init(T* pops, const GridArgs& g, int profile, double ux0, double uy0,
                       double nu, hipStream_t s);
template <typename T>
hipError_t launch_grid_step(const T* src, T* dst, const long long* fib_now, const int* flags_now,
                            long long* fib_old, int* flags_old, const GridArgs& g, hipStream_t s);
template <typename T>
hipError_t launch_grid_step_batch(const T* src, T* dst, const long long* fib_now,
                                  const int* flags_now, long long* fib_old, int* flags_old,
                                  const InstDev* inst, const int2* rounds, int tiles, int rows,
                                  int order, int grid, bool any_open, const int* near_map,
                                  int stamp, int* status, hipStream_t s);
template <typename T>
hipError_t launch_grid_far(const T* src, T* dst, const long long* fib_now, const int* flags_now,
                           long long* fib_old, int* flags_old, const int* near_map, int stamp,
                           int* status, const GridArgs& g, hipStream_t s,
                           hipEvent_t done = nullptr, const unsigned long long* ready = nullptr,
                           unsigned long long ready_target = 0);
template <typename T>
hipError_t launch_grid_near(const T* src, T* dst, const long long* fib_now, const int* flags_now,
                            long long* fib_old, int* flags_old, const NearRect* rects,
                            const CapsuleDev* caps, const InstDev* inst, int ncap, hipStream_t s);
template <typename T>
hipError_t launch_contact(const ContactArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_spread_tape(const SpreadTapeArgs<T>& a, int ncap, hipStream_t s);
template <typename T>
hipError_t contact_set_lds_limit(int max_nv);
// Blocks of the grid kernel for one lattice (a multiple of kNumXcd).
int grid_blocks(int ny, int nseg);
// Blocks of a lattice's grid pass with `rows` nodes per thread (bands of
// 4 * rows rows, dealt to the XCDs in groups of 8 bands), a multiple of 8.
int grid_blocks_rows(int ny, int nseg, int rows);
// Tiles of a lattice in the linear mapping: bands times segments, rounded up
// to a multiple of 8.
int grid_tiles_linear(int ny, int nseg, int rows);
// One IB block per capsule.  `wide`: the instance with the larger register
// budget, for a launch that runs alone with at most one block per compute
// unit (not beside the far pass).
template <typename T>
hipError_t launch_ib(const IBArgs<T>& a, int ncap, size_t lds_bytes, hipStream_t s,
                     bool wide);
template <typename T>
size_t ib_lds_bytes(int patch_cap, int max_nv);
template <typename T>
hipError_t ib_set_lds_limit(size_t bytes);

// get/set helpers.  plane: population index for the per-plane calls.
template <typename T>
hipError_t launch_get_pop_plane(const T* src, double* out, int plane, int unshift,
                                const GridArgs& g, hipStream_t s);
template <typename T>
hipError_t launch_set_pop_plane(T* dst, const double* in, int plane, const GridArgs& g,
                                hipStream_t s);
template <typename T>
hipError_t launch_get_moments(const T* src, const long long* fib, double* out,
                              const GridArgs& g, hipStream_t s);
hipError_t launch_get_force(const long long* fib, double* out, const GridArgs& g, hipStream_t s);
template <typename T>
hipError_t launch_get_nodes(const T* nodes, const CapsuleDev* caps, int cap, int nv,
                            int node_stride, int what, double* out, hipStream_t s);
template <typename T>
hipError_t launch_set_nodes(T* nodes, CapsuleDev* caps, int cap, int nv, int node_stride,
                            const double* in, hipStream_t s);

}  // namespace lbib
