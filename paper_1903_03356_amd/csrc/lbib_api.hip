// C-ABI host layer of the LBM - immersed boundary capsule library: argument
// validation, binding of caller-owned device buffers, the per-step launch
// schedule and state transfers.  Declarations and contracts: include/lbib.h.
#include "lbib.h"
#include "lbib_adjoint.h"
#include "lbib_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace lbib;

static thread_local std::string t_err;

struct TimedLaunch {
    int kind;  // 0 grid, 1 IB
    hipEvent_t start, stop;
};

// Tile shapes of the batched grid pass: nodes per thread (rows of a band / 4)
// and the tile order (0 banded groups of 8 bands, 1 linear over band and
// segment, 2 chunked: linear runs of a lattice's tiles, one per XCD)
constexpr int kTileShapes = 9;
constexpr int kTileRows[kTileShapes] = {1, 2, 4, 1, 2, 4, 1, 2, 4};
constexpr int kTileOrder[kTileShapes] = {0, 0, 0, 1, 1, 1, 2, 2, 2};
// Candidate resident blocks per compute unit of the persistent launch (0: one
// block per tile)
constexpr int kTileResident[4] = {0, 2, 4, 8};
// Host record of one lattice and where its arrays sit in the shared buffers.
struct Inst {
    lbib_grid grid;
    lbib_walls walls;
    double tau = 0, nu = 0;
    int nxp = 0, nseg = 0;
    size_t pop_off = 0;   // elements of a population buffer
    size_t fib_off = 0;   // long longs of one force level
    size_t flag_off = 0;  // ints of one flag level
    long long tile0[kTileShapes] = {};  // first tile in the batched pass, per tile shape
    int ncap = 0, nodes = 0;
};


// Tiles of one lattice in tile shape k.
static int lattice_tiles(int ny, int nseg, int k)
{
    return kTileOrder[k] != 0 ? grid_tiles_linear(ny, nseg, kTileRows[k])
                              : grid_blocks_rows(ny, nseg, kTileRows[k]);
}

// Buffer layout of a context: the lattices one after the other in every
// buffer; the capsule table followed by the lattice table, the round tables
// of the batched grid launch (one per tile shape), the near-region tables,
// the capsules' bounding boxes and their patch boxes.
struct Layout {
    std::vector<Inst> inst;
    int rb = 4;
    size_t pop_elems = 0, fib_level = 0, flag_level = 0;
    int max_caps = 0, max_nodes = 0, max_nv = 0;
    long long tiles[kTileShapes] = {};  // tiles of the batched pass, per tile shape
    size_t plane_max = 0;
    size_t inst_table = 0, round_table = 0, rect_table = 0, near_map = 0, bounds = 0,
           hints = 0;  // in BUF_CAPS
    size_t round_off[kTileShapes] = {};  // the round table of each tile shape
};

struct lbib_ctx {
    Layout L;
    double nu0 = 0;
    int rb = 4;
    void* buf[LBIB_NUM_BUFFERS] = {};
    hipStream_t stream = nullptr;
    int ncap = 0, nodes_used = 0;
    int patch_cap = 0;      // largest patch the on-chip budget allows
    size_t lds_bytes = 0;   // IB kernel LDS at that patch size
    int patch_use = 0;      // patch capacity of the launches: what the capsules need
    size_t lds_use = 0;
    int lds_ncap = -1;      // capsule count patch_use was computed for
    long long steps = 0;
    int mode = -1;
    std::string err;
    bool timing = false;
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> pool;
    std::vector<int> cap_off, cap_nv, cap_inst;  // host copy of the capsule table layout
    std::vector<double> cap_kb, cap_P0;
    std::vector<int> cap_rigid;
    // overlapped schedule: far part of the grid step on a second stream
    // (-1 automatic: large lattices only; 0 off; 1 on; 2 on, queue-level waits only)
    int overlap = -1;
    double contact_cutoff = 0.0;  // Eq. 27 contact force below this node distance; 0 = off
    hipStream_t s_far = nullptr;
    hipEvent_t e_ib = nullptr, e_far[2] = {nullptr, nullptr};
    // captured step blocks of the direct schedule: kGraphSteps steps from an
    // even and from an odd step (1 on; 0 and -1, the automatic default, off:
    // replays measured no faster than direct launches, whose dispatch already
    // keeps up with the kernels); captured on s_cap, replayed on `stream`; the
    // key records what they were captured for
    int graph = -1;
    hipStream_t s_cap = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int g_ncap = -1, g_mode = -1, g_patch = -1, g_tile = -1;
    double g_contact = -1.0;
    long long graph_replays = 0;
    // tile shape of the batched grid pass (lbib_set_tile, lbib_autotune):
    // index into kTileRows and resident blocks per compute unit (0: one block
    // per tile)
    int tile_shape = 0, tile_resident = 0;
    int num_cu = 256;
    int device = 0;  // HIP device that was current at create
    // overlapped schedule of one lattice: IB blocks launched so far that add
    // to the device counter (the far pass of step n waits for the count after
    // the launch of step n)
    unsigned long long ib_blocks_issued = 0;
    bool far_waits_inside = false;  // the next far launch waits on that count
    // the forcing (phase A: Dynamic steps 1-3) of step `steps` is already
    // spread into its force level, with that step's near map stamped: the
    // overlapped schedule of one lattice ends a call with it (Dynamic only:
    // there phase A writes no node state), so the next call starts with the
    // grid pass.  set_state drops it (the state it was computed from changes).
    bool a_ready = false;
    // membrane checks (lbib_set_limits), 0 = off
    float max_edge = 0.0f, max_dA = 0.0f;
};

// ------------------------------------------------- static gradient scratch
//
// Workspace of lbib_adjoint_noalloc: a file-scope device array, one copy per
// GPU that loads the library, held until the process ends.  Host code never
// passes the array's name to a kernel or a copy (in host code it names a
// host-side stand-in, not device memory): each device's address comes from
// hipGetSymbolAddress, taken once per device with that device current (at the
// first lbib_create on it, else at the entry point's first call there), and
// only that address is used.
static __device__ __align__(256) unsigned char scratch[LBIB_ADJOINT_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on device `dev`, which must be the current device.
static hipError_t resolve_scratch(int dev, void** out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// ----------------------------------------------------------------- helpers

static lbib_status fail(lbib_ctx* ctx, lbib_status code, const std::string& msg)
{
    if (ctx) ctx->err = msg;
    t_err = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(ctx, LBIB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Row stride of the lattice arrays, in cells: nx rounded up to whole 64-cell
// segments, plus one segment when that is a multiple of 512 cells, so that the
// row and plane strides are not large powers of two (equal strides map the
// nine population planes and the rows the XCDs sweep onto the same HBM
// channels).
static int row_stride(int nx)
{
    int nxp = (nx + kSegW - 1) / kSegW * kSegW;
    if (nxp % 512 == 0) nxp += kSegW;
    return nxp;
}

static bool grid_ok(const lbib_grid* g)
{
    return g && g->nx >= 8 && g->ny >= 8 && g->nx <= (1 << 20) && g->ny <= (1 << 20) &&
           (long long)g->nx * g->ny <= (1LL << 31) && (g->real_bytes == 4 || g->real_bytes == 8) &&
           g->max_capsules >= 1 && g->max_capsules <= (1 << 20) && g->max_nodes_total >= 3 &&
           g->max_nodes_total <= (1 << 26) && g->max_nodes_capsule >= 3 &&
           g->max_nodes_capsule <= 2048;
}

constexpr int kMaxInstances = 1 << 16;
constexpr int kMaxOverlapCapsules = 4096;  // near regions per step (one near-kernel block group each)
// one lattice from this size: the far kernel waits for the IB launch of its
// step inside, from the second step of a call on (step_overlap_t)
constexpr long long kFarWaitInsideCells = 1LL << 23;
constexpr long long kOverlapMinCells = 1LL << 22;  // automatic overlap from 4.2 M cells

// Fills L from the lattices' sizes and capacities; false if any is invalid or
// the totals leave the supported range.
static bool make_layout(const lbib_grid* grids, int n, Layout& L)
{
    if (!grids || n < 1 || n > kMaxInstances) return false;
    L = Layout();
    L.rb = grids[0].real_bytes;
    long long caps = 0, nodes = 0, cells = 0;
    for (int i = 0; i < n; i++) {
        const lbib_grid* g = &grids[i];
        if (!grid_ok(g) || g->real_bytes != L.rb) return false;
        Inst I;
        I.grid = *g;
        I.nxp = row_stride(g->nx);
        I.nseg = I.nxp / kSegW;
        const size_t lc = (size_t)I.nxp * g->ny;
        I.pop_off = L.pop_elems;
        I.fib_off = L.fib_level;
        I.flag_off = L.flag_level;
        for (int k = 0; k < kTileShapes; k++) {
            I.tile0[k] = L.tiles[k];
            L.tiles[k] += lattice_tiles(g->ny, I.nseg, k);
        }
        L.pop_elems += 9 * lc;
        L.fib_level += 2 * lc;
        L.flag_level += ((size_t)g->ny * I.nseg + 63) / 64 * 64;
        caps += g->max_capsules;
        nodes += g->max_nodes_total;
        cells += (long long)g->nx * g->ny;
        L.max_nv = std::max(L.max_nv, g->max_nodes_capsule);
        L.plane_max = std::max(L.plane_max, (size_t)g->nx * g->ny);
        L.inst.push_back(I);
    }
    // one-row tiles are the most numerous shape
    if (caps > (1 << 20) || nodes > (1 << 26) || L.tiles[0] > (1LL << 30) || cells > (1LL << 33))
        return false;
    L.max_caps = (int)caps;
    L.max_nodes = (int)nodes;
    L.inst_table = round256((size_t)L.max_caps * sizeof(CapsuleDev));
    L.round_table = L.inst_table + round256((size_t)n * sizeof(InstDev));
    size_t o = L.round_table;
    for (int k = 0; k < kTileShapes; k++) {
        L.round_off[k] = o;
        o += round256((size_t)(L.tiles[k] / kNumXcd) * sizeof(int2));
    }
    L.rect_table = o;
    L.near_map = L.rect_table + round256((size_t)2 * L.max_caps * sizeof(NearRect));
    L.bounds = L.near_map + round256((size_t)2 * L.flag_level * sizeof(int));
    L.hints = L.bounds + round256((size_t)L.max_caps * sizeof(float4));
    return true;
}

static size_t status_offset(const Layout& L)
{
    return (size_t)L.max_caps * kDiagStride * sizeof(double);
}

static size_t layout_bytes(const Layout& L, int id)
{
    switch (id) {
    case LBIB_BUF_POPS_A:
    case LBIB_BUF_POPS_B: return round256(L.pop_elems * L.rb);
    case LBIB_BUF_FORCE: return round256(2 * L.fib_level * sizeof(long long));
    case LBIB_BUF_FLAGS: return round256(2 * L.flag_level * sizeof(int));
    case LBIB_BUF_NODES: return round256((size_t)NF_COUNT * L.max_nodes * L.rb);
    case LBIB_BUF_CAPS:
        return L.hints + round256((size_t)L.max_caps * sizeof(int4));
    case LBIB_BUF_DIAG: return round256(status_offset(L) + 64);
    case LBIB_BUF_STAGE: {
        size_t n = 3 * L.plane_max;
        if ((size_t)6 * L.max_nodes > n) n = (size_t)6 * L.max_nodes;
        if (n < 64) n = 64;
        return round256(n * sizeof(double));
    }
    default: return 0;
    }
}

extern "C" size_t lbib_required_bytes_batch(const lbib_grid* grids, int32_t n_inst, int32_t id)
{
    Layout L;
    if (!make_layout(grids, n_inst, L)) return 0;
    return layout_bytes(L, id);
}

extern "C" size_t lbib_required_bytes(const lbib_grid* g, int32_t id)
{
    return lbib_required_bytes_batch(g, 1, id);
}

static GridArgs grid_args(const Inst& I)
{
    GridArgs g;
    g.nx = I.grid.nx;
    g.ny = I.grid.ny;
    g.nxp = I.nxp;
    g.nseg = I.nseg;
    g.periodic_y = I.walls.periodic_y;
    g.omega = 1.0 / I.tau;
    g.gx = I.walls.body_force_x;
    g.u_bot = I.walls.periodic_y ? 0.0 : I.walls.u_bottom;
    g.u_top = I.walls.periodic_y ? 0.0 : I.walls.u_top;
    g.periodic_x = I.walls.periodic_x;
    g.u_in = I.walls.periodic_x ? 0.0 : I.walls.inlet_umax;
    g.rho_out = I.walls.periodic_x ? 1.0 : I.walls.outlet_rho;
    // storage reference: the Poiseuille profile of a periodic channel that
    // starts from it (zero on both wall rows, so Zou-He sees plain deviations)
    const bool poiseuille = I.walls.init_profile == 2 && I.walls.periodic_x && !I.walls.periodic_y;
    g.uref_c = poiseuille ? I.walls.body_force_x / (2.0 * I.nu) : 0.0;
    return g;
}

static char* bufp(const lbib_ctx* c, int id) { return static_cast<char*>(c->buf[id]); }

static void* pops(const lbib_ctx* c, long long parity)
{
    return bufp(c, (parity & 1) ? LBIB_BUF_POPS_B : LBIB_BUF_POPS_A);
}

template <typename T>
static T* pops_of(const lbib_ctx* c, long long parity, const Inst& I)
{
    return static_cast<T*>(pops(c, parity)) + I.pop_off;
}

static long long* fib(const lbib_ctx* c, long long parity)
{
    return reinterpret_cast<long long*>(bufp(c, LBIB_BUF_FORCE)) + (parity & 1) * c->L.fib_level;
}

static int* flags(const lbib_ctx* c, long long parity)
{
    return reinterpret_cast<int*>(bufp(c, LBIB_BUF_FLAGS)) + (parity & 1) * c->L.flag_level;
}

static int* status_word(const lbib_ctx* c)
{
    return reinterpret_cast<int*>(bufp(c, LBIB_BUF_DIAG) + status_offset(c->L));
}

static const InstDev* inst_table(const lbib_ctx* c)
{
    return reinterpret_cast<const InstDev*>(bufp(c, LBIB_BUF_CAPS) + c->L.inst_table);
}

static bool any_open(const lbib_ctx* c)
{
    for (const Inst& I : c->L.inst)
        if (!I.walls.periodic_x) return true;
    return false;
}

static const int2* round_table(const lbib_ctx* c, int shape)
{
    return reinterpret_cast<const int2*>(bufp(c, LBIB_BUF_CAPS) + c->L.round_off[shape]);
}

static NearRect* rect_table(const lbib_ctx* c, long long parity)
{
    return reinterpret_cast<NearRect*>(bufp(c, LBIB_BUF_CAPS) + c->L.rect_table) +
           (parity & 1) * c->L.max_caps;
}

// Near map of step n: (row, segment) -> stamp n + 1 where the step's near
// regions lie (two parities, so IB(n+1) never writes the map far(n) reads).
static int* near_map(const lbib_ctx* c, long long parity)
{
    return reinterpret_cast<int*>(bufp(c, LBIB_BUF_CAPS) + c->L.near_map) +
           (parity & 1) * c->L.flag_level;
}

static int step_stamp(long long n) { return (int)((n + 1) & 0x7fffffff); }

// Device counter of finished IB blocks (overlapped schedule), beside the
// status word in the diagnostics buffer; zeroed at create and only incremented.
static unsigned long long* ib_done_counter(const lbib_ctx* c)
{
    return reinterpret_cast<unsigned long long*>(bufp(c, LBIB_BUF_DIAG) + status_offset(c->L) + 32);
}

// Undoes a forcing spread ahead (lbib_ctx::a_ready): clears the step's force
// level, its segment flags and its near map, so that the next call spreads the
// forcing again from the state as it then stands.
static lbib_status drop_pending_forcing(lbib_ctx* c)
{
    if (!c->a_ready) return LBIB_OK;
    const long long n = c->steps;
    HIPCHK(c, hipMemsetAsync(fib(c, n), 0, c->L.fib_level * sizeof(long long), c->stream));
    HIPCHK(c, hipMemsetAsync(flags(c, n), 0, c->L.flag_level * sizeof(int), c->stream));
    HIPCHK(c, hipMemsetAsync(near_map(c, n), 0, c->L.flag_level * sizeof(int), c->stream));
    c->a_ready = false;
    return LBIB_OK;
}

static hipEvent_t take_event(lbib_ctx* c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence, whose cache write-back would land
    // inside the measured interval (lbib_get_timing synchronises the stream
    // itself before it reads the events)
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// ------------------------------------------------------------------ create

static lbib_status check_lattice(const lbib_grid* grid, double tau, const lbib_walls* walls)
{
    if (grid->nx < 8 || grid->ny < 8) return fail(nullptr, LBIB_EINVAL, "nx and ny must be >= 8");
    if (grid->real_bytes != 4 && grid->real_bytes != 8)
        return fail(nullptr, LBIB_EINVAL, "real_bytes must be 4 or 8");
    if (!grid_ok(grid)) return fail(nullptr, LBIB_ECAPACITY, "grid capacities out of range");
    if (!(std::isfinite(tau) && tau > 0.5)) return fail(nullptr, LBIB_EINVAL, "tau must be > 1/2");
    if (walls->periodic_x != 0 && walls->periodic_x != 1)
        return fail(nullptr, LBIB_EINVAL, "periodic_x must be 0 or 1");
    if (walls->periodic_y != 0 && walls->periodic_y != 1)
        return fail(nullptr, LBIB_EINVAL, "periodic_y must be 0 or 1");
    if (!(std::isfinite(walls->u_bottom) && std::isfinite(walls->u_top) &&
          std::isfinite(walls->body_force_x) && std::isfinite(walls->init_ux) &&
          std::isfinite(walls->init_uy) && std::isfinite(walls->inlet_umax) &&
          std::isfinite(walls->outlet_rho)))
        return fail(nullptr, LBIB_EINVAL, "non-finite wall or profile value");
    if (walls->init_profile < 0 || walls->init_profile > 4)
        return fail(nullptr, LBIB_EINVAL, "init_profile must be 0..4");
    if (!walls->periodic_x) {
        if (walls->periodic_y || walls->u_bottom != 0.0 || walls->u_top != 0.0 ||
            walls->body_force_x != 0.0)
            return fail(nullptr, LBIB_EINVAL,
                        "an open channel (periodic_x = 0) needs stationary walls and no body force");
        if (!(walls->outlet_rho > 0.5 && walls->outlet_rho < 2.0) ||
            !(std::fabs(walls->inlet_umax) < 0.3))
            return fail(nullptr, LBIB_EINVAL, "outlet_rho must be in (0.5, 2), |inlet_umax| < 0.3");
    } else if (walls->init_profile == 4) {
        return fail(nullptr, LBIB_EINVAL, "init_profile 4 (inlet parabola) needs periodic_x = 0");
    }
    return LBIB_OK;
}

static lbib_status create_common(const lbib_grid* grids, const double* taus,
                                 const lbib_walls* walls, int32_t n_inst,
                                 void* const* device_buffers, int32_t n_buffers, void* hip_stream,
                                 lbib_ctx** out)
{
    if (!out) return fail(nullptr, LBIB_EINVAL, "out is NULL");
    if (!grids || !taus || !walls || !device_buffers)
        return fail(nullptr, LBIB_EINVAL, "NULL argument");
    if (n_inst < 1 || n_inst > kMaxInstances)
        return fail(nullptr, LBIB_EINVAL, "n_inst must be 1..65536");
    for (int i = 0; i < n_inst; i++) {
        lbib_status s = check_lattice(&grids[i], taus[i], &walls[i]);
        if (s != LBIB_OK) return s;
        if (grids[i].real_bytes != grids[0].real_bytes)
            return fail(nullptr, LBIB_EINVAL, "all lattices of a batch need the same real_bytes");
    }
    if (n_buffers != LBIB_NUM_BUFFERS)
        return fail(nullptr, LBIB_EINVAL, "n_buffers must be LBIB_NUM_BUFFERS");
    for (int i = 0; i < LBIB_NUM_BUFFERS; i++)
        if (!device_buffers[i]) return fail(nullptr, LBIB_EINVAL, "NULL device buffer");
    Layout L;
    if (!make_layout(grids, n_inst, L))
        return fail(nullptr, LBIB_ECAPACITY, "batch totals out of range");

    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(nullptr, LBIB_EDEVICE, "no HIP device");

    lbib_ctx* c = new lbib_ctx();
    c->L = L;
    c->device = dev;
    {
        // set-up of the static gradient scratch on this device; a failure
        // here only matters to lbib_adjoint_noalloc, which tries again
        void* p = nullptr;
        (void)resolve_scratch(dev, &p);
    }
    if (prop.multiProcessorCount > 0) c->num_cu = prop.multiProcessorCount;
    for (int i = 0; i < n_inst; i++) {
        Inst& I = c->L.inst[i];
        I.walls = walls[i];
        I.tau = taus[i];
        I.nu = (taus[i] - 0.5) / 3.0;
    }
    c->rb = L.rb;
    for (int i = 0; i < LBIB_NUM_BUFFERS; i++) c->buf[i] = device_buffers[i];
    c->stream = static_cast<hipStream_t>(hip_stream);
    auto bail = [&](lbib_status code, const std::string& m) {
        delete c;
        return fail(nullptr, code, m);
    };

    // LDS of the IB kernel: node scratch for the largest capsule, the rest
    // holds the capsule's fluid patch.
    const size_t lds_max = prop.sharedMemPerBlock > 0 ? prop.sharedMemPerBlock : 65536;
    const size_t budget = lds_max - 1024;  // static shared memory of the kernel
    const size_t per_node = (size_t)kNodeLdsArrays * c->rb, per_cell = (size_t)3 * c->rb;
    const size_t node_bytes = per_node * L.max_nv;
    if (node_bytes + 1024 * per_cell > budget)
        return bail(LBIB_ECAPACITY, "max_nodes_capsule too large for the on-chip memory");
    c->patch_cap = (int)((budget - node_bytes) / per_cell);
    c->lds_bytes = c->rb == 4 ? ib_lds_bytes<float>(c->patch_cap, L.max_nv)
                              : ib_lds_bytes<double>(c->patch_cap, L.max_nv);
    hipError_t e = c->rb == 4 ? ib_set_lds_limit<float>(c->lds_bytes)
                              : ib_set_lds_limit<double>(c->lds_bytes);
    if (e != hipSuccess) return bail(LBIB_EDEVICE, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));

    const int zero_ids[] = {LBIB_BUF_POPS_B, LBIB_BUF_FORCE, LBIB_BUF_FLAGS, LBIB_BUF_NODES,
                            LBIB_BUF_CAPS, LBIB_BUF_DIAG};
    for (int id : zero_ids) {
        e = hipMemsetAsync(c->buf[id], 0, layout_bytes(L, id), c->stream);
        if (e != hipSuccess) return bail(LBIB_EDEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
    }
    // lattice table and block-round table of the batched grid launch
    std::vector<InstDev> tab(n_inst);
    std::vector<int2> rounds[kTileShapes];
    for (int k = 0; k < kTileShapes; k++) rounds[k].resize(L.tiles[k] / kNumXcd);
    for (int i = 0; i < n_inst; i++) {
        const Inst& I = c->L.inst[i];
        const GridArgs g = grid_args(I);
        InstDev& d = tab[i];
        std::memset(&d, 0, sizeof(d));
        d.nx = g.nx;
        d.ny = g.ny;
        d.nxp = g.nxp;
        d.nseg = g.nseg;
        d.periodic_y = g.periodic_y;
        d.periodic_x = g.periodic_x;
        d.u_in = g.u_in;
        d.rho_out = g.rho_out;
        d.pop_off = (int64_t)I.pop_off;
        d.fib_off = (int64_t)I.fib_off;
        d.flag_off = (int64_t)I.flag_off;
        d.omega = g.omega;
        d.gx = g.gx;
        d.u_bot = g.u_bot;
        d.u_top = g.u_top;
        d.uref_c = g.uref_c;
        for (int k = 0; k < kTileShapes; k++) {
            const int r0 = (int)(I.tile0[k] / kNumXcd);
            const int r1 = r0 + lattice_tiles(g.ny, g.nseg, k) / kNumXcd;
            for (int r = r0; r < r1; r++) rounds[k][r] = make_int2(i, r0);
        }
    }
    e = hipMemcpyAsync(bufp(c, LBIB_BUF_CAPS) + L.inst_table, tab.data(),
                       tab.size() * sizeof(InstDev), hipMemcpyHostToDevice, c->stream);
    for (int k = 0; k < kTileShapes && e == hipSuccess; k++)
        if (!rounds[k].empty())
            e = hipMemcpyAsync(bufp(c, LBIB_BUF_CAPS) + L.round_off[k], rounds[k].data(),
                               rounds[k].size() * sizeof(int2), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return bail(LBIB_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    for (int i = 0; i < n_inst && e == hipSuccess; i++) {
        const Inst& I = c->L.inst[i];
        const GridArgs g = grid_args(I);
        e = c->rb == 4 ? launch_init<float>(pops_of<float>(c, 0, I), g, I.walls.init_profile,
                                            I.walls.init_ux, I.walls.init_uy, I.nu, c->stream)
                       : launch_init<double>(pops_of<double>(c, 0, I), g, I.walls.init_profile,
                                             I.walls.init_ux, I.walls.init_uy, I.nu, c->stream);
    }
    if (e != hipSuccess) return bail(LBIB_EDEVICE, std::string("init kernel: ") + hipGetErrorString(e));
    // the host tables above must outlive their copies
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return bail(LBIB_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    *out = c;
    return LBIB_OK;
}

extern "C" lbib_status lbib_create(const lbib_grid* grid, double tau, const lbib_walls* walls,
                                   void* const* device_buffers, int32_t n_buffers,
                                   void* hip_stream, lbib_ctx** out)
{
    return create_common(grid, &tau, walls, 1, device_buffers, n_buffers, hip_stream, out);
}

extern "C" lbib_status lbib_create_batch(const lbib_grid* grids, const double* taus,
                                         const lbib_walls* walls, int32_t n_inst,
                                         void* const* device_buffers, int32_t n_buffers,
                                         void* hip_stream, lbib_ctx** out)
{
    return create_common(grids, taus, walls, n_inst, device_buffers, n_buffers, hip_stream, out);
}

extern "C" int32_t lbib_num_lattices(const lbib_ctx* c)
{
    return c ? (int32_t)c->L.inst.size() : -1;
}

// ------------------------------------------------------------- add_capsule

template <typename T>
static lbib_status add_capsule_t(lbib_ctx* c, int inst, const double* xy, int n, const double* ks,
                                 int n_ks, double kb, double ka, double mass, int32_t* id,
                                 bool rigid = false, double inertia = 0.0)
{
    Inst& I = c->L.inst[inst];
    // stress-free shape (Sec. 2.2.1): element lengths, turning angles, area, perimeter
    std::vector<double> l0(n), th0(n);
    double A2 = 0, P = 0, mx = 0, my = 0;
    double minx = 1e300, maxx = -1e300, miny = 1e300, maxy = -1e300;
    for (int v = 0; v < n; v++) {
        const int m = (v + 1) % n, p = (v + n - 1) % n;
        const double tx = xy[2 * m] - xy[2 * v], ty = xy[2 * m + 1] - xy[2 * v + 1];
        l0[v] = std::sqrt(tx * tx + ty * ty);
        P += l0[v];
        A2 += xy[2 * v] * xy[2 * m + 1] - xy[2 * m] * xy[2 * v + 1];
        const double ax = xy[2 * v] - xy[2 * p], ay = xy[2 * v + 1] - xy[2 * p + 1];
        th0[v] = std::atan2(ax * ty - ay * tx, ax * tx + ay * ty);
        mx += xy[2 * v];
        my += xy[2 * v + 1];
        minx = std::fmin(minx, xy[2 * v]);
        maxx = std::fmax(maxx, xy[2 * v]);
        miny = std::fmin(miny, xy[2 * v + 1]);
        maxy = std::fmax(maxy, xy[2 * v + 1]);
        if (l0[v] <= 0.0) return fail(c, LBIB_EINVAL, "coincident consecutive nodes");
    }
    const double A0 = 0.5 * A2;
    if (!(A0 > 0)) return fail(c, LBIB_EINVAL, "nodes must be counter-clockwise (positive area)");
    const long long W = (long long)std::floor(maxx) - (long long)std::floor(minx) + 7;
    const long long H = (long long)std::floor(maxy) - (long long)std::floor(miny) + 7;
    if (W * H > c->patch_cap)
        return fail(c, LBIB_ECAPACITY, "capsule patch exceeds the on-chip capacity");

    const double refx = std::nearbyint(mx / n), refy = std::nearbyint(my / n);
    const int off = c->nodes_used;
    const size_t S = c->L.max_nodes;
    std::vector<T> f((size_t)NF_COUNT * n, T(0));
    for (int v = 0; v < n; v++) {
        const double rx = xy[2 * v] - refx, ry = xy[2 * v + 1] - refy;
        const T hx = (T)rx, hy = (T)ry;
        f[NF_HX * n + v] = hx;
        f[NF_HY * n + v] = hy;
        f[NF_LX * n + v] = (T)(rx - (double)hx);
        f[NF_LY * n + v] = (T)(ry - (double)hy);
        f[NF_L0 * n + v] = (T)l0[v];
        f[NF_L0L * n + v] = (T)(l0[v] - (double)(T)l0[v]);
        f[NF_TH0 * n + v] = (T)th0[v];
        f[NF_KS * n + v] = (T)(n_ks == 1 ? ks[0] : ks[v]);
    }
    // rigid particle: area centroid and body-frame offsets of the nodes
    double rcx = 0.0, rcy = 0.0;
    if (rigid) {
        double a2 = 0.0;
        for (int v = 0; v < n; v++) {
            const int m = (v + 1) % n;
            const double cr = xy[2 * v] * xy[2 * m + 1] - xy[2 * m] * xy[2 * v + 1];
            a2 += cr;
            rcx += (xy[2 * v] + xy[2 * m]) * cr;
            rcy += (xy[2 * v + 1] + xy[2 * m + 1]) * cr;
        }
        rcx /= 3.0 * a2;
        rcy /= 3.0 * a2;
        for (int v = 0; v < n; v++) {
            f[NF_R0X * n + v] = (T)(xy[2 * v] - rcx);
            f[NF_R0Y * n + v] = (T)(xy[2 * v + 1] - rcy);
        }
    }
    for (int k = 0; k < NF_COUNT; k++)
        HIPCHK(c, hipMemcpyAsync(bufp(c, LBIB_BUF_NODES) + (k * S + off) * sizeof(T),
                                 f.data() + (size_t)k * n, n * sizeof(T), hipMemcpyHostToDevice,
                                 c->stream));
    CapsuleDev cd;
    std::memset(&cd, 0, sizeof(cd));
    cd.node_offset = off;
    cd.nv = n;
    cd.primed = 0;
    cd.ref_x = refx;
    cd.ref_y = refy;
    cd.kb = kb;
    cd.ka = ka;
    cd.mv = mass / n;
    cd.A0 = A0;
    cd.P0 = P;
    cd.inst = inst;
    const GridArgs g = grid_args(I);
    cd.nx = g.nx;
    cd.ny = g.ny;
    cd.nxp = g.nxp;
    cd.nseg = g.nseg;
    cd.periodic_y = g.periodic_y;
    cd.periodic_x = g.periodic_x;
    cd.pop_off = (int64_t)I.pop_off;
    cd.fib_off = (int64_t)I.fib_off;
    cd.flag_off = (int64_t)I.flag_off;
    cd.gx = g.gx;
    cd.nu = I.nu;
    cd.uref_c = g.uref_c;
    if (rigid) {
        cd.rigid = 1;
        cd.rX = rcx;
        cd.rY = rcy;
        cd.rI = inertia;
        cd.rm = mass;
    }
    HIPCHK(c, hipMemcpyAsync(bufp(c, LBIB_BUF_CAPS) + (size_t)c->ncap * sizeof(CapsuleDev), &cd,
                             sizeof(cd), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *id = c->ncap;
    c->cap_off.push_back(off);
    c->cap_nv.push_back(n);
    c->cap_inst.push_back(inst);
    c->cap_kb.push_back(kb);
    c->cap_P0.push_back(P);
    c->cap_rigid.push_back(rigid ? 1 : 0);
    c->ncap++;
    c->nodes_used += n;
    I.ncap++;
    I.nodes += n;
    return LBIB_OK;
}

extern "C" lbib_status lbib_add_capsule_to(lbib_ctx* c, int32_t inst, const double* xy,
                                           int32_t n, const double* ks, int32_t n_ks, double kb,
                                           double ka, double mass, int32_t* id)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    if (!xy || !ks || !id) return fail(c, LBIB_EINVAL, "NULL argument");
    if (inst < 0 || inst >= (int)c->L.inst.size()) return fail(c, LBIB_EINVAL, "bad lattice index");
    if (c->steps > 0) return fail(c, LBIB_ESTATE, "capsules must be added before the first step");
    const Inst& I = c->L.inst[inst];
    if (n < 3) return fail(c, LBIB_EINVAL, "a capsule needs at least 3 nodes");
    if (n_ks != 1 && n_ks != n) return fail(c, LBIB_EINVAL, "n_ks must be 1 or n");
    if (n > I.grid.max_nodes_capsule)
        return fail(c, LBIB_ECAPACITY, "n exceeds max_nodes_capsule");
    if (I.ncap >= I.grid.max_capsules) return fail(c, LBIB_ECAPACITY, "capsule table full");
    if (I.nodes + n > I.grid.max_nodes_total) return fail(c, LBIB_ECAPACITY, "node arrays full");
    if (!(std::isfinite(kb) && std::isfinite(ka) && std::isfinite(mass) && mass > 0))
        return fail(c, LBIB_EINVAL, "kb, ka must be finite and mass > 0");
    for (int i = 0; i < n_ks; i++)
        if (!(std::isfinite(ks[i]) && ks[i] >= 0)) return fail(c, LBIB_EINVAL, "ks must be >= 0");
    for (int v = 0; v < 2 * n; v++)
        if (!std::isfinite(xy[v])) return fail(c, LBIB_EINVAL, "non-finite node coordinate");
    if (!I.walls.periodic_y)
        for (int v = 0; v < n; v++)
            if (xy[2 * v + 1] < 3.0 || xy[2 * v + 1] > I.grid.ny - 4.0)
                return fail(c, LBIB_EINVAL, "nodes must satisfy 3 <= y <= ny - 4");
    if (!I.walls.periodic_x)
        for (int v = 0; v < n; v++)
            if (xy[2 * v] < 3.0 || xy[2 * v] > I.grid.nx - 4.0)
                return fail(c, LBIB_EINVAL, "open channel: nodes must satisfy 3 <= x <= nx - 4");
    return c->rb == 4 ? add_capsule_t<float>(c, inst, xy, n, ks, n_ks, kb, ka, mass, id)
                      : add_capsule_t<double>(c, inst, xy, n, ks, n_ks, kb, ka, mass, id);
}

extern "C" lbib_status lbib_add_rigid_to(lbib_ctx* c, int32_t inst, const double* xy, int32_t n,
                                         double mass, double inertia, int32_t* id)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    if (!xy || !id) return fail(c, LBIB_EINVAL, "NULL argument");
    if (!(std::isfinite(inertia) && inertia > 0))
        return fail(c, LBIB_EINVAL, "inertia must be finite and > 0");
    if (c->mode == LBIB_KINEMATIC)
        return fail(c, LBIB_ESTATE, "rigid particles move with the Dynamic scheme only");
    const double ks = 0.0;
    // the checks of lbib_add_capsule_to, then the rigid record
    if (inst < 0 || inst >= (int)c->L.inst.size()) return fail(c, LBIB_EINVAL, "bad lattice index");
    if (c->steps > 0) return fail(c, LBIB_ESTATE, "capsules must be added before the first step");
    const Inst& I = c->L.inst[inst];
    if (n < 3) return fail(c, LBIB_EINVAL, "a capsule needs at least 3 nodes");
    if (n > I.grid.max_nodes_capsule)
        return fail(c, LBIB_ECAPACITY, "n exceeds max_nodes_capsule");
    if (I.ncap >= I.grid.max_capsules) return fail(c, LBIB_ECAPACITY, "capsule table full");
    if (I.nodes + n > I.grid.max_nodes_total) return fail(c, LBIB_ECAPACITY, "node arrays full");
    if (!(std::isfinite(mass) && mass > 0)) return fail(c, LBIB_EINVAL, "mass must be > 0");
    for (int v = 0; v < 2 * n; v++)
        if (!std::isfinite(xy[v])) return fail(c, LBIB_EINVAL, "non-finite node coordinate");
    if (!I.walls.periodic_y)
        for (int v = 0; v < n; v++)
            if (xy[2 * v + 1] < 3.0 || xy[2 * v + 1] > I.grid.ny - 4.0)
                return fail(c, LBIB_EINVAL, "nodes must satisfy 3 <= y <= ny - 4");
    if (!I.walls.periodic_x)
        for (int v = 0; v < n; v++)
            if (xy[2 * v] < 3.0 || xy[2 * v] > I.grid.nx - 4.0)
                return fail(c, LBIB_EINVAL, "open channel: nodes must satisfy 3 <= x <= nx - 4");
    return c->rb == 4 ? add_capsule_t<float>(c, inst, xy, n, &ks, 1, 0.0, 0.0, mass, id, true, inertia)
                      : add_capsule_t<double>(c, inst, xy, n, &ks, 1, 0.0, 0.0, mass, id, true,
                                              inertia);
}

extern "C" lbib_status lbib_add_capsule(lbib_ctx* c, const double* xy, int32_t n, const double* ks,
                                        int32_t n_ks, double kb, double ka, double mass,
                                        int32_t* id)
{
    return lbib_add_capsule_to(c, 0, xy, n, ks, n_ks, kb, ka, mass, id);
}

// -------------------------------------------------------------------- step

// Patch capacity of the IB launches: a closed polygon of perimeter P fits in
// a square of side P / 2, so (P0 + 8)^2 cells hold the patch (bounding box
// plus the 3-cell halo) of any shape up to twice the stress-free perimeter P0
// of the largest capsule.  Smaller LDS per block lets more capsules share a
// compute unit; a capsule that outgrows it raises LBIB_FLAG_PATCH.
template <typename T>
static void size_patches(lbib_ctx* c)
{
    if (c->lds_ncap == c->ncap) return;
    double pmax = 0.0;
    for (double p : c->cap_P0) pmax = std::max(pmax, p);
    const double side = std::ceil(pmax) + 8.0;
    const double need = side * side;
    c->patch_use = need < (double)c->patch_cap ? (int)need : c->patch_cap;
    c->lds_use = ib_lds_bytes<T>(c->patch_use, c->L.max_nv);
    c->lds_ncap = c->ncap;
}

template <typename T>
static IBArgs<T> ib_args(const lbib_ctx* c, long long n, int phase)
{
    // state n: populations f*^{n-1} in buffer n%2, force F^{n-1} in level (n-1)%2
    IBArgs<T> a;
    a.pops = static_cast<const T*>(pops(c, n));
    a.fib_prev = fib(c, n + 1);
    a.fib_next = fib(c, n);
    a.flags_next = flags(c, n);
    a.nodes = reinterpret_cast<T*>(bufp(c, LBIB_BUF_NODES));
    a.caps = reinterpret_cast<CapsuleDev*>(bufp(c, LBIB_BUF_CAPS));
    a.diag = reinterpret_cast<double*>(bufp(c, LBIB_BUF_DIAG));
    a.status = status_word(c);
    a.node_stride = c->L.max_nodes;
    a.phase = phase;
    a.dynamic = c->mode == LBIB_DYNAMIC;
    a.patch_cap = c->patch_use;
    a.max_nv = c->L.max_nv;
    a.tape_nodes = nullptr;
    a.tape_ref = nullptr;
    a.rects = nullptr;
    a.near_map = nullptr;
    a.stamp = 0;
    a.contact = c->contact_cutoff > 0.0;
    a.hints = reinterpret_cast<int4*>(bufp(c, LBIB_BUF_CAPS) + c->L.hints);
    a.done_count = nullptr;
    a.max_edge = c->max_edge;
    a.max_dA = c->max_dA;
    return a;
}

// The IB kernel's larger register budget holds one block per compute unit; it
// serves the launches that run alone (no near regions: not beside a far pass)
// and fit the device in one round.
template <typename T>
static bool ib_wide(const lbib_ctx* c, const IBArgs<T>& a)
{
    return a.rects == nullptr && c->ncap <= c->num_cu;
}

template <typename T>
static lbib_status launch_timed(lbib_ctx* c, int kind, hipError_t (*fn)(lbib_ctx*, void*),
                                void* arg, hipStream_t on = nullptr)
{
    const hipStream_t st = on ? on : c->stream;
    TimedLaunch t{kind, nullptr, nullptr};
    if (c->timing) {
        t.start = take_event(c);
        t.stop = take_event(c);
        if (!t.start || !t.stop) return fail(c, LBIB_EDEVICE, "hipEventCreate failed");
        HIPCHK(c, hipEventRecord(t.start, st));
    }
    HIPCHK(c, fn(c, arg));
    if (c->timing) {
        HIPCHK(c, hipEventRecord(t.stop, st));
        c->timed.push_back(t);
    }
    return LBIB_OK;
}

template <typename T>
struct IBLaunch {
    long long n;
    int phase;
    bool rects;
};

template <typename T>
static hipError_t do_ib(lbib_ctx* c, void* p)
{
    const IBLaunch<T>* q = static_cast<const IBLaunch<T>*>(p);
    IBArgs<T> a = ib_args<T>(c, q->n, q->phase);
    if (q->rects) {
        a.rects = rect_table(c, q->n);
        a.near_map = near_map(c, q->n);
        a.stamp = step_stamp(q->n);
        if (c->L.inst.size() == 1) a.done_count = ib_done_counter(c);
    }
    hipError_t e = launch_ib<T>(a, c->ncap, c->lds_use, c->stream, ib_wide(c, a));
    if (e == hipSuccess && a.done_count) c->ib_blocks_issued += (unsigned long long)c->ncap;
    return e;
}

// Blocks of a persistent batched launch: `resident` per compute unit, a
// multiple of 8 (so tile t stays on XCD t % 8), at most one per tile.
static int batch_grid(const lbib_ctx* c, int shape, int resident)
{
    const int tiles = (int)c->L.tiles[shape];
    if (resident <= 0) return tiles;
    const long long want = (long long)resident * c->num_cu / kNumXcd * kNumXcd;
    return (int)std::max<long long>(kNumXcd, std::min<long long>(want, tiles));
}

// The batched grid pass in tile shape `shape`; with a near map, only its far
// part (units whose entry does not carry `stamp`, where no IB force reaches).
template <typename T>
static hipError_t launch_batch_shape(const lbib_ctx* c, const T* src, T* dst,
                                     const long long* fib_now, const int* flags_now,
                                     long long* fib_old, int* flags_old, int shape, int resident,
                                     hipStream_t st, const int* far_map = nullptr, int stamp = 0)
{
    return launch_grid_step_batch<T>(src, dst, fib_now, flags_now, fib_old, flags_old,
                                     inst_table(c), round_table(c, shape), (int)c->L.tiles[shape],
                                     kTileRows[shape], kTileOrder[shape],
                                     batch_grid(c, shape, resident), any_open(c), far_map, stamp,
                                     status_word(c), st);
}

template <typename T>
static hipError_t do_grid(lbib_ctx* c, void* p)
{
    const long long n = *static_cast<const long long*>(p);
    if (c->L.inst.size() == 1) {
        const GridArgs g = grid_args(c->L.inst[0]);
        return launch_grid_step<T>(static_cast<const T*>(pops(c, n)),
                                   static_cast<T*>(pops(c, n + 1)), fib(c, n), flags(c, n),
                                   fib(c, n + 1), flags(c, n + 1), g, c->stream);
    }
    return launch_batch_shape<T>(c, static_cast<const T*>(pops(c, n)),
                                 static_cast<T*>(pops(c, n + 1)), fib(c, n), flags(c, n),
                                 fib(c, n + 1), flags(c, n + 1), c->tile_shape, c->tile_resident,
                                 c->stream);
}

template <typename T>
static lbib_status launch_contact_t(lbib_ctx* c)
{
    ContactArgs<T> a;
    a.nodes = reinterpret_cast<T*>(bufp(c, LBIB_BUF_NODES));
    a.caps = reinterpret_cast<const CapsuleDev*>(bufp(c, LBIB_BUF_CAPS));
    a.bounds = reinterpret_cast<float4*>(bufp(c, LBIB_BUF_CAPS) + c->L.bounds);
    a.node_stride = c->L.max_nodes;
    a.ncap = c->ncap;
    a.max_nv = c->L.max_nv;
    a.cutoff = c->contact_cutoff;
    HIPCHK(c, launch_contact<T>(a, c->stream));
    return LBIB_OK;
}

// Far part of step n.  Untimed single-lattice launches mark e_far(n)
// complete with the kernel itself; everything else records it behind.
template <typename T>
static hipError_t do_far(lbib_ctx* c, void* p)
{
    const long long n = *static_cast<const long long*>(p);
    const bool own_event = c->L.inst.size() == 1 && !c->timing;
    if (c->L.inst.size() > 1)
        return launch_batch_shape<T>(c, static_cast<const T*>(pops(c, n)),
                                     static_cast<T*>(pops(c, n + 1)), fib(c, n), flags(c, n),
                                     fib(c, n + 1), flags(c, n + 1), c->tile_shape,
                                     c->tile_resident, c->s_far, near_map(c, n), step_stamp(n));
    const GridArgs g = grid_args(c->L.inst[0]);
    return launch_grid_far<T>(static_cast<const T*>(pops(c, n)), static_cast<T*>(pops(c, n + 1)),
                              fib(c, n), flags(c, n), fib(c, n + 1), flags(c, n + 1),
                              near_map(c, n), step_stamp(n), status_word(c), g, c->s_far,
                              own_event ? c->e_far[n & 1] : nullptr,
                              c->far_waits_inside ? ib_done_counter(c) : nullptr,
                              c->ib_blocks_issued);
}

template <typename T>
static hipError_t do_near(lbib_ctx* c, void* p)
{
    const long long n = *static_cast<const long long*>(p);
    return launch_grid_near<T>(static_cast<const T*>(pops(c, n)), static_cast<T*>(pops(c, n + 1)),
                               fib(c, n), flags(c, n), fib(c, n + 1), flags(c, n + 1),
                               rect_table(c, n),
                               reinterpret_cast<const CapsuleDev*>(bufp(c, LBIB_BUF_CAPS)),
                               inst_table(c), c->ncap, c->stream);
}

// Overlapped schedule of a lattice, or of every lattice of a batch, with
// capsules (periodic in x, no contact force).  Per step n:
//   main stream: wait far(n-1) -> near(n) -> IB(n+1)
//   far stream:  wait IB(n)    -> far(n)
// IB(n) writes the near regions R_n and stamps them into the near map.
// near(n) computes R_n with the IB force, far(n) the rest with the body force
// only.  far(n) depends only on IB(n), which ran beside far(n-1), so the far
// parts run back to back; near(n) and IB(n+1) run beside far(n).  IB(n+1)
// reads only populations near(n) wrote and force levels far(n) never touches.
// The call ends with the main stream waiting for the last far part.
template <typename T>
static lbib_status step_overlap_t(lbib_ctx* c, int nsteps)
{
    if (!c->s_far) {
        // The events only order the two streams of this device: a device-scope
        // release and acquire suffice (the system-scope fence, there for host
        // visibility, costs a cache write-back at every hand-off).
        const unsigned ev = hipEventDisableTiming | hipEventDisableSystemFence;
        HIPCHK(c, hipStreamCreateWithFlags(&c->s_far, hipStreamNonBlocking));
        HIPCHK(c, hipEventCreateWithFlags(&c->e_ib, ev));
        HIPCHK(c, hipEventCreateWithFlags(&c->e_far[0], ev));
        HIPCHK(c, hipEventCreateWithFlags(&c->e_far[1], ev));
    }
    // the forcing of the first step, unless the last call spread it ahead;
    // the event orders the first far launch after all work on the main stream
    if (!c->a_ready) {
        const long long n = c->steps;
        IBLaunch<T> q{n, n == 0 ? (PH_PRIME | PH_A) : PH_A, true};
        lbib_status s = launch_timed<T>(c, 1, do_ib<T>, &q);
        if (s != LBIB_OK) return s;
    }
    HIPCHK(c, hipEventRecord(c->e_ib, c->stream));
    // Dynamic, one lattice: the last launch also spreads the next step's
    // forcing (phase A writes no node state there), so the next call needs
    // no opening IB launch in front of its first far pass
    const bool ahead = c->mode == LBIB_DYNAMIC && c->L.inst.size() == 1;
    // Far pass n waits for IB(n).  From the second step of a call on, on one
    // large lattice, the far kernel waits inside, on the count of finished IB
    // blocks: that spares the queue-level hand-off between the two streams
    // (about 5 us of every step at 4096^2).  It needs IB(n) to be running by
    // the time far(n) fills the device, which holds there: IB(n) becomes ready
    // a near pass after far(n - 2) ends, far(n) only when far(n - 1) ends.  The
    // first far launch of a call starts beside the call's first IB launch, so
    // it, batches and smaller lattices wait on the queue.
    long long cells = 0;
    for (const Inst& I : c->L.inst) cells += (long long)I.grid.nx * I.grid.ny;
    const bool inside = c->L.inst.size() == 1 && cells >= kFarWaitInsideCells && c->overlap != 2;
    for (int k = 0; k < nsteps; k++) {
        const long long n = c->steps + k;
        long long nn = n;
        c->far_waits_inside = inside && k > 0;
        if (!c->far_waits_inside) HIPCHK(c, hipStreamWaitEvent(c->s_far, c->e_ib, 0));
        lbib_status s = launch_timed<T>(c, 0, do_far<T>, &nn, c->s_far);
        if (s != LBIB_OK) return s;
        if (k > 0) HIPCHK(c, hipStreamWaitEvent(c->stream, c->e_far[(n - 1) & 1], 0));
        if (c->L.inst.size() > 1 || c->timing)  // otherwise the far launch marked it
            HIPCHK(c, hipEventRecord(c->e_far[n & 1], c->s_far));
        s = launch_timed<T>(c, 2, do_near<T>, &nn);
        if (s != LBIB_OK) return s;
        const bool more = k + 1 < nsteps || ahead;
        IBLaunch<T> q{n + 1, more ? (PH_B | PH_A) : PH_B, more};
        s = launch_timed<T>(c, 1, do_ib<T>, &q);
        if (s != LBIB_OK) return s;
        HIPCHK(c, hipEventRecord(c->e_ib, c->stream));
    }
    c->a_ready = ahead;
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->e_far[(c->steps + nsteps - 1) & 1], 0));
    c->steps += nsteps;
    return LBIB_OK;
}

// Single-pass schedule.  With the contact force on, its kernel runs on the
// positions the next force evaluation uses: before every launch with a
// Dynamic node update (x^n of step 7), and, for the Kinematic scheme, between
// the node update and the forcing (x^n of step i), which then take separate
// launches.
// One step of the direct schedule: the IB launch(es) that finish step n - 1
// (phase B, unless pb = 0) and start step n (phase A), then the grid step.
// With the contact force (Eq. 27): Dynamic takes it before each launch that
// holds B; Kinematic splits the launch so that it is added at A.
template <typename T>
static lbib_status step_body(lbib_ctx* c, long long n, int pb, int pa, bool contact, bool dyn)
{
    if (c->ncap > 0 && (pb | pa)) {
        lbib_status s = LBIB_OK;
        if (contact && !dyn) {
            if (pb) {
                IBLaunch<T> qb{n, pb, false};
                s = launch_timed<T>(c, 1, do_ib<T>, &qb);
                if (s != LBIB_OK) return s;
            }
            s = launch_contact_t<T>(c);
            if (s != LBIB_OK) return s;
            IBLaunch<T> qa{n, pa, false};
            s = launch_timed<T>(c, 1, do_ib<T>, &qa);
        } else {
            if (contact && pb) {
                s = launch_contact_t<T>(c);
                if (s != LBIB_OK) return s;
            }
            IBLaunch<T> q{n, pb | pa, false};
            s = launch_timed<T>(c, 1, do_ib<T>, &q);
        }
        if (s != LBIB_OK) return s;
    }
    long long nn = n;
    return launch_timed<T>(c, 0, do_grid<T>, &nn);
}

// Steps per replay of a captured block (even: a replay leaves the buffer
// parity as it found it)
constexpr int kGraphSteps = 16;

static void drop_graphs(lbib_ctx* c)
{
    for (hipGraphExec_t& g : c->gexec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

// Captures steps n0 .. n0 + kGraphSteps - 1 (n0 >= 1, every one a full B + A
// step) into an executable graph.  Every launch argument depends on the step
// only through its parity, so the graph serves every later block that starts
// on a step of the same parity.
template <typename T>
static lbib_status capture_steps(lbib_ctx* c, long long n0, bool contact, bool dyn,
                                 hipGraphExec_t* out)
{
    if (!c->s_cap) HIPCHK(c, hipStreamCreateWithFlags(&c->s_cap, hipStreamNonBlocking));
    HIPCHK(c, hipStreamBeginCapture(c->s_cap, hipStreamCaptureModeThreadLocal));
    const hipStream_t keep = c->stream;
    c->stream = c->s_cap;
    lbib_status s = LBIB_OK;
    for (int i = 0; i < kGraphSteps && s == LBIB_OK; i++)
        s = step_body<T>(c, n0 + i, PH_B, PH_A, contact, dyn);
    c->stream = keep;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->s_cap, &g);
    if (s != LBIB_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return s != LBIB_OK ? s
                            : fail(c, LBIB_EDEVICE,
                                   std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        *out = nullptr;
        return fail(c, LBIB_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    return LBIB_OK;
}

template <typename T>
static lbib_status step_t(lbib_ctx* c, int nsteps)
{
    size_patches<T>(c);
    const bool contact = c->contact_cutoff > 0.0 && c->ncap > 1;
    const bool dyn = c->mode == LBIB_DYNAMIC;
    const bool can_overlap = !contact && !any_open(c) && c->ncap > 0 &&
                             c->ncap <= kMaxOverlapCapsules;
    long long cells = 0;
    for (const Inst& I : c->L.inst) cells += (long long)I.grid.nx * I.grid.ny;
    // automatic: the split pays once the grid step clearly outlasts the IB
    // launch, the near pass and the stream hand-offs (32 capsules, measured:
    // +7 % at 16.8 M cells, +12 % at 8.4 M, +5.5 % at 4.2 M, -10 % at 2.1 M,
    // -19 % at 1.0 M).  A batch of small lattices loses (256 lattices,
    // 8.0 M cells, 388 capsules: -17 %, the IB launch runs 2.4x longer beside
    // the far pass), so a batch splits only when asked.
    const bool want = c->overlap >= 1 || (c->overlap < 0 && c->L.inst.size() == 1 &&
                                          cells >= kOverlapMinCells);
    if (can_overlap && want) return step_overlap_t<T>(c, nsteps);
    // replays of captured blocks for the inner steps; timed runs launch directly
    const bool graphs = c->graph == 1 && !c->timing;
    const int tile = c->tile_shape * 256 + c->tile_resident;
    if (graphs && (c->g_ncap != c->ncap || c->g_mode != c->mode || c->g_patch != c->patch_use ||
                   c->g_contact != c->contact_cutoff || c->g_tile != tile)) {
        drop_graphs(c);
        c->g_ncap = c->ncap;
        c->g_mode = c->mode;
        c->g_patch = c->patch_use;
        c->g_contact = c->contact_cutoff;
        c->g_tile = tile;
    }
    for (int k = 0; k < nsteps;) {
        const long long n = c->steps + k;
        if (graphs && k >= 1 && nsteps - k >= kGraphSteps) {
            hipGraphExec_t& ge = c->gexec[n & 1];
            if (!ge) {
                lbib_status s = capture_steps<T>(c, n, contact, dyn, &ge);
                if (s != LBIB_OK) return s;
            }
            HIPCHK(c, hipGraphLaunch(ge, c->stream));
            c->graph_replays++;
            k += kGraphSteps;
            continue;
        }
        const int pb = k == 0 ? 0 : PH_B;
        const int pa = k == 0 && c->a_ready ? 0 : n == 0 ? (PH_PRIME | PH_A) : PH_A;
        lbib_status s = step_body<T>(c, n, pb, pa, contact, dyn);
        if (s != LBIB_OK) return s;
        k++;
    }
    if (c->ncap > 0) {
        if (contact && dyn) {
            lbib_status s = launch_contact_t<T>(c);
            if (s != LBIB_OK) return s;
        }
        IBLaunch<T> q{c->steps + nsteps, PH_B, false};
        lbib_status s = launch_timed<T>(c, 1, do_ib<T>, &q);
        if (s != LBIB_OK) return s;
    }
    c->a_ready = false;
    c->steps += nsteps;
    return LBIB_OK;
}

extern "C" lbib_status lbib_step(lbib_ctx* c, int32_t nsteps, lbib_mode mode)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    if (nsteps < 0) return fail(c, LBIB_EINVAL, "nsteps must be >= 0");
    if (mode != LBIB_KINEMATIC && mode != LBIB_DYNAMIC) return fail(c, LBIB_EINVAL, "bad mode");
    if (c->mode >= 0 && c->mode != (int)mode)
        return fail(c, LBIB_ESTATE, "the coupling mode is fixed after the first step");
    if (mode == LBIB_KINEMATIC)
        for (int r : c->cap_rigid)
            if (r) return fail(c, LBIB_EINVAL, "rigid particles move with the Dynamic scheme only");
    if (nsteps == 0) return LBIB_OK;
    c->mode = mode;
    return c->rb == 4 ? step_t<float>(c, nsteps) : step_t<double>(c, nsteps);
}

// ------------------------------------------------------------- get / set

template <typename T>
static lbib_status get_t(lbib_ctx* c, int what, int cap, void* dst, size_t bytes, int on_dev)
{
    // field states: cap names the lattice
    const bool field = what == LBIB_F_POPS || what == LBIB_F_POPS_DEV ||
                       what == LBIB_F_MOMENTS || what == LBIB_F_FORCE;
    if (field && (cap < 0 || cap >= (int)c->L.inst.size()))
        return fail(c, LBIB_EINVAL, "bad lattice index");
    const Inst& I = c->L.inst[field ? cap : 0];
    const GridArgs g = grid_args(I);
    const size_t plane = (size_t)I.grid.nx * I.grid.ny;
    const long long* fib_last = fib(c, c->steps + 1) + I.fib_off;
    double* stage = reinterpret_cast<double*>(bufp(c, LBIB_BUF_STAGE));
    const hipMemcpyKind d2h = hipMemcpyDeviceToHost;
    auto finish = [&](const double* src, size_t n) -> lbib_status {
        if (!on_dev) {
            HIPCHK(c, hipMemcpyAsync(dst, src, n * sizeof(double), d2h, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
        return LBIB_OK;
    };
    switch (what) {
    case LBIB_F_POPS:
    case LBIB_F_POPS_DEV: {
        if (bytes < 9 * plane * sizeof(double)) return fail(c, LBIB_EINVAL, "dst too small");
        for (int i = 0; i < 9; i++) {
            double* o = on_dev ? static_cast<double*>(dst) + i * plane : stage;
            HIPCHK(c, launch_get_pop_plane<T>(pops_of<const T>(c, c->steps, I), o, i,
                                              what == LBIB_F_POPS, g, c->stream));
            if (!on_dev)
                HIPCHK(c, hipMemcpyAsync(static_cast<double*>(dst) + i * plane, stage,
                                         plane * sizeof(double), d2h, c->stream));
        }
        if (!on_dev) HIPCHK(c, hipStreamSynchronize(c->stream));
        return LBIB_OK;
    }
    case LBIB_F_MOMENTS: {
        if (bytes < 3 * plane * sizeof(double)) return fail(c, LBIB_EINVAL, "dst too small");
        double* o = on_dev ? static_cast<double*>(dst) : stage;
        HIPCHK(c, launch_get_moments<T>(pops_of<const T>(c, c->steps, I), fib_last, o, g,
                                        c->stream));
        return finish(o, 3 * plane);
    }
    case LBIB_F_FORCE: {
        if (bytes < 2 * plane * sizeof(double)) return fail(c, LBIB_EINVAL, "dst too small");
        double* o = on_dev ? static_cast<double*>(dst) : stage;
        HIPCHK(c, launch_get_force(fib_last, o, g, c->stream));
        return finish(o, 2 * plane);
    }
    case LBIB_C_NODES:
    case LBIB_C_PREV:
    case LBIB_C_VEL:
    case LBIB_C_FORCE:
    case LBIB_C_STATE: {
        if (cap < 0 || cap >= c->ncap) return fail(c, LBIB_EINVAL, "bad capsule id");
        const int nv = c->cap_nv[cap];
        const size_t n = (what == LBIB_C_STATE ? 6 : 2) * (size_t)nv;
        if (bytes < n * sizeof(double)) return fail(c, LBIB_EINVAL, "dst too small");
        double* o = on_dev ? static_cast<double*>(dst) : stage;
        HIPCHK(c, launch_get_nodes<T>(reinterpret_cast<const T*>(bufp(c, LBIB_BUF_NODES)),
                                      reinterpret_cast<const CapsuleDev*>(bufp(c, LBIB_BUF_CAPS)),
                                      cap, nv, c->L.max_nodes, what, o, c->stream));
        return finish(o, n);
    }
    case LBIB_C_DIAG: {
        if (cap < 0 || cap >= c->ncap) return fail(c, LBIB_EINVAL, "bad capsule id");
        if (bytes < kDiagStride * sizeof(double)) return fail(c, LBIB_EINVAL, "dst too small");
        size_patches<T>(c);
        IBArgs<T> a = ib_args<T>(c, c->steps, PH_DIAG);
        HIPCHK(c, launch_ib<T>(a, c->ncap, c->lds_use, c->stream, ib_wide(c, a)));
        const double* src = reinterpret_cast<const double*>(bufp(c, LBIB_BUF_DIAG)) +
                            (size_t)cap * kDiagStride;
        if (on_dev)
            HIPCHK(c, hipMemcpyAsync(dst, src, kDiagStride * sizeof(double),
                                     hipMemcpyDeviceToDevice, c->stream));
        return finish(src, kDiagStride);
    }
    case LBIB_C_RIGID: {
        if (cap < 0 || cap >= c->ncap) return fail(c, LBIB_EINVAL, "bad capsule id");
        if (on_dev) return fail(c, LBIB_EINVAL, "LBIB_C_RIGID is copied to host memory only");
        if (bytes < 10 * sizeof(double)) return fail(c, LBIB_EINVAL, "dst too small");
        CapsuleDev cd;
        HIPCHK(c, hipMemcpyAsync(&cd, bufp(c, LBIB_BUF_CAPS) + (size_t)cap * sizeof(CapsuleDev),
                                 sizeof(cd), d2h, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        double* o = static_cast<double*>(dst);
        o[0] = cd.rX;
        o[1] = cd.rY;
        o[2] = cd.rth;
        o[3] = cd.ru[0];
        o[4] = cd.ru[1];
        o[5] = cd.rw;
        o[6] = cd.rF[0];
        o[7] = cd.rF[1];
        o[8] = cd.rM;
        o[9] = cd.rigid;
        return LBIB_OK;
    }
    case LBIB_STATUS: {
        if (bytes < sizeof(int)) return fail(c, LBIB_EINVAL, "dst too small");
        const hipMemcpyKind k = on_dev ? hipMemcpyDeviceToDevice : d2h;
        HIPCHK(c, hipMemcpyAsync(dst, status_word(c), sizeof(int), k, c->stream));
        if (!on_dev) HIPCHK(c, hipStreamSynchronize(c->stream));
        return LBIB_OK;
    }
    default: return fail(c, LBIB_EINVAL, "unknown state id");
    }
}

extern "C" lbib_status lbib_get_state(lbib_ctx* c, int32_t what, int32_t cap, void* dst,
                                      size_t bytes, int32_t on_dev)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    if (!dst) return fail(c, LBIB_EINVAL, "dst is NULL");
    return c->rb == 4 ? get_t<float>(c, what, cap, dst, bytes, on_dev)
                      : get_t<double>(c, what, cap, dst, bytes, on_dev);
}

template <typename T>
static lbib_status set_t(lbib_ctx* c, int what, int cap, const void* src, size_t bytes, int on_dev)
{
    double* stage = reinterpret_cast<double*>(bufp(c, LBIB_BUF_STAGE));
    if (what == LBIB_F_POPS || what == LBIB_C_STATE) {
        lbib_status d = drop_pending_forcing(c);
        if (d != LBIB_OK) return d;
    }
    if (what == LBIB_F_POPS) {
        if (cap < 0 || cap >= (int)c->L.inst.size())
            return fail(c, LBIB_EINVAL, "bad lattice index");
        const Inst& I = c->L.inst[cap];
        const GridArgs g = grid_args(I);
        const size_t plane = (size_t)I.grid.nx * I.grid.ny;
        if (bytes < 9 * plane * sizeof(double)) return fail(c, LBIB_EINVAL, "src too small");
        for (int i = 0; i < 9; i++) {
            const double* in = static_cast<const double*>(src) + i * plane;
            if (!on_dev) {
                HIPCHK(c, hipMemcpyAsync(stage, in, plane * sizeof(double), hipMemcpyHostToDevice,
                                         c->stream));
                in = stage;
            }
            HIPCHK(c, launch_set_pop_plane<T>(pops_of<T>(c, c->steps, I), in, i, g, c->stream));
        }
        if (!on_dev) HIPCHK(c, hipStreamSynchronize(c->stream));
        return LBIB_OK;
    }
    if (what == LBIB_C_STATE) {
        if (cap < 0 || cap >= c->ncap) return fail(c, LBIB_EINVAL, "bad capsule id");
        const int nv = c->cap_nv[cap];
        const size_t n = 6 * (size_t)nv;
        if (bytes < n * sizeof(double)) return fail(c, LBIB_EINVAL, "src too small");
        const double* in = static_cast<const double*>(src);
        if (!on_dev) {
            for (size_t j = 0; j < n; j++)
                if (!std::isfinite(in[j])) return fail(c, LBIB_EINVAL, "non-finite node state");
            HIPCHK(c, hipMemcpyAsync(stage, in, n * sizeof(double), hipMemcpyHostToDevice,
                                     c->stream));
            in = stage;
        }
        HIPCHK(c, launch_set_nodes<T>(reinterpret_cast<T*>(bufp(c, LBIB_BUF_NODES)),
                                      reinterpret_cast<CapsuleDev*>(bufp(c, LBIB_BUF_CAPS)), cap,
                                      nv, c->L.max_nodes, in, c->stream));
        if (!on_dev) HIPCHK(c, hipStreamSynchronize(c->stream));
        return LBIB_OK;
    }
    return fail(c, LBIB_EINVAL, "state id cannot be set");
}

extern "C" lbib_status lbib_set_state(lbib_ctx* c, int32_t what, int32_t cap, const void* src,
                                      size_t bytes, int32_t on_dev)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    if (!src) return fail(c, LBIB_EINVAL, "src is NULL");
    return c->rb == 4 ? set_t<float>(c, what, cap, src, bytes, on_dev)
                      : set_t<double>(c, what, cap, src, bytes, on_dev);
}

// ----------------------------------------------------------------- adjoint

// Workspace of lbib_adjoint.  Segments of K = `every` steps (the last one
// may be shorter); segment s covers time levels sK .. min(sK + K, N).
//   grid tape   K + 1 slots, slot r = level sK + r of the current segment:
//               populations P, IB force F - g and its segment flags
//   node tape   N + 1 slots: node state, the force each node spread, and the
//               reference points of every level
//   checkpoints one grid slot per segment when there are several (level sK)
// then the reverse-sweep arrays.  A recomputed segment needs no node state:
// its force levels come back from the taped node forces (k_spread_tape).
struct AdjLayout {
    size_t pops = 0, fib = 0, flags = 0, gslot = 0;
    size_t nodes = 0, ref = 0, nslot = 0;
    size_t ntape = 0, ckpt = 0;
    size_t lam[2] = {0, 0}, lfm = 0, lft = 0, lfm_flags = 0, zero_flags = 0;
    size_t gacc = 0, lamx = 0, lamd = 0, ksbar = 0, out = 0, total = 0;
    int every = 0, nseg = 0, blocks = 0;
};

static bool adj_layout(const lbib_ctx* c, int nsteps, int every, AdjLayout& A)
{
    if (!c || c->L.inst.size() != 1 || nsteps < 1 || every < 0) return false;
    const Inst& I = c->L.inst[0];
    const size_t cells = (size_t)I.nxp * I.grid.ny;
    const size_t nseg = I.nseg;
    A.every = (every == 0 || every >= nsteps) ? nsteps : every;
    A.nseg = (nsteps + A.every - 1) / A.every;
    A.pops = round256(9 * cells * c->rb);
    A.fib = round256(2 * cells * sizeof(long long));
    A.flags = round256((size_t)I.grid.ny * nseg * sizeof(int));
    A.gslot = A.pops + A.fib + A.flags;
    A.nodes = round256((size_t)kTapeFields * c->L.max_nodes * c->rb);
    A.ref = round256((size_t)2 * c->L.max_caps * sizeof(double));
    A.nslot = A.nodes + A.ref;
    size_t o = A.gslot * (size_t)(A.every + 1);
    A.ntape = o;
    o += A.nslot * (size_t)(nsteps + 1);
    A.ckpt = o;
    if (A.nseg > 1) o += A.gslot * (size_t)A.nseg;
    A.lam[0] = o;
    o += A.pops;
    A.lam[1] = o;
    o += A.pops;
    A.lfm = o;
    o += round256(2 * cells * c->rb);
    A.lft = o;
    o += round256(2 * cells * c->rb);
    A.lfm_flags = o;
    o += A.flags;
    A.zero_flags = o;
    o += A.flags;
    A.blocks = grid_blocks(I.grid.ny, I.nseg);
    A.gacc = o;
    o += round256((size_t)A.blocks * sizeof(double));
    A.lamx = o;
    o += round256((size_t)2 * c->L.max_nodes * sizeof(double));
    A.lamd = o;
    o += round256((size_t)2 * c->L.max_nodes * sizeof(double));
    A.ksbar = o;
    o += round256((size_t)c->L.max_nodes * sizeof(double));
    A.out = o;
    o += 256;
    A.total = o;
    return true;
}

extern "C" size_t lbib_adjoint_bytes(const lbib_ctx* c, int32_t nsteps, int32_t checkpoint_every)
{
    AdjLayout A;
    return adj_layout(c, nsteps, checkpoint_every, A) ? A.total : 0;
}

template <typename T>
static lbib_status adjoint_t(lbib_ctx* c, int N, int mode, int objective, int capid, char* ws,
                             const AdjLayout& A, double* out_J, double* out_g, double* out_ks)
{
    const Inst& I = c->L.inst[0];
    const GridArgs g = grid_args(I);
    const hipStream_t st = c->stream;
    const hipMemcpyKind d2d = hipMemcpyDeviceToDevice;
    const int K = A.every;
    // grid tape, by slot; node tape, by level; checkpoints, by segment
    auto gslot = [&](int r) { return ws + A.gslot * (size_t)r; };
    auto gP = [&](int r) { return reinterpret_cast<T*>(gslot(r)); };
    auto gF = [&](int r) { return reinterpret_cast<long long*>(gslot(r) + A.pops); };
    auto gFl = [&](int r) { return reinterpret_cast<int*>(gslot(r) + A.pops + A.fib); };
    auto sN = [&](int n) { return reinterpret_cast<T*>(ws + A.ntape + A.nslot * (size_t)n); };
    auto sR = [&](int n) {
        return reinterpret_cast<double*>(ws + A.ntape + A.nslot * (size_t)n + A.nodes);
    };
    auto ck = [&](int seg) { return ws + A.ckpt + A.gslot * (size_t)seg; };
    T* lam[2] = {reinterpret_cast<T*>(ws + A.lam[0]), reinterpret_cast<T*>(ws + A.lam[1])};
    T* lfm = reinterpret_cast<T*>(ws + A.lfm);
    T* lft = reinterpret_cast<T*>(ws + A.lft);
    int* lfm_flags = reinterpret_cast<int*>(ws + A.lfm_flags);
    int* zero_flags = reinterpret_cast<int*>(ws + A.zero_flags);
    double* gacc = reinterpret_cast<double*>(ws + A.gacc);
    double* lamx = reinterpret_cast<double*>(ws + A.lamx);
    double* lamd = reinterpret_cast<double*>(ws + A.lamd);
    double* ksbar = reinterpret_cast<double*>(ws + A.ksbar);
    double* out = reinterpret_cast<double*>(ws + A.out);
    const size_t pop_bytes = 9 * (size_t)I.nxp * I.grid.ny * sizeof(T);

    // LDS of the IB reverse kernel: FP64 node arrays, the rest holds the patch
    int dev = 0;
    hipDeviceProp_t prop;
    HIPCHK(c, hipGetDevice(&dev));
    HIPCHK(c, hipGetDeviceProperties(&prop, dev));
    const size_t budget = (prop.sharedMemPerBlock > 0 ? prop.sharedMemPerBlock : 65536) - 1024;
    const size_t node_part = ib_adj_lds_bytes<T>(0, c->L.max_nv) + 16;
    if (node_part + (size_t)1024 * 6 * sizeof(T) > budget)
        return fail(c, LBIB_ECAPACITY, "capsules too large for the adjoint on-chip memory");
    const int adj_patch = (int)std::min<size_t>((budget - node_part) / (6 * sizeof(T)),
                                                (size_t)c->patch_cap);
    const size_t adj_lds = ib_adj_lds_bytes<T>(adj_patch, c->L.max_nv);
    HIPCHK(c, ib_adj_set_lds_limit<T>(adj_lds));

    // forward steps c0 .. e0-1 of one segment; the grid slot 0 holds level c0
    // and the force accumulators of slots 1 .. e0-c0 are zero.  The first run
    // takes the IB launches and tapes the nodes; a recomputed segment spreads
    // the taped node forces instead (the same force levels, no node state)
    auto run_segment = [&](int c0, int e0, bool again) -> lbib_status {
        for (int n = c0; n < e0; n++) {
            const int r = n - c0;
            if (again) {
                SpreadTapeArgs<T> sa;
                sa.fib = gF(r + 1);
                sa.flags = gFl(r + 1);
                sa.tape = sN(n);
                sa.ref = sR(n);
                sa.caps = reinterpret_cast<const CapsuleDev*>(bufp(c, LBIB_BUF_CAPS));
                sa.status = status_word(c);
                sa.node_stride = c->L.max_nodes;
                HIPCHK(c, launch_spread_tape<T>(sa, c->ncap, st));
            } else {
                IBArgs<T> a = ib_args<T>(c, n, n == 0 ? (PH_PRIME | PH_A) : (PH_B | PH_A));
                a.pops = gP(r);
                a.fib_prev = gF(r);
                a.fib_next = gF(r + 1);
                a.flags_next = gFl(r + 1);
                a.tape_nodes = sN(n);
                a.tape_ref = sR(n);
                HIPCHK(c, launch_ib<T>(a, c->ncap, c->lds_use, st, ib_wide(c, a)));
            }
            HIPCHK(c, launch_grid_step<T>(gP(r), gP(r + 1), gF(r + 1), gFl(r + 1), gF(r + 1),
                                          zero_flags, g, st));
        }
        return LBIB_OK;
    };
    // zero the force accumulators and flags of grid slots 1 .. m with one fill
    // over the whole slot range (their populations are written before they are
    // read), in place of one short fill launch per slot
    auto clear_slots = [&](int m) -> hipError_t {
        return m > 0 ? hipMemsetAsync(gslot(1), 0, A.gslot * (size_t)m, st) : hipSuccess;
    };
    auto seg_lo = [&](int s) { return s * K; };
    auto seg_hi = [&](int s) { return std::min(s * K + K, N); };

    size_patches<T>(c);
    HIPCHK(c, hipMemsetAsync(ws, 0, A.total, st));
    HIPCHK(c, hipMemcpyAsync(gP(0), pops(c, 0), pop_bytes, d2d, st));
    c->mode = mode;

    // ---- forward run, taped segment by segment
    for (int s = 0; s < A.nseg; s++) {
        const int c0 = seg_lo(s), e0 = seg_hi(s);
        if (s > 0) {
            HIPCHK(c, hipMemcpyAsync(gslot(0), gslot(K), A.gslot, d2d, st));
            HIPCHK(c, clear_slots(e0 - c0));
        }
        if (A.nseg > 1) HIPCHK(c, hipMemcpyAsync(ck(s), gslot(0), A.gslot, d2d, st));
        lbib_status e = run_segment(c0, e0, false);
        if (e != LBIB_OK) return e;
    }
    const int cl = seg_lo(A.nseg - 1), rN = N - cl;
    {
        IBArgs<T> a = ib_args<T>(c, N, PH_B);
        a.pops = gP(rN);
        a.fib_prev = gF(rN);
        a.fib_next = gF(rN);
        a.flags_next = gFl(rN);
        a.tape_nodes = sN(N);
        a.tape_ref = sR(N);
        HIPCHK(c, launch_ib<T>(a, c->ncap, c->lds_use, st, ib_wide(c, a)));
    }
    // the context now stands at step N
    HIPCHK(c, hipMemcpyAsync(pops(c, N), gP(rN), pop_bytes, d2d, st));
    HIPCHK(c, hipMemcpyAsync(fib(c, N + 1), gF(rN), 2 * (size_t)I.nxp * I.grid.ny * sizeof(long long),
                             d2d, st));
    HIPCHK(c, hipMemcpyAsync(flags(c, N + 1), gFl(rN), (size_t)I.grid.ny * I.nseg * sizeof(int),
                             d2d, st));
    c->steps = N;
    c->a_ready = false;
    int flags_fwd = 0;
    HIPCHK(c, hipMemcpyAsync(&flags_fwd, status_word(c), sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (flags_fwd)
        return fail(c, LBIB_ENUMERIC, "device status flags set in the forward run: " +
                                          std::to_string(flags_fwd));

    // ---- reverse sweep
    const CapsuleDev* caps = reinterpret_cast<const CapsuleDev*>(bufp(c, LBIB_BUF_CAPS));
    HIPCHK(c, launch_adj_seed<T>(sN(N), sR(N), caps, capid, c->L.max_nodes, objective, lamx, out,
                                 st));
    bool bend = false;
    for (double kb : c->cap_kb) bend = bend || kb != 0.0;
    // slot r of the grid tape holds level n (the segment starts at n - r)
    auto ib_adj = [&](int n, int r, int doA, int doB, int prime) -> hipError_t {
        IBAdjArgs<T> b;
        b.pops = gP(r);
        b.fib_prev = gF(r);
        b.nodes_n = sN(n);
        b.ref_n = sR(n);
        b.nodes_p = doB ? sN(n - 1) : sN(n);
        b.ref_p = doB ? sR(n - 1) : sR(n);
        b.consts = reinterpret_cast<const T*>(bufp(c, LBIB_BUF_NODES));
        b.caps = caps;
        b.lft = lft;
        b.lam_p = lam[n & 1];
        b.lfm = lfm;
        b.lfm_flags = lfm_flags;
        b.lamx = lamx;
        b.lamd = lamd;
        b.ksbar = ksbar;
        b.status = status_word(c);
        b.stride = c->L.max_nodes;
        b.doA = doA;
        b.doB = doB;
        b.prime = prime;
        b.dynamic = mode == LBIB_DYNAMIC;
        b.bend = bend;
        b.patch_cap = adj_patch;
        b.max_nv = c->L.max_nv;
        return launch_ib_adj<T>(b, c->ncap, adj_lds, st);
    };
    auto grid_adj_args = [&](int n, int r) {
        GridAdjArgs<T> ga;
        ga.pops = gP(r);
        ga.fib = gF(r + 1);
        ga.flags = gFl(r + 1);
        ga.lam_in = lam[(n + 1) & 1];
        ga.lam_out = lam[n & 1];
        ga.lfm = lfm;
        ga.lfm_flags = lfm_flags;
        ga.lft = lft;
        ga.gacc = gacc;
        return ga;
    };
    HIPCHK(c, ib_adj(N, rN, 0, 1, 0));
    for (int s = A.nseg - 1; s >= 0; s--) {
        const int c0 = seg_lo(s), e0 = seg_hi(s);
        if (s < A.nseg - 1) {
            HIPCHK(c, hipMemcpyAsync(gslot(0), ck(s), A.gslot, d2d, st));
            HIPCHK(c, clear_slots(e0 - c0));
            lbib_status e = run_segment(c0, e0, true);
            if (e != LBIB_OK) return e;
        }
        for (int n = e0 - 1; n >= c0; n--) {
            HIPCHK(c, launch_grid_adj<T>(grid_adj_args(n, n - c0), g, st));
            HIPCHK(c, ib_adj(n, n - c0, 1, n >= 1, n == 0));
        }
    }
    {
        GridAdjArgs<T> ga = grid_adj_args(0, 0);
        ga.lam_in = lam[0];
        HIPCHK(c, launch_init_adj<T>(ga, g, I.walls.init_profile, I.nu, st));
    }
    HIPCHK(c, launch_reduce_sum(gacc, A.blocks, out, st));
    double host_out[2] = {0, 0};
    HIPCHK(c, hipMemcpyAsync(host_out, out, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(out_ks, ksbar, (size_t)c->nodes_used * sizeof(double),
                             hipMemcpyDeviceToHost, st));
    int flags_rev = 0;
    HIPCHK(c, hipMemcpyAsync(&flags_rev, status_word(c), sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (flags_rev)
        return fail(c, LBIB_ENUMERIC, "device status flags set in the reverse sweep: " +
                                          std::to_string(flags_rev));
    *out_g = host_out[0];
    *out_J = host_out[1];
    return LBIB_OK;
}

// Argument and state checks shared by lbib_adjoint and lbib_adjoint_noalloc;
// fills the workspace layout.
static lbib_status adjoint_validate(lbib_ctx* c, int32_t nsteps, int32_t checkpoint_every,
                                    lbib_mode mode, int32_t objective, int32_t capsule,
                                    const double* out_J, const double* out_dJ_dg,
                                    const double* out_dJ_dks, int32_t n_ks, AdjLayout& A)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    if (!out_J || !out_dJ_dg || !out_dJ_dks) return fail(c, LBIB_EINVAL, "NULL argument");
    if (c->L.inst.size() != 1) return fail(c, LBIB_EINVAL, "the adjoint needs a single lattice");
    if (nsteps < 1) return fail(c, LBIB_EINVAL, "nsteps must be >= 1");
    if (checkpoint_every < 0) return fail(c, LBIB_EINVAL, "checkpoint_every must be >= 0");
    if (mode != LBIB_KINEMATIC && mode != LBIB_DYNAMIC) return fail(c, LBIB_EINVAL, "bad mode");
    if (objective != LBIB_OBJ_TAYLOR && objective != LBIB_OBJ_CENTROID_Y)
        return fail(c, LBIB_EINVAL, "unknown objective");
    if (capsule < 0 || capsule >= c->ncap) return fail(c, LBIB_EINVAL, "bad capsule id");
    if (c->steps != 0) return fail(c, LBIB_ESTATE, "the adjoint run starts from step 0");
    if (c->mode >= 0 && c->mode != (int)mode)
        return fail(c, LBIB_ESTATE, "the coupling mode is fixed after the first step");
    if (c->contact_cutoff > 0.0 && c->ncap > 1)
        return fail(c, LBIB_EINVAL, "the adjoint does not differentiate the contact force");
    if (!c->L.inst[0].walls.periodic_x)
        return fail(c, LBIB_EINVAL, "the adjoint needs a periodic channel (periodic_x = 1)");
    for (int r : c->cap_rigid)
        if (r) return fail(c, LBIB_EINVAL, "the adjoint does not differentiate rigid particles");
    if (n_ks < c->nodes_used) return fail(c, LBIB_EINVAL, "out_dJ_dks shorter than the node count");
    if (!adj_layout(c, nsteps, checkpoint_every, A))
        return fail(c, LBIB_EINVAL, "invalid adjoint layout");
    return LBIB_OK;
}

extern "C" lbib_status lbib_adjoint(lbib_ctx* c, int32_t nsteps, int32_t checkpoint_every,
                                    lbib_mode mode, int32_t objective, int32_t capsule,
                                    void* workspace, size_t workspace_bytes, double* out_J,
                                    double* out_dJ_dg, double* out_dJ_dks, int32_t n_ks)
{
    AdjLayout A;
    lbib_status v = adjoint_validate(c, nsteps, checkpoint_every, mode, objective, capsule, out_J,
                                     out_dJ_dg, out_dJ_dks, n_ks, A);
    if (v != LBIB_OK) return v;
    if (!workspace) return fail(c, LBIB_EINVAL, "NULL argument");
    if (workspace_bytes < A.total) return fail(c, LBIB_EINVAL, "workspace too small");
    char* ws = static_cast<char*>(workspace);
    return c->rb == 4 ? adjoint_t<float>(c, nsteps, mode, objective, capsule, ws, A, out_J,
                                         out_dJ_dg, out_dJ_dks)
                      : adjoint_t<double>(c, nsteps, mode, objective, capsule, ws, A, out_J,
                                          out_dJ_dg, out_dJ_dks);
}

extern "C" lbib_status lbib_adjoint_noalloc(lbib_ctx* c, int32_t nsteps, int32_t checkpoint_every,
                                            lbib_mode mode, int32_t objective, int32_t capsule,
                                            double* out_J, double* out_dJ_dg, double* out_dJ_dks,
                                            int32_t n_ks)
{
    AdjLayout A;
    lbib_status v = adjoint_validate(c, nsteps, checkpoint_every, mode, objective, capsule, out_J,
                                     out_dJ_dg, out_dJ_dks, n_ks, A);
    if (v != LBIB_OK) return v;
    if (A.total > (size_t)LBIB_ADJOINT_SCRATCH_BYTES)
        return fail(c, LBIB_ECAPACITY,
                    "the gradient needs " + std::to_string(A.total) +
                        " workspace bytes; the static scratch holds " +
                        std::to_string((size_t)LBIB_ADJOINT_SCRATCH_BYTES) +
                        " (use lbib_adjoint with a caller-owned workspace, or a checkpoint interval)");
    int cur = 0;
    HIPCHK(c, hipGetDevice(&cur));
    if (cur != c->device)
        return fail(c, LBIB_EDEVICE, "call lbib_adjoint_noalloc with the context's device current");
    void* p = nullptr;
    hipError_t e = resolve_scratch(c->device, &p);
    if (e != hipSuccess)
        return fail(c, LBIB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    // adjoint_t clears the A.total bytes it uses before the forward run
    char* ws = static_cast<char*>(p);
    return c->rb == 4 ? adjoint_t<float>(c, nsteps, mode, objective, capsule, ws, A, out_J,
                                         out_dJ_dg, out_dJ_dks)
                      : adjoint_t<double>(c, nsteps, mode, objective, capsule, ws, A, out_J,
                                          out_dJ_dg, out_dJ_dks);
}

// ---------------------------------------------------------- check, timing

extern "C" lbib_status lbib_check(lbib_ctx* c, int32_t* flags_out)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    int st = 0;
    HIPCHK(c, hipMemcpyAsync(&st, status_word(c), sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (flags_out) *flags_out = st;
    if (st) return fail(c, LBIB_ENUMERIC, "device status flags set: " + std::to_string(st));
    return LBIB_OK;
}

extern "C" lbib_status lbib_set_contact(lbib_ctx* c, double cutoff)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    if (!std::isfinite(cutoff) || cutoff < 0.0 || cutoff > 16.0)
        return fail(c, LBIB_EINVAL, "cutoff must be in [0, 16]");
    if (cutoff > 0.0) {
        hipError_t e = c->rb == 4 ? contact_set_lds_limit<float>(c->L.max_nv)
                                  : contact_set_lds_limit<double>(c->L.max_nv);
        if (e != hipSuccess)
            return fail(c, LBIB_EDEVICE, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    }
    c->contact_cutoff = cutoff;
    return LBIB_OK;
}

extern "C" lbib_status lbib_set_overlap(lbib_ctx* c, int32_t enable)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    if (enable < -1 || enable > 2) return fail(c, LBIB_EINVAL, "enable must be -1, 0, 1 or 2");
    c->overlap = enable;
    return LBIB_OK;
}

extern "C" lbib_status lbib_set_limits(lbib_ctx* c, double max_edge, double max_area_change)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    if (!(max_edge >= 0.0 && max_edge < 1e30) || !(max_area_change >= 0.0 && max_area_change < 1e30))
        return fail(c, LBIB_EINVAL, "limits must be finite and >= 0");
    c->max_edge = (float)max_edge;
    c->max_dA = (float)max_area_change;
    return LBIB_OK;
}

extern "C" lbib_status lbib_set_graph(lbib_ctx* c, int32_t enable)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    if (enable < -1 || enable > 1) return fail(c, LBIB_EINVAL, "enable must be -1, 0 or 1");
    c->graph = enable;
    return LBIB_OK;
}

extern "C" int64_t lbib_graph_replays(const lbib_ctx* c) { return c ? c->graph_replays : -1; }

extern "C" lbib_status lbib_set_tile(lbib_ctx* c, int32_t rows, int32_t linear, int32_t resident)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    if (linear < 0 || linear > 2) return fail(c, LBIB_EINVAL, "linear (tile order) must be 0, 1 or 2");
    int shape = -1;
    for (int k = 0; k < kTileShapes; k++)
        if (kTileRows[k] == rows && kTileOrder[k] == linear) shape = k;
    if (shape < 0) return fail(c, LBIB_EINVAL, "rows must be 1, 2 or 4");
    if (resident < 0 || resident > 64) return fail(c, LBIB_EINVAL, "resident must be in [0, 64]");
    c->tile_shape = shape;
    c->tile_resident = resident;
    return LBIB_OK;
}

// Times every tile-shape candidate of the batched grid pass on the context's
// own lattices and keeps the fastest.  The pass runs on the current state
// with the force level of the coming step as both its force input and the
// level it clears: between calls that level is zero (the last grid pass
// cleared it), so the trial passes read no force, clear nothing, and write
// only the other population buffer, which the next step rewrites in full.
template <typename T>
static lbib_status autotune_t(lbib_ctx* c, int launches, double* us)
{
    const long long n = c->steps;
    const T* src = static_cast<const T*>(pops(c, n));
    T* dst = static_cast<T*>(pops(c, n + 1));
    long long* f = fib(c, n);
    int* fl = flags(c, n);
    hipEvent_t e0 = nullptr, e1 = nullptr;  // timing only, as take_event's
    HIPCHK(c, hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    if (hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, LBIB_EDEVICE, "hipEventCreate failed");
    }
    lbib_status st = LBIB_OK;
    double best = 1e300;
    int best_s = 0, best_r = 0;
    for (int s = 0; s < kTileShapes && st == LBIB_OK; s++)
        for (int r = 0; r < 4 && st == LBIB_OK; r++) {
            hipError_t e = launch_batch_shape<T>(c, src, dst, f, fl, f, fl, s, kTileResident[r],
                                                 c->stream);
            if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
            for (int i = 0; i < launches && e == hipSuccess; i++)
                e = launch_batch_shape<T>(c, src, dst, f, fl, f, fl, s, kTileResident[r],
                                          c->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                st = fail(c, LBIB_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
                break;
            }
            const double t = 1e3 * ms / launches;
            us[s * 4 + r] = t;
            if (t < best) {
                best = t;
                best_s = s;
                best_r = r;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != LBIB_OK) return st;
    c->tile_shape = best_s;
    c->tile_resident = kTileResident[best_r];
    return LBIB_OK;
}

extern "C" lbib_status lbib_autotune(lbib_ctx* c, int32_t launches, int32_t* out_rows,
                                     int32_t* out_linear, int32_t* out_resident, double* out_us,
                                     int32_t n_us)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    if (launches < 1 || launches > 1000) return fail(c, LBIB_EINVAL, "launches must be in [1, 1000]");
    if (c->L.inst.size() < 2) return fail(c, LBIB_EINVAL, "tile shapes apply to batch contexts");
    double us[kTileShapes * 4];
    const lbib_status st = c->rb == 4 ? autotune_t<float>(c, launches, us)
                                      : autotune_t<double>(c, launches, us);
    if (st != LBIB_OK) return st;
    if (out_rows) *out_rows = kTileRows[c->tile_shape];
    if (out_linear) *out_linear = kTileOrder[c->tile_shape];
    if (out_resident) *out_resident = c->tile_resident;
    for (int i = 0; out_us && i < n_us && i < kTileShapes * 4; i++) out_us[i] = us[i];
    return LBIB_OK;
}

extern "C" lbib_status lbib_set_timing(lbib_ctx* c, int32_t enable)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    c->timing = enable != 0;
    return LBIB_OK;
}

extern "C" lbib_status lbib_get_timing(lbib_ctx* c, double* out)
{
    if (!c) return fail(nullptr, LBIB_EINVAL, "ctx is NULL");
    if (!out) return fail(c, LBIB_EINVAL, "out is NULL");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double t[3] = {0, 0, 0}, cnt[3] = {0, 0, 0};
    for (const TimedLaunch& tl : c->timed) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, tl.start, tl.stop));
        t[tl.kind] += ms;
        cnt[tl.kind] += 1;
        c->pool.push_back(tl.start);
        c->pool.push_back(tl.stop);
    }
    c->timed.clear();
    out[0] = t[0];
    out[1] = cnt[0];
    out[2] = t[1];
    out[3] = cnt[1];
    out[4] = t[2];
    out[5] = cnt[2];
    return LBIB_OK;
}

extern "C" int64_t lbib_steps_done(const lbib_ctx* c) { return c ? c->steps : -1; }

extern "C" const char* lbib_last_error(const lbib_ctx* c)
{
    return c ? c->err.c_str() : t_err.c_str();
}

extern "C" void lbib_destroy(lbib_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (const TimedLaunch& tl : c->timed) {
        (void)hipEventDestroy(tl.start);
        (void)hipEventDestroy(tl.stop);
    }
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    drop_graphs(c);
    if (c->s_cap) (void)hipStreamDestroy(c->s_cap);
    if (c->s_far) {
        (void)hipStreamSynchronize(c->s_far);
        (void)hipStreamDestroy(c->s_far);
        (void)hipEventDestroy(c->e_ib);
        (void)hipEventDestroy(c->e_far[0]);
        (void)hipEventDestroy(c->e_far[1]);
    }
    delete c;
}
