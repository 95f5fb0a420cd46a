// Host runtime of liblb.so: the C ABI declared in include/lb.h.
//
// Responsibilities: validate configurations, lay out the caller's workspace,
// write the initial state, choose tile shapes (by timing candidates on the
// caller's stream), build HIP graphs of step chunks, dispatch the templated
// gfx950 kernels of lb_kernels.hpp and map HIP failures to LB_EHIP.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "lb.h"
#include "lb_kernels.hpp"
#include "lb_tune_cache.hpp"


using namespace lbk;

namespace lbrt {

thread_local std::string g_err;

int32_t fail(int32_t code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace lbrt

using lbrt::fail;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_bytes(int storage)
{
    switch (storage) {
        case LB_F64: return 8;
        case LB_F32: return 4;
        default: return 2;
    }
}

int64_t pitch_of(int nx) { return (int64_t)align_up((size_t)nx, 64); }

bool site_shift(int storage) { return storage == LB_F16S || storage == LB_BF16S; }

// Bytes of one row block: 2 x 9 population segments of pitch elements, plus
// (16-bit modes) the two FP32 site-density segments.
int64_t row_bytes_of(int storage, int64_t pitch)
{
    return (int64_t)2 * NQ * pitch * (int64_t)elem_bytes(storage) + (site_shift(storage) ? 2 * 4 * pitch : 0);
}

// ---------------------------------------------------------------------------
// Kernel dispatch tables.
using StepFn = void (*)(const Member *, int, int64_t, int64_t, int, FieldOut);
using ScatterFn = void (*)(const Member *, int, const double *, const double *, const double *, int, int);
using GatherFn = void (*)(const Member *, int, double *, int);

constexpr int TX_VALUES[4] = {64, 128, 256, 512};
int tx_index(int tx)
{
    for (int k = 0; k < 4; ++k)
        if (TX_VALUES[k] == tx) return k;
    return -1;
}

template <int ST, int F, int B, bool FIELDS>
StepFn step_for_tx(int k)
{
    switch (k) {
        case 0: return (StepFn)k_step<ST, F, B, 64, FIELDS>;
        case 1: return (StepFn)k_step<ST, F, B, 128, FIELDS>;
        case 2: return (StepFn)k_step<ST, F, B, 256, FIELDS>;
        default: return (StepFn)k_step<ST, F, B, 512, FIELDS>;
    }
}

template <int ST, int F, bool FIELDS>
StepFn step_for_bc(int bc, int k)
{
    switch (bc) {
        case BC_WALLS: return step_for_tx<ST, F, BC_WALLS, FIELDS>(k);
        case BC_PERIODIC: return step_for_tx<ST, F, BC_PERIODIC, FIELDS>(k);
        default: return step_for_tx<ST, F, BC_WALLS_WET, FIELDS>(k);
    }
}

// bc is a kernel boundary variant (BcY, lb_handle::kbc)
template <int ST, bool FIELDS>
StepFn step_for(int forcing, int bc, int k)
{
    if (forcing == LB_FORCE_SHIFT) return step_for_bc<ST, FORCE_SHIFT, FIELDS>(bc, k);
    return step_for_bc<ST, FORCE_GUO, FIELDS>(bc, k);
}

StepFn pick_step(int storage, int forcing, int bc, int k, bool fields)
{
    if (fields) {
        // the field pass does not depend on the forcing scheme
        switch (storage) {
            case LB_F64: return step_for_bc<ST_F64, FORCE_SHIFT, true>(bc, k);
            case LB_F32: return step_for_bc<ST_F32, FORCE_SHIFT, true>(bc, k);
            case LB_F16S: return step_for_bc<ST_F16S, FORCE_SHIFT, true>(bc, k);
            default: return step_for_bc<ST_BF16S, FORCE_SHIFT, true>(bc, k);
        }
    }
    switch (storage) {
        case LB_F64: return step_for<ST_F64, false>(forcing, bc, k);
        case LB_F32: return step_for<ST_F32, false>(forcing, bc, k);
        case LB_F16S: return step_for<ST_F16S, false>(forcing, bc, k);
        default: return step_for<ST_BF16S, false>(forcing, bc, k);
    }
}

using Step2Fn = void (*)(const Member *, int, int64_t, int64_t, int);

template <int ST, int F>
Step2Fn step2_for_bc(int bc)
{
    switch (bc) {
        case BC_WALLS: return (Step2Fn)k_step2<ST, F, BC_WALLS>;
        case BC_PERIODIC: return (Step2Fn)k_step2<ST, F, BC_PERIODIC>;
        default: return (Step2Fn)k_step2<ST, F, BC_WALLS_WET>;
    }
}

template <int ST>
Step2Fn step2_for(int forcing, int bc)
{
    return forcing == LB_FORCE_SHIFT ? step2_for_bc<ST, FORCE_SHIFT>(bc) : step2_for_bc<ST, FORCE_GUO>(bc);
}

Step2Fn pick_step2(int storage, int forcing, int bc)
{
    switch (storage) {
        case LB_F64: return step2_for<ST_F64>(forcing, bc);
        case LB_F32: return step2_for<ST_F32>(forcing, bc);
        case LB_F16S: return step2_for<ST_F16S>(forcing, bc);
        default: return step2_for<ST_BF16S>(forcing, bc);
    }
}

template <int ST, int F>
Step2Fn step3_for_bc(int bc)
{
    switch (bc) {
        case BC_WALLS: return (Step2Fn)k_step3<ST, F, BC_WALLS>;
        case BC_PERIODIC: return (Step2Fn)k_step3<ST, F, BC_PERIODIC>;
        default: return (Step2Fn)k_step3<ST, F, BC_WALLS_WET>;
    }
}

template <int ST>
Step2Fn step3_for(int forcing, int bc)
{
    return forcing == LB_FORCE_SHIFT ? step3_for_bc<ST, FORCE_SHIFT>(bc) : step3_for_bc<ST, FORCE_GUO>(bc);
}

Step2Fn pick_step3(int storage, int forcing, int bc)
{
    switch (storage) {
        case LB_F64: return step3_for<ST_F64>(forcing, bc);
        case LB_F32: return step3_for<ST_F32>(forcing, bc);
        case LB_F16S: return step3_for<ST_F16S>(forcing, bc);
        default: return step3_for<ST_BF16S>(forcing, bc);
    }
}

// state conversion depends only on periodic y or walls (an lb_config bc_y)
template <int ST>
ScatterFn scatter_for(int bc) { return bc == LB_WALLS ? k_scatter<ST, BC_WALLS> : k_scatter<ST, BC_PERIODIC>; }
template <int ST>
GatherFn gather_for(int bc) { return bc == LB_WALLS ? k_gather<ST, BC_WALLS> : k_gather<ST, BC_PERIODIC>; }

ScatterFn pick_scatter(int storage, int bc)
{
    switch (storage) {
        case LB_F64: return scatter_for<ST_F64>(bc);
        case LB_F32: return scatter_for<ST_F32>(bc);
        case LB_F16S: return scatter_for<ST_F16S>(bc);
        default: return scatter_for<ST_BF16S>(bc);
    }
}

GatherFn pick_gather(int storage, int bc)
{
    switch (storage) {
        case LB_F64: return gather_for<ST_F64>(bc);
        case LB_F32: return gather_for<ST_F32>(bc);
        case LB_F16S: return gather_for<ST_F16S>(bc);
        default: return gather_for<ST_BF16S>(bc);
    }
}

// ---------------------------------------------------------------------------
// Workspace layout.
struct Layout {
    size_t members;                 // Member table
    std::vector<size_t> fbuf[2];    // per member, buffer 0 and 1
    size_t fields;                  // [4][ny][nx] FP64 of the largest member
    size_t part;                    // [ny_max][RED_NQ] FP64 row partials
    size_t red;                     // [RED_NQ] FP64 results + profile [ny_max]
    size_t total;
};

bool build_layout(const lb_config *c, Layout &L)
{
    size_t off = 0;
    L.members = off;
    off = align_up(off + sizeof(Member) * (size_t)c->n_members, ALIGN);
    int64_t max_sites = 0, max_ny = 0;
    for (int b = 0; b < 2; ++b) L.fbuf[b].resize(c->n_members);
    for (int m = 0; m < c->n_members; ++m) {
        const lb_member &mm = c->members[m];
        const size_t bytes = (size_t)mm.ny * (size_t)row_bytes_of(c->storage, pitch_of(mm.nx));
        for (int b = 0; b < 2; ++b) {
            L.fbuf[b][m] = off;
            off = align_up(off + bytes, ALIGN);
        }
        max_sites = std::max<int64_t>(max_sites, (int64_t)mm.nx * mm.ny);
        max_ny = std::max<int64_t>(max_ny, mm.ny);
    }
    L.fields = off;
    off = align_up(off + (size_t)4 * (size_t)max_sites * sizeof(double), ALIGN);
    L.part = off;
    off = align_up(off + (size_t)max_ny * RED_NQ * sizeof(double), ALIGN);
    L.red = off;
    off = align_up(off + ((size_t)RED_NQ + (size_t)max_ny) * sizeof(double), ALIGN);
    L.total = off;
    return true;
}

// Eq. 6 on a wall row: sum_i w_i S(x + c_i) c_i,y in index order, where the
// boundary nodes are the row below row 0 (side 0) or above row ny - 1
// (side 1).  The x part cancels exactly (the two diagonal links).
double wall_link_sum(int side)
{
    double sw = 0.0;
    for (int i = 0; i < NQ; ++i) {
        const double S = (side == 0 ? cy(i) < 0 : cy(i) > 0) ? 1.0 : 0.0;
        sw += wgt(i) * S * cy(i);
    }
    return sw;
}

int32_t validate(const lb_config *c)
{
    if (!c) return fail(LB_EINVAL, "config is NULL");
    if (c->n_members < 1 || c->n_members > LB_MAX_MEMBERS)
        return fail(LB_EINVAL, "n_members = %d outside [1, %d]", c->n_members, LB_MAX_MEMBERS);
    if (!c->members) return fail(LB_EINVAL, "members is NULL");
    if (c->forcing != LB_FORCE_SHIFT && c->forcing != LB_FORCE_GUO)
        return fail(LB_EINVAL, "forcing = %d is not LB_FORCE_SHIFT or LB_FORCE_GUO", c->forcing);
    if (c->storage < LB_F64 || c->storage > LB_BF16S) return fail(LB_EINVAL, "storage = %d out of range", c->storage);
    if (c->bc_y != LB_WALLS && c->bc_y != LB_PERIODIC_Y) return fail(LB_EINVAL, "bc_y = %d out of range", c->bc_y);
    if (c->diag_trim < 1) return fail(LB_EINVAL, "diag_trim = %d must be >= 1", c->diag_trim);
    if (c->tile_x != 0 && tx_index(c->tile_x) < 0)
        return fail(LB_EINVAL, "tile_x = %d must be 0, 64, 128, 256 or 512", c->tile_x);
    if (c->tile_h < 0) return fail(LB_EINVAL, "tile_h = %d must be >= 0", c->tile_h);
    if (c->graph_chunk > 0 && (c->graph_chunk % 2 != 0))
        return fail(LB_EINVAL, "graph_chunk = %d must be even", c->graph_chunk);
    if (c->steps_per_pass < 0 || c->steps_per_pass > 3)
        return fail(LB_EINVAL, "steps_per_pass = %d must be 0, 1, 2 or 3", c->steps_per_pass);
    for (int m = 0; m < c->n_members; ++m) {
        const lb_member &mm = c->members[m];
        if (mm.nx < 3 || mm.ny < 3) return fail(LB_EINVAL, "member %d: nx = %d, ny = %d must be >= 3", m, mm.nx, mm.ny);
        if ((int64_t)mm.nx * mm.ny > ((int64_t)1 << 31))
            return fail(LB_EINVAL, "member %d: %d x %d sites exceed 2^31", m, mm.nx, mm.ny);
        if (row_bytes_of(c->storage, pitch_of(mm.nx)) > (int64_t)INT32_MAX)
            return fail(LB_EINVAL, "member %d: a row block of nx = %d exceeds 2^31 bytes", m, mm.nx);
        for (int s = 0; s < 2; ++s)
            if (!(mm.tau[s] > 0.5) || !std::isfinite(mm.tau[s]))
                return fail(LB_EINVAL, "member %d: tau[%d] = %g must be finite and > 1/2", m, s, mm.tau[s]);
        if (c->forcing == LB_FORCE_GUO && mm.tau[0] != mm.tau[1])
            return fail(LB_EINVAL, "member %d: Guo forcing needs tau_A == tau_B", m);
        if (!std::isfinite(mm.G_AB)) return fail(LB_EINVAL, "member %d: G_AB is not finite", m);
        for (int s = 0; s < 2; ++s)
            for (int a = 0; a < 2; ++a)
                if (!std::isfinite(mm.g[s][a])) return fail(LB_EINVAL, "member %d: g[%d][%d] is not finite", m, s, a);
        for (int s = 0; s < 2; ++s)
            if (!std::isfinite(mm.G_wall[s])) return fail(LB_EINVAL, "member %d: G_wall[%d] is not finite", m, s);
        if (mm.wall_psi != LB_PSI_MIRROR && mm.wall_psi != LB_PSI_ZERO)
            return fail(LB_EINVAL, "member %d: wall_psi = %d is not LB_PSI_MIRROR or LB_PSI_ZERO", m, mm.wall_psi);
        if (mm.reserved != 0) return fail(LB_EINVAL, "member %d: reserved = %d must be 0", m, mm.reserved);
        if (mm.reserved2[0] != 0.0 || mm.reserved2[1] != 0.0)
            return fail(LB_EINVAL, "member %d: reserved2 must be 0", m);
        if (!mm.rhoA0 || !mm.rhoB0) return fail(LB_EINVAL, "member %d: initial densities are NULL", m);
        if (mm.ny <= 2 * c->diag_trim) return fail(LB_EINVAL, "member %d: ny = %d leaves no rows after trimming %d", m, mm.ny, c->diag_trim);
    }
    return LB_OK;
}

}  // namespace

struct lb_handle {
    lb_config cfg{};
    std::vector<lb_member> mem;     // parameters (host pointers cleared after init)
    std::vector<Member> dm;         // device table mirror
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;  // private stream used only to record graphs
    char *ws = nullptr;
    Layout L;
    int64_t t = 0;
    int cur = 0;
    int tile_x = 0;
    int64_t n_items = 0;
    int kbc = BC_WALLS;             // boundary variant of the step kernels: BC_PERIODIC, BC_WALLS, or
                                    // BC_WALLS_WET when a member has a wall force or psi = 0 beyond walls
    int steps_per_pass = 1;         // 2 / 3: lb_step runs the two- / three-step pass
    int64_t n_items2 = 0;
    int64_t n_items3 = 0;
    int chunk = 0;
    int chunk_flip = 0;             // buffer parity change of one graph replay
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipGraph_t graph_src[2] = {nullptr, nullptr};
    int device = 0;
    std::vector<double> bulk_ref;   // per member: phibar at rows diag_trim and ny - diag_trim - 1 at t = 0
    int tiles_cached = 0;           // 1: the tile choice came from the persisted cache
};

namespace {

std::mutex g_live_mu;
std::set<const lb_handle *> g_live;

bool is_live(const lb_handle *h)
{
    std::lock_guard<std::mutex> lk(g_live_mu);
    return h && g_live.count(h) > 0;
}

Member *dev_members(lb_handle *h) { return (Member *)(h->ws + h->L.members); }

// Tiles of each member (tile_x columns by th[m] rows) and their work items:
// member m owns items [item_begin, item_end) in row-major tile order.
void plan_tiles(lb_handle *h, int tx, const std::vector<int> &th)
{
    int64_t item = 0;
    for (size_t m = 0; m < h->dm.size(); ++m) {
        Member &M = h->dm[m];
        M.tiles_x = (M.nx + tx - 1) / tx;
        M.tile_h = std::max(1, std::min(th[m], M.ny));
        M.tiles_y = (M.ny + M.tile_h - 1) / M.tile_h;
        M.item_begin = item;
        item += (int64_t)M.tiles_x * M.tiles_y;
        M.item_end = item;
    }
    h->n_items = item;
    h->tile_x = tx;
}

// Bands of the two-step pass: TX2 output columns by th[m] rows.
void plan_tiles2(lb_handle *h, const std::vector<int> &th)
{
    int64_t item = 0;
    for (size_t m = 0; m < h->dm.size(); ++m) {
        Member &M = h->dm[m];
        M.tiles_x2 = (M.nx + TX2 - 1) / TX2;
        M.tile_h2 = std::max(1, std::min(th[m], M.ny));
        M.tiles_y2 = (M.ny + M.tile_h2 - 1) / M.tile_h2;
        M.item2_begin = item;
        item += (int64_t)M.tiles_x2 * M.tiles_y2;
        M.item2_end = item;
    }
    h->n_items2 = item;
}

// Bands of the three-step pass: TX3 output columns by th[m] rows.
void plan_tiles3(lb_handle *h, const std::vector<int> &th)
{
    int64_t item = 0;
    for (size_t m = 0; m < h->dm.size(); ++m) {
        Member &M = h->dm[m];
        M.tiles_x3 = (M.nx + TX3 - 1) / TX3;
        M.tile_h3 = std::max(1, std::min(th[m], M.ny));
        M.tiles_y3 = (M.ny + M.tile_h3 - 1) / M.tile_h3;
        M.item3_begin = item;
        item += (int64_t)M.tiles_x3 * M.tiles_y3;
        M.item3_end = item;
    }
    h->n_items3 = item;
}

int32_t upload_members(lb_handle *h)
{
    HIP_TRY(hipMemcpyAsync(dev_members(h), h->dm.data(), sizeof(Member) * h->dm.size(), hipMemcpyHostToDevice, h->stream));
    return LB_OK;
}

// n steps from buffer cur: three-step passes when selected, then two-step
// passes when selected or when two steps remain of three-step passes, then
// single steps.  Every pass reads buffer cur and writes the other one.
int32_t launch_steps(lb_handle *h, hipStream_t s, int64_t n, int &cur)
{
    if (h->steps_per_pass == 3) {
        Step2Fn fn3 = pick_step3(h->cfg.storage, h->cfg.forcing, h->kbc);
        for (; n >= 3; n -= 3) {
            hipLaunchKernelGGL(fn3, dim3((unsigned)((h->n_items3 + NW2 - 1) / NW2)), dim3(64 * NW2), 0, s,
                               (const Member *)dev_members(h),
                               (int)h->dm.size(), (int64_t)0, h->n_items3, cur);
            cur ^= 1;
        }
    }
    if (h->steps_per_pass >= 2) {
        Step2Fn fn2 = pick_step2(h->cfg.storage, h->cfg.forcing, h->kbc);
        for (; n >= 2; n -= 2) {
            hipLaunchKernelGGL(fn2, dim3((unsigned)((h->n_items2 + NW2 - 1) / NW2)), dim3(64 * NW2), 0, s,
                               (const Member *)dev_members(h),
                               (int)h->dm.size(), (int64_t)0, h->n_items2, cur);
            cur ^= 1;
        }
    }
    StepFn fn = pick_step(h->cfg.storage, h->cfg.forcing, h->kbc, tx_index(h->tile_x), false);
    const FieldOut none{nullptr, nullptr, nullptr, nullptr};
    for (int64_t k = 0; k < n; ++k) {
        hipLaunchKernelGGL(fn, dim3((unsigned)h->n_items), dim3(h->tile_x), 0, s, (const Member *)dev_members(h),
                           (int)h->dm.size(), (int64_t)0, h->n_items, cur, none);
        cur ^= 1;
    }
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

void free_graphs(lb_handle *h)
{
    for (int p = 0; p < 2; ++p) {
        if (h->graph[p]) (void)hipGraphExecDestroy(h->graph[p]);
        if (h->graph_src[p]) (void)hipGraphDestroy(h->graph_src[p]);
        h->graph[p] = nullptr;
        h->graph_src[p] = nullptr;
    }
}

// Record one graph per starting buffer parity: chunk launches of the step.
int32_t build_graphs(lb_handle *h)
{
    free_graphs(h);
    if (h->chunk <= 0) return LB_OK;
    for (int p = 0; p < 2; ++p) {
        HIP_TRY(hipStreamBeginCapture(h->capture, hipStreamCaptureModeThreadLocal));
        int c = p;
        int32_t rc = launch_steps(h, h->capture, h->chunk, c);
        h->chunk_flip = c ^ p;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(h->capture, &g);
        if (rc != LB_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(LB_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
        h->graph_src[p] = g;
        HIP_TRY(hipGraphInstantiate(&h->graph[p], g, nullptr, nullptr, 0));
    }
    return LB_OK;
}

// Time `reps` steps that read the current buffer and write the other one
// (state unchanged) with tile shape (tx, th); returns milliseconds per step.
int32_t time_shape(lb_handle *h, int tx, const std::vector<int> &th, int reps, float &ms)
{
    plan_tiles(h, tx, th);
    int32_t rc = upload_members(h);
    if (rc) return rc;
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    StepFn fn = pick_step(h->cfg.storage, h->cfg.forcing, h->kbc, tx_index(tx), false);
    const FieldOut none{nullptr, nullptr, nullptr, nullptr};
    auto once = [&]() {
        hipLaunchKernelGGL(fn, dim3((unsigned)h->n_items), dim3(tx), 0, h->stream, (const Member *)dev_members(h),
                           (int)h->dm.size(), (int64_t)0, h->n_items, h->cur, none);
    };
    once();  // warm-up
    HIP_TRY(hipEventRecord(a, h->stream));
    for (int r = 0; r < reps; ++r) once();
    HIP_TRY(hipEventRecord(b, h->stream));
    HIP_TRY(hipEventSynchronize(b));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventElapsedTime(&ms, a, b));
    ms /= (float)reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return LB_OK;
}

// Time `reps` two-step passes (read the current buffer, write the other one)
// with band heights th; returns milliseconds per step (half a pass).
int32_t time_shape2(lb_handle *h, const std::vector<int> &th, int reps, float &ms)
{
    plan_tiles2(h, th);
    int32_t rc = upload_members(h);
    if (rc) return rc;
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    Step2Fn fn = pick_step2(h->cfg.storage, h->cfg.forcing, h->kbc);
    auto once = [&]() {
        hipLaunchKernelGGL(fn, dim3((unsigned)((h->n_items2 + NW2 - 1) / NW2)), dim3(64 * NW2), 0, h->stream,
                           (const Member *)dev_members(h),
                           (int)h->dm.size(), (int64_t)0, h->n_items2, h->cur);
    };
    once();  // warm-up
    HIP_TRY(hipEventRecord(a, h->stream));
    for (int r = 0; r < reps; ++r) once();
    HIP_TRY(hipEventRecord(b, h->stream));
    HIP_TRY(hipEventSynchronize(b));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventElapsedTime(&ms, a, b));
    ms /= (float)(2 * reps);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return LB_OK;
}

// Time `reps` three-step passes with band heights th; returns milliseconds
// per step (a third of a pass).
int32_t time_shape3(lb_handle *h, const std::vector<int> &th, int reps, float &ms)
{
    plan_tiles3(h, th);
    int32_t rc = upload_members(h);
    if (rc) return rc;
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    Step2Fn fn = pick_step3(h->cfg.storage, h->cfg.forcing, h->kbc);
    auto once = [&]() {
        hipLaunchKernelGGL(fn, dim3((unsigned)((h->n_items3 + NW2 - 1) / NW2)), dim3(64 * NW2), 0, h->stream,
                           (const Member *)dev_members(h),
                           (int)h->dm.size(), (int64_t)0, h->n_items3, h->cur);
    };
    once();  // warm-up
    HIP_TRY(hipEventRecord(a, h->stream));
    for (int r = 0; r < reps; ++r) once();
    HIP_TRY(hipEventRecord(b, h->stream));
    HIP_TRY(hipEventSynchronize(b));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventElapsedTime(&ms, a, b));
    ms /= (float)(3 * reps);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return LB_OK;
}

// Tile shapes.  Explicit tile_x / tile_h apply to every member.  Otherwise
// each candidate is timed with a coordinate search over one tile height per
// member size class (members of equal nx, ny share it), timing whole
// ensemble passes that read the current buffer and write the other one (the
// state is unchanged); the fastest is kept.  The single-step pass always
// gets a shape (it serves odd remainders and the field pass); the two- and
// three-step passes are planned when they may be used (the two-step pass also
// takes two remaining steps of three-step passes), and with
// steps_per_pass == 0 the fastest per step is selected.
int32_t search_tiles(lb_handle *h)
{
    const lb_config &c = h->cfg;
    const size_t nm = h->dm.size();
    int64_t max_nx = 0, sites = 0;
    for (auto &M : h->dm) {
        max_nx = std::max<int64_t>(max_nx, M.nx);
        sites += (int64_t)M.nx * M.ny;
    }
    // size classes
    std::vector<int> cls(nm);
    std::vector<std::pair<int, int>> shapes;
    for (size_t m = 0; m < nm; ++m) {
        const std::pair<int, int> key{h->dm[m].nx, h->dm[m].ny};
        auto it = std::find(shapes.begin(), shapes.end(), key);
        cls[m] = (int)(it - shapes.begin());
        if (it == shapes.end()) shapes.push_back(key);
    }
    // about 20 ms of work per timing at ~20 GLUPS
    const int reps = (int)std::max<int64_t>(2, std::min<int64_t>(20, (int64_t)4e8 / std::max<int64_t>(sites, 1)));
    // coordinate search over per-class heights; time(thm, ms) times one shape
    auto search = [&](const std::vector<int> &heights, int start, auto &&time_fn, std::vector<int> &best_th,
                      float &best_ms) -> int32_t {
        std::vector<int> hc(shapes.size(), heights.size() > 1 ? start : heights.front());
        best_ms = 1e30f;
        for (size_t k = 0; k < shapes.size(); ++k) {
            int keep = hc[k];
            for (int th : heights) {
                hc[k] = th;
                std::vector<int> thm(nm);
                for (size_t m = 0; m < nm; ++m) thm[m] = hc[cls[m]];
                float ms = 0;
                int32_t rc = time_fn(thm, ms);
                if (rc) return rc;
                if (ms < best_ms) {
                    best_ms = ms;
                    keep = th;
                }
            }
            hc[k] = keep;
        }
        best_th.assign(nm, 0);
        for (size_t m = 0; m < nm; ++m) best_th[m] = hc[cls[m]];
        return LB_OK;
    };
    const int spp = c.steps_per_pass != 0 ? c.steps_per_pass : (c.tile_x != 0 ? 1 : 0);

    // --- single-step pass
    float best1 = 1e30f;
    int best_tx = c.tile_x != 0 ? c.tile_x : 128;
    std::vector<int> best_th(nm, c.tile_h > 0 ? c.tile_h : 16);
    if (c.tile_x == 0 && spp != 2 && spp != 3) {
        std::vector<int> heights = {8, 12, 16, 32, 64, 128};
        if (c.tile_h > 0) heights = {c.tile_h};
        for (int tx : {64, 128, 256, 512}) {
            if (tx > 64 && tx / 2 >= max_nx) continue;
            std::vector<int> th;
            float ms = 0;
            int32_t rc = search(heights, 32, [&](const std::vector<int> &thm, float &t) {
                return time_shape(h, tx, thm, reps, t);
            }, th, ms);
            if (rc) return rc;
            if (ms < best1) {
                best1 = ms;
                best_tx = tx;
                best_th = th;
            }
        }
    }
    plan_tiles(h, best_tx, best_th);

    // --- two-step pass
    h->steps_per_pass = 1;
    if (spp != 1) {
        std::vector<int> th2(nm, c.tile_h > 0 ? c.tile_h : 12);
        float best2 = 0.0f;
        if (c.tile_h == 0 || spp == 0) {
            std::vector<int> heights = {6, 7, 8, 9, 10, 12, 16, 24};
            if (c.tile_h > 0) heights = {c.tile_h};
            int32_t rc = search(heights, 12, [&](const std::vector<int> &thm, float &t) {
                return time_shape2(h, thm, reps, t);
            }, th2, best2);
            if (rc) return rc;
        }
        plan_tiles2(h, th2);
        if (spp == 2 || (spp == 0 && best2 < best1)) h->steps_per_pass = 2;
        if (spp == 0 && best2 < best1) best1 = best2;
    }

    // --- three-step pass
    std::vector<int> th3(nm, c.tile_h > 0 ? c.tile_h : 24);
    if (spp == 0 || spp == 3) {
        float best3 = 1e30f;
        if (c.tile_h == 0 || spp == 0) {
            std::vector<int> heights = {8, 12, 16, 24, 32, 48, 64, 96, 128, 160};
            // Heights that fill whole rounds of the GPU's wave slots: each work
            // item is one wave, the FP64 pass runs one wave per SIMD and the
            // others two, so S = CUs x 4 (x 2) items run at once.  With n items
            // per row of bands, a height h takes r = ceil(nb n / S) rounds for
            // its nb = ceil(ny / h) bands; the most bands that fit those rounds,
            // floor(r S / n), of ceil(ny / that) rows each, leave none of the
            // last round idle.  Tall bands feel it most (10000 x 5000 FP64:
            // 37.9 GLUPS at 160 rows, 39.5-40.3 at the filled 455, 313, 228,
            // 186 and 152).  Every candidate, and a few taller ones, gets its
            // filled height as a candidate too; one size class only (mixed
            // sizes share rounds).
            if (shapes.size() == 1) {
                int cus = 0;
                if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess)
                    cus = 0;
                const int64_t slots = (int64_t)cus * 4 * (c.storage == LB_F64 ? 1 : 2);
                const int64_t per_band = (int64_t)nm * ((shapes[0].first + TX3 - 1) / TX3);
                const int64_t ny3 = shapes[0].second;
                std::vector<int> from = heights;
                for (int tall : {192, 256, 320, 384, 512}) from.push_back(tall);
                for (int hgt : from) {
                    if (slots <= 0) break;
                    const int64_t nb = (ny3 + hgt - 1) / hgt;
                    const int64_t r = (nb * per_band + slots - 1) / slots;
                    const int64_t nbf = r * slots / per_band;
                    if (nbf < 1) continue;
                    const int hf = (int)((ny3 + nbf - 1) / nbf);
                    if (hf >= 8 && hf <= 512 && std::find(heights.begin(), heights.end(), hf) == heights.end())
                        heights.push_back(hf);
                }
            }
            if (c.tile_h > 0) heights = {c.tile_h};
            int32_t rc = search(heights, 24, [&](const std::vector<int> &thm, float &t) {
                return time_shape3(h, thm, reps, t);
            }, th3, best3);
            if (rc) return rc;
        }
        if (spp == 3 || best3 < best1) h->steps_per_pass = 3;
    }
    plan_tiles3(h, th3);
    return upload_members(h);
}

// Size classes of the members (distinct nx, ny in order of first
// appearance) and each member's class.
void size_classes(const lb_handle *h, std::vector<std::pair<int, int>> &shapes, std::vector<int> &cls)
{
    shapes.clear();
    cls.assign(h->dm.size(), 0);
    for (size_t m = 0; m < h->dm.size(); ++m) {
        const std::pair<int, int> key{h->dm[m].nx, h->dm[m].ny};
        auto it = std::find(shapes.begin(), shapes.end(), key);
        cls[m] = (int)(it - shapes.begin());
        if (it == shapes.end()) shapes.push_back(key);
    }
}

// Key of the tile choice: device, every input of the search and the member sizes.
std::string tune_key(const lb_handle *h)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    const lb_config &c = h->cfg;
    // s2: the search with the round-filling band heights of the three-step pass
    std::string k = arch + "|cu" + std::to_string(cus) + "|s2|st" + std::to_string(c.storage) + "|f" +
                    std::to_string(c.forcing) + "|bc" + std::to_string(h->kbc) + "|spp" +
                    std::to_string(c.steps_per_pass) + "|tx" + std::to_string(c.tile_x) + "|th" +
                    std::to_string(c.tile_h) + "|";
    for (size_t m = 0; m < h->dm.size(); ++m)
        k += (m ? "," : "") + std::to_string(h->dm[m].nx) + "x" + std::to_string(h->dm[m].ny);
    for (char &ch : k)
        if (ch == '"' || ch == '\\') ch = '_';
    return k;
}

// Tile choice: from the persisted cache when it holds this configuration,
// else by the timed search (whose result is then recorded).  Explicit tile
// shapes need no search and bypass the cache.
int32_t choose_tiles(lb_handle *h)
{
    const lb_config &c = h->cfg;
    h->tiles_cached = 0;
    if (c.tile_x != 0 && c.tile_h != 0) return search_tiles(h);
    std::vector<std::pair<int, int>> shapes;
    std::vector<int> cls;
    size_classes(h, shapes, cls);
    const std::string key = tune_key(h);
    lbtune::Choice ch;
    if (lbtune::lookup(key, ch) && ch.spp >= 1 && ch.spp <= 3 && tx_index(ch.tx) >= 0 &&
        ch.th.size() == shapes.size() && ch.th2.size() == shapes.size() && ch.th3.size() == shapes.size()) {
        std::vector<int> th(h->dm.size()), th2(h->dm.size()), th3(h->dm.size());
        for (size_t m = 0; m < h->dm.size(); ++m) {
            th[m] = std::max(1, ch.th[cls[m]]);
            th2[m] = std::max(1, ch.th2[cls[m]]);
            th3[m] = std::max(1, ch.th3[cls[m]]);
        }
        plan_tiles(h, ch.tx, th);
        plan_tiles2(h, th2);
        plan_tiles3(h, th3);
        h->steps_per_pass = ch.spp;
        h->tiles_cached = 1;
        return upload_members(h);
    }
    int32_t rc = search_tiles(h);
    if (rc) return rc;
    ch.spp = h->steps_per_pass;
    ch.tx = h->tile_x;
    ch.th.assign(shapes.size(), 0);
    ch.th2.assign(shapes.size(), 0);
    ch.th3.assign(shapes.size(), 0);
    for (size_t m = 0; m < h->dm.size(); ++m) {
        ch.th[cls[m]] = h->dm[m].tile_h;
        ch.th2[cls[m]] = h->dm[m].tile_h2;
        ch.th3[cls[m]] = h->dm[m].tile_h3;
    }
    lbtune::store(key, ch);
    return LB_OK;
}

// Per-member code scales of the 16-bit modes.  A code holds the residual
// f*_i - w_i rho of a site's own density rho: the velocity terms of Eq. 3 and
// the non-equilibrium part.  At |u| <= 1/2, |c_i . u| <= 0.71, so
// |f^eq_i - w_i rho| <= w_i rho (3 * 0.71 + 4.5 * 0.5 + 1.5 * 0.25) < 5 w_i rho;
// with a factor 8 instead of 5, and rho_ref twice the largest initial density
// of either component (compression, components that spread), the binary16
// code q = residual * S_i stays below 2^14, far from the format's 65504.
// bfloat16 has the FP32 exponent range and needs no scale (S_i = 1).
void set_scales(const lb_config *c, const lb_member &mm, Member &M)
{
    const int64_t n = (int64_t)mm.nx * mm.ny;
    double hi = 0.0;
    for (int s = 0; s < 2; ++s) {
        const double *rho = s == 0 ? mm.rhoA0 : mm.rhoB0;
        for (int64_t k = 0; k < n; ++k) hi = std::max(hi, std::fabs(rho[k]));
    }
    const double rho_ref = 2.0 * std::max(hi, 1e-6);
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < NQ; ++i) {
            int e = 0;
            if (c->storage == LB_F16S) e = (int)std::floor(std::log2(16384.0 / (8.0 * wgt(i) * rho_ref)));
            e = std::max(-60, std::min(60, e));
            M.scale[s][i] = std::ldexp(1.0f, e);
            M.iscale[s][i] = std::ldexp(1.0f, -e);
        }
    // the kernels take S_i per weight class (the rule above depends on w_i
    // only, not on s) and bfloat16 codes as unscaled (e = 0 above: S_i = 1)
    for (int k = 0; k < 3; ++k) {
        const int i = k == 0 ? 0 : (k == 1 ? 1 : 5);
        M.cscale[k] = M.scale[0][i];
        M.ciscale[k] = M.iscale[0][i];
    }
}

// Field pass of member m (rho_A, rho_B, u_x, u_y of f(t) into device
// buffers; any may be null).  Asynchronous.
int32_t enqueue_fields(lb_handle *h, int32_t m, double *d_rhoA, double *d_rhoB, double *d_ux, double *d_uy)
{
    const Member &M = h->dm[m];
    StepFn fn = pick_step(h->cfg.storage, h->cfg.forcing, h->kbc, tx_index(h->tile_x), true);
    FieldOut fo{d_rhoA, d_rhoB, d_ux, d_uy};
    const int64_t n_items = M.item_end - M.item_begin;
    hipLaunchKernelGGL(fn, dim3((unsigned)n_items), dim3(h->tile_x), 0, h->stream, (const Member *)dev_members(h),
                       (int)h->dm.size(), M.item_begin, n_items, h->cur, fo);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

// Field pass of member m into the workspace field buffer, then the per-row
// partial sums and their totals: red[0..RED_NQ) and the row profile of phi at
// red + RED_NQ.  Asynchronous.
int32_t enqueue_reductions(lb_handle *h, int32_t m)
{
    const Member &M = h->dm[m];
    const lb_member &mm = h->mem[m];
    const int64_t n = (int64_t)M.nx * M.ny;
    double *fld = (double *)(h->ws + h->L.fields);
    int32_t rc = enqueue_fields(h, m, fld, fld + n, fld + 2 * n, fld + 3 * n);
    if (rc) return rc;
    double *part = (double *)(h->ws + h->L.part);
    double *red = (double *)(h->ws + h->L.red);
    hipLaunchKernelGGL(k_reduce_rows, dim3(M.ny), dim3(RED_THREADS), 0, h->stream, (const double *)fld,
                       (const double *)(fld + n), (const double *)(fld + 2 * n), (const double *)(fld + 3 * n), M.nx,
                       M.ny, h->cfg.diag_trim, mm.g[0][0], mm.g[0][1], mm.g[1][0], mm.g[1][1], part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, h->stream, (const double *)part, M.nx, M.ny, red,
                       red + RED_NQ);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

// The bulk references of the mixing width: phibar at the first and the last
// row of the trimmed domain, from the current state of every member.
int32_t record_bulk_refs(lb_handle *h)
{
    const int trim = h->cfg.diag_trim;
    h->bulk_ref.assign(2 * h->dm.size(), 0.0);
    double *prof = (double *)(h->ws + h->L.red) + RED_NQ;
    for (size_t m = 0; m < h->dm.size(); ++m) {
        int32_t rc = enqueue_reductions(h, (int32_t)m);
        if (rc) return rc;
        const int ny = h->dm[m].ny;
        HIP_TRY(hipMemcpyAsync(&h->bulk_ref[2 * m], prof + trim, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(&h->bulk_ref[2 * m + 1], prof + (ny - trim - 1), sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    return LB_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

const char *lb_last_error(void) { return lbrt::g_err.c_str(); }

size_t lb_workspace_bytes(const lb_config *cfg)
{
    if (validate(cfg) != LB_OK) return 0;
    Layout L;
    build_layout(cfg, L);
    return L.total;
}

int32_t lb_init(const lb_config *cfg, void *d_workspace, size_t bytes, void *hip_stream, lb_handle **out)
{
    if (!out) return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    int32_t rc = validate(cfg);
    if (rc) return rc;
    if (!d_workspace) return fail(LB_EINVAL, "workspace is NULL");
    if (((uintptr_t)d_workspace) % ALIGN) return fail(LB_EINVAL, "workspace is not %zu-byte aligned", ALIGN);
    Layout L;
    build_layout(cfg, L);
    if (bytes < L.total) return fail(LB_ENOMEM, "workspace of %zu bytes, %zu needed", bytes, L.total);

    lb_handle *h = new (std::nothrow) lb_handle();
    if (!h) return fail(LB_EINVAL, "host allocation failed");
    h->cfg = *cfg;
    h->mem.assign(cfg->members, cfg->members + cfg->n_members);
    h->cfg.members = nullptr;
    h->stream = (hipStream_t)hip_stream;
    h->ws = (char *)d_workspace;
    h->L = L;
    h->chunk = cfg->graph_chunk == 0 ? 100 : (cfg->graph_chunk < 0 ? 0 : cfg->graph_chunk);

    auto bail = [&](int32_t code) {
        free_graphs(h);
        if (h->capture) (void)hipStreamDestroy(h->capture);
        delete h;
        return code;
    };
    if (hipGetDevice(&h->device) != hipSuccess) return bail(fail(LB_EHIP, "hipGetDevice failed"));
    if (hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(LB_EHIP, "hipStreamCreateWithFlags failed"));

    h->dm.resize(cfg->n_members);
    for (int m = 0; m < cfg->n_members; ++m) {
        const lb_member &mm = cfg->members[m];
        Member &M = h->dm[m];
        std::memset(&M, 0, sizeof M);
        M.nx = mm.nx;
        M.ny = mm.ny;
        M.pitch = (int32_t)pitch_of(mm.nx);
        // row blocks [y][s][i][x]: the 18 row segments of one lattice row are
        // adjacent; in the 16-bit modes the two FP32 site-density segments
        // [s][x] follow them
        M.istride = M.pitch;
        M.sstride = (int64_t)NQ * M.pitch;
        M.ystride = row_bytes_of(cfg->storage, M.pitch) / (int64_t)elem_bytes(cfg->storage);
        M.rho_off = site_shift(cfg->storage) ? (int32_t)(2 * NQ * M.pitch * (int64_t)elem_bytes(cfg->storage)) : 0;
        M.rho_sstride = site_shift(cfg->storage) ? 4 * M.pitch : 0;
        M.f[0] = h->ws + L.fbuf[0][m];
        M.f[1] = h->ws + L.fbuf[1][m];
        for (int s = 0; s < 2; ++s) {
            M.tau[s] = mm.tau[s];
            M.itau[s] = 1.0 / mm.tau[s];
            M.g[s][0] = mm.g[s][0];
            M.g[s][1] = mm.g[s][1];
        }
        M.G = mm.G_AB;
        // Eq. 6: a^w_s = -G_sb sum_i w_i S(x + c_i) c_i on the wall rows
        M.wall_force = cfg->bc_y == LB_WALLS && (mm.G_wall[0] != 0.0 || mm.G_wall[1] != 0.0);
        M.psi_zero = mm.wall_psi == LB_PSI_ZERO;
        for (int side = 0; side < 2; ++side) {
            const double sw = wall_link_sum(side);
            for (int s = 0; s < 2; ++s) M.aw[s][side] = -(mm.G_wall[s] * sw);
        }
        set_scales(cfg, mm, M);
        if (M.wall_force || M.psi_zero) h->kbc = BC_WALLS_WET;
    }
    if (cfg->bc_y == LB_PERIODIC_Y) h->kbc = BC_PERIODIC;
    plan_tiles(h, cfg->tile_x ? cfg->tile_x : 64, std::vector<int>(cfg->n_members, cfg->tile_h ? cfg->tile_h : 16));
    plan_tiles2(h, std::vector<int>(cfg->n_members, 12));
    plan_tiles3(h, std::vector<int>(cfg->n_members, 24));
    if ((rc = upload_members(h))) return bail(rc);

    // initial state f(0) = w_i rho_s(0), written as the pre-streamed buffer
    double *stage = (double *)(h->ws + L.fields);
    for (int m = 0; m < cfg->n_members; ++m) {
        const lb_member &mm = cfg->members[m];
        const size_t n = (size_t)mm.nx * mm.ny;
        if (hipMemcpyAsync(stage, mm.rhoA0, n * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
            hipMemcpyAsync(stage + n, mm.rhoB0, n * sizeof(double), hipMemcpyHostToDevice, h->stream) != hipSuccess)
            return bail(fail(LB_EHIP, "copy of initial densities failed"));
        ScatterFn fn = pick_scatter(cfg->storage, cfg->bc_y);
        const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
        hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, h->stream, (const Member *)dev_members(h), m,
                           (const double *)nullptr, (const double *)stage, (const double *)(stage + n), 1, 0);
        if (hipGetLastError() != hipSuccess) return bail(fail(LB_EHIP, "initial scatter launch failed"));
        // the staging area is reused by the next member only after this one is written
        if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(fail(LB_EHIP, "stream synchronisation failed"));
    }
    for (auto &mm : h->mem) {
        mm.rhoA0 = nullptr;
        mm.rhoB0 = nullptr;
    }
    if ((rc = choose_tiles(h))) return bail(rc);
    if ((rc = record_bulk_refs(h))) return bail(rc);
    if ((rc = build_graphs(h))) return bail(rc);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(fail(LB_EHIP, "stream synchronisation failed"));
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        g_live.insert(h);
    }
    *out = h;
    return LB_OK;
}

int32_t lb_step(lb_handle *h, int64_t n)
{
    if (!is_live(h)) return fail(LB_ESTATE, "handle is not live");
    if (n < 0) return fail(LB_EINVAL, "n = %lld must be >= 0", (long long)n);
    int64_t left = n;
    if (h->chunk > 0) {
        while (left >= h->chunk) {
            HIP_TRY(hipGraphLaunch(h->graph[h->cur], h->stream));
            h->cur ^= h->chunk_flip;
            left -= h->chunk;
        }
    }
    int c = h->cur;
    int32_t rc = launch_steps(h, h->stream, left, c);
    if (rc) return rc;
    h->cur = c;
    h->t += n;
    return LB_OK;
}

int32_t lb_fields(lb_handle *h, int32_t m, double *d_rhoA, double *d_rhoB, double *d_ux, double *d_uy)
{
    if (!is_live(h)) return fail(LB_ESTATE, "handle is not live");
    if (m < 0 || m >= (int32_t)h->dm.size()) return fail(LB_EINVAL, "member %d out of range", m);
    return enqueue_fields(h, m, d_rhoA, d_rhoB, d_ux, d_uy);
}

int32_t lb_diagnostics(lb_handle *h, int32_t m, lb_diag *out, double *phi_profile)
{
    if (!is_live(h)) return fail(LB_ESTATE, "handle is not live");
    if (m < 0 || m >= (int32_t)h->dm.size()) return fail(LB_EINVAL, "member %d out of range", m);
    if (!out) return fail(LB_EINVAL, "out is NULL");
    const Member &M = h->dm[m];
    double *red = (double *)(h->ws + h->L.red);
    int32_t rc = enqueue_reductions(h, m);
    if (rc) return rc;
    std::vector<double> host((size_t)RED_NQ + (phi_profile ? (size_t)M.ny : 0));
    HIP_TRY(hipMemcpyAsync(host.data(), red, host.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const double nd = (double)M.nx * (double)(M.ny - 2 * h->cfg.diag_trim);
    out->t = h->t;
    out->mass[0] = host[0];
    out->mass[1] = host[1];
    out->Ek = host[3] / nd;
    out->Ep = host[4] / nd;
    out->buoyancy = host[5] / nd;
    out->omega2 = host[6] / nd;
    out->umax = host[7];
    out->finite = host[8] == 0.0 ? 1 : 0;
    if (phi_profile) std::memcpy(phi_profile, host.data() + RED_NQ, (size_t)M.ny * sizeof(double));
    if (!out->finite) return fail(LB_ENONFINITE, "member %d: %.0f non-finite densities or velocities at t = %lld", m,
                                  host[8], (long long)h->t);
    return LB_OK;
}

int32_t lb_mixing_width(lb_handle *h, int32_t m, const double *ref, lb_mixing *out)
{
    if (!is_live(h)) return fail(LB_ESTATE, "handle is not live");
    if (m < 0 || m >= (int32_t)h->dm.size()) return fail(LB_EINVAL, "member %d out of range", m);
    if (!out) return fail(LB_EINVAL, "out is NULL");
    const double lo = ref ? ref[0] : h->bulk_ref[2 * m], hi = ref ? ref[1] : h->bulk_ref[2 * m + 1];
    if (!std::isfinite(lo) || !std::isfinite(hi) || lo == hi)
        return fail(LB_EINVAL, "member %d: bulk references %g and %g must be finite and differ", m, lo, hi);
    const Member &M = h->dm[m];
    int32_t rc = enqueue_reductions(h, m);
    if (rc) return rc;
    double *red = (double *)(h->ws + h->L.red);
    // the width goes to red[RED_NQ - 1] (the non-finite count, not needed here)
    hipLaunchKernelGGL(k_mixing_width, dim3(1), dim3(RED_THREADS), 0, h->stream, (const double *)(red + RED_NQ),
                       M.ny, h->cfg.diag_trim, lo, hi, red + RED_NQ - 1);
    HIP_TRY(hipGetLastError());
    double w = 0.0;
    HIP_TRY(hipMemcpyAsync(&w, red + RED_NQ - 1, sizeof w, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    out->t = h->t;
    out->width = w;
    out->bulk_ref[0] = lo;
    out->bulk_ref[1] = hi;
    return LB_OK;
}

int32_t lb_energy_budget(lb_handle *h, int32_t m, lb_budget *out)
{
    if (!is_live(h)) return fail(LB_ESTATE, "handle is not live");
    if (m < 0 || m >= (int32_t)h->dm.size()) return fail(LB_EINVAL, "member %d out of range", m);
    if (!out) return fail(LB_EINVAL, "out is NULL");
    if (h->cfg.diag_trim < 2)
        return fail(LB_EINVAL, "the budget stencils reach two rows: diag_trim = %d must be >= 2", h->cfg.diag_trim);
    const Member &M = h->dm[m];
    const lb_member &mm = h->mem[m];
    const int64_t n = (int64_t)M.nx * M.ny;
    double *fld = (double *)(h->ws + h->L.fields);
    int32_t rc = lb_fields(h, m, fld, fld + n, fld + 2 * n, fld + 3 * n);
    if (rc) return rc;
    // the paper's Eq. 14 and viscosity carry one tau: the mean of tau_A, tau_B
    const double tau = 0.5 * (mm.tau[0] + mm.tau[1]);
    BudgetConst K;
    K.cs2 = 1.0 / 3.0;
    K.gc = mm.G_AB * K.cs2 / 4.0;
    K.kappa = K.cs2 * K.cs2 * mm.G_AB / 4.0;
    K.c0 = K.cs2 * K.cs2;
    K.tf = (tau - 0.5) * (tau - 0.5);
    K.gA[0] = mm.g[0][0];
    K.gA[1] = mm.g[0][1];
    K.gB[0] = mm.g[1][0];
    K.gB[1] = mm.g[1][1];
    double *part = (double *)(h->ws + h->L.part);
    double *red = (double *)(h->ws + h->L.red);
    const int nb = (M.ny - 2 * h->cfg.diag_trim + BT_R - 1) / BT_R;   // bands of D rows (<= ny)
    hipLaunchKernelGGL(k_budget_rows, dim3(nb), dim3(RED_THREADS), 0, h->stream, (const double *)fld, M.nx, M.ny,
                       h->cfg.diag_trim, K, part);
    hipLaunchKernelGGL(k_sum_rows<BUDGET_NQ>, dim3(1), dim3(RED_THREADS), 0, h->stream, (const double *)part, nb, red);
    HIP_TRY(hipGetLastError());
    double host[BUDGET_NQ];
    HIP_TRY(hipMemcpyAsync(host, red, sizeof host, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const double nd = (double)M.nx * (double)(M.ny - 2 * h->cfg.diag_trim);
    out->t = h->t;
    out->pb = host[1] / nd;
    out->korteweg = host[2] / nd;
    out->ktau = host[3] / nd;
    const double rho_mean = host[0] / (double)n;
    out->eta = rho_mean * K.cs2 * (tau - 0.5);
    out->viscous = out->eta * (host[4] / nd);
    out->buoyancy = host[5] / nd;
    return LB_OK;
}

int32_t lb_interface_length(lb_handle *h, int32_t m, lb_interface *out)
{
    if (!is_live(h)) return fail(LB_ESTATE, "handle is not live");
    if (m < 0 || m >= (int32_t)h->dm.size()) return fail(LB_EINVAL, "member %d out of range", m);
    if (!out) return fail(LB_EINVAL, "out is NULL");
    const Member &M = h->dm[m];
    const int64_t n = (int64_t)M.nx * M.ny;
    double *fld = (double *)(h->ws + h->L.fields);
    int32_t rc = lb_fields(h, m, fld, fld + n, nullptr, nullptr);
    if (rc) return rc;
    double *part = (double *)(h->ws + h->L.part);
    double *red = (double *)(h->ws + h->L.red);
    const int nD = M.ny - 2 * h->cfg.diag_trim;
    hipLaunchKernelGGL(k_interface_rows, dim3(nD), dim3(RED_THREADS), 0, h->stream, (const double *)fld, M.nx, M.ny,
                       h->cfg.diag_trim, part);
    hipLaunchKernelGGL(k_sum_rows<IFACE_NQ>, dim3(1), dim3(RED_THREADS), 0, h->stream, (const double *)part, nD, red);
    HIP_TRY(hipGetLastError());
    double host[IFACE_NQ];
    HIP_TRY(hipMemcpyAsync(host, red, sizeof host, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    out->t = h->t;
    for (int q = 0; q < IFACE_NQ; ++q) out->crossings[q] = (int64_t)host[q];
    // Cauchy-Crofton: rows and columns are 1 apart, diagonals 1/sqrt(2)
    out->length = M_PI / 8.0 * ((double)(out->crossings[0] + out->crossings[1]) +
                                (double)(out->crossings[2] + out->crossings[3]) / std::sqrt(2.0));
    return LB_OK;
}

int32_t lb_components(lb_handle *h, int32_t m, lb_topology *out)
{
    if (!is_live(h)) return fail(LB_ESTATE, "handle is not live");
    if (m < 0 || m >= (int32_t)h->dm.size()) return fail(LB_EINVAL, "member %d out of range", m);
    if (!out) return fail(LB_EINVAL, "out is NULL");
    const Member &M = h->dm[m];
    const int64_t n = (int64_t)M.nx * M.ny;
    const int nD = M.ny - 2 * h->cfg.diag_trim;
    const int64_t nsites = (int64_t)nD * M.nx;
    double *fld = (double *)(h->ws + h->L.fields);
    // densities in the first half of the field buffer, the union-find
    // parents (4 B per site of D) in the velocity half
    int32_t rc = lb_fields(h, m, fld, fld + n, nullptr, nullptr);
    if (rc) return rc;
    int *parent = (int *)(fld + 2 * n);
    double *part = (double *)(h->ws + h->L.part);
    double *red = (double *)(h->ws + h->L.red);
    const unsigned grid = (unsigned)std::min<int64_t>((nsites + 255) / 256, 65536);
    hipLaunchKernelGGL(k_cc_init, dim3(grid), dim3(256), 0, h->stream, parent, nsites);
    hipLaunchKernelGGL(k_cc_hook, dim3(grid), dim3(256), 0, h->stream, (const double *)fld, M.nx, M.ny,
                       h->cfg.diag_trim, parent);
    hipLaunchKernelGGL(k_cc_compress, dim3(grid), dim3(256), 0, h->stream, parent, nsites);
    hipLaunchKernelGGL(k_cc_rows, dim3(nD), dim3(RED_THREADS), 0, h->stream, (const double *)fld, M.nx, M.ny,
                       h->cfg.diag_trim, (const int *)parent, part);
    hipLaunchKernelGGL(k_sum_rows<3>, dim3(1), dim3(RED_THREADS), 0, h->stream, (const double *)part, nD, red);
    HIP_TRY(hipGetLastError());
    double host[3];
    HIP_TRY(hipMemcpyAsync(host, red, sizeof host, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (host[2] != 0.0) return fail(LB_EINTERNAL, "component labelling left %.0f edges unjoined", host[2]);
    out->t = h->t;
    out->components[0] = (int64_t)host[0];
    out->components[1] = (int64_t)host[1];
    return LB_OK;
}

int32_t lb_get_populations(lb_handle *h, int32_t m, double *d_f)
{
    if (!is_live(h)) return fail(LB_ESTATE, "handle is not live");
    if (m < 0 || m >= (int32_t)h->dm.size()) return fail(LB_EINVAL, "member %d out of range", m);
    if (!d_f) return fail(LB_EINVAL, "d_f is NULL");
    const Member &M = h->dm[m];
    const int64_t n = (int64_t)M.nx * M.ny;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(pick_gather(h->cfg.storage, h->cfg.bc_y), dim3(grid), dim3(256), 0, h->stream,
                       (const Member *)dev_members(h), m, d_f, h->cur);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

int32_t lb_set_populations(lb_handle *h, int32_t m, const double *d_f)
{
    if (!is_live(h)) return fail(LB_ESTATE, "handle is not live");
    if (m < 0 || m >= (int32_t)h->dm.size()) return fail(LB_EINVAL, "member %d out of range", m);
    if (!d_f) return fail(LB_EINVAL, "d_f is NULL");
    const Member &M = h->dm[m];
    const int64_t n = (int64_t)M.nx * M.ny;
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(pick_scatter(h->cfg.storage, h->cfg.bc_y), dim3(grid), dim3(256), 0, h->stream,
                       (const Member *)dev_members(h), m, d_f, (const double *)nullptr, (const double *)nullptr, 0,
                       h->cur);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

int64_t lb_time(const lb_handle *h)
{
    if (!is_live(h)) {
        fail(LB_ESTATE, "handle is not live");
        return -1;
    }
    return h->t;
}

int32_t lb_tile_shape(const lb_handle *h, int32_t m, int32_t *tile_x, int32_t *tile_h)
{
    if (!is_live(h)) return fail(LB_ESTATE, "handle is not live");
    if (m < 0 || m >= (int32_t)h->dm.size()) return fail(LB_EINVAL, "member %d out of range", m);
    const int spp = h->steps_per_pass;
    if (tile_x) *tile_x = spp == 3 ? TX3 : (spp == 2 ? TX2 : h->tile_x);
    if (tile_h) *tile_h = spp == 3 ? h->dm[m].tile_h3 : (spp == 2 ? h->dm[m].tile_h2 : h->dm[m].tile_h);
    return LB_OK;
}

int32_t lb_steps_per_pass(const lb_handle *h)
{
    if (!is_live(h)) return fail(LB_ESTATE, "handle is not live");
    return h->steps_per_pass;
}

int32_t lb_tiles_cached(const lb_handle *h)
{
    if (!is_live(h)) return fail(LB_ESTATE, "handle is not live");
    return h->tiles_cached;
}

int32_t lb_storage_scale(const lb_handle *h, int32_t m, double *scale, double *weight)
{
    if (!is_live(h)) return fail(LB_ESTATE, "handle is not live");
    if (m < 0 || m >= (int32_t)h->dm.size()) return fail(LB_EINVAL, "member %d out of range", m);
    const bool site = site_shift(h->cfg.storage);
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < NQ; ++i) {
            if (scale) scale[s * NQ + i] = h->dm[m].scale[s][i];
            if (weight) weight[s * NQ + i] = site ? (double)(float)wgt(i) : 0.0;
        }
    return LB_OK;
}

int32_t lb_destroy(lb_handle *h)
{
    {
        std::lock_guard<std::mutex> lk(g_live_mu);
        if (!h || !g_live.count(h)) return fail(LB_ESTATE, "handle is not live");
        g_live.erase(h);
    }
    hipError_t e = hipStreamSynchronize(h->stream);
    free_graphs(h);
    if (h->capture) (void)hipStreamDestroy(h->capture);
    delete h;
    if (e != hipSuccess) return fail(LB_EHIP, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
    return LB_OK;
}

// ---------------------------------------------------------------------------
// lb_diagnostics_noalloc: the reductions of lb_diagnostics over caller fields,
// with the per-row partial sums and the results in a file-scope device array
// instead of a workspace.  Every GPU the library runs on holds one copy of
// the array until the process ends; calls on one GPU share it.

}  // extern "C"

namespace {

constexpr int64_t NOALLOC_PART = (int64_t)LB_NOALLOC_MAX_NY * RED_NQ;   // [ny][RED_NQ] row partials
constexpr int64_t NOALLOC_DOUBLES = NOALLOC_PART + RED_NQ + LB_NOALLOC_MAX_NY;   // + totals + row profile

__device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up once per
// device; the array's name is only a host-side stand-in).
int32_t scratch_on_current_device(double **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(LB_EINVAL, "device %d beyond %d", dev, NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        double *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LB_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LB_OK;
}

}  // namespace

extern "C" {

int32_t lb_diagnostics_noalloc(const double *d_rhoA, const double *d_rhoB, const double *d_ux, const double *d_uy,
                               int32_t nx, int32_t ny, int32_t trim, const double *g, void *hip_stream, lb_diag *out,
                               double *phi_profile)
{
    if (!d_rhoA || !d_rhoB || !d_ux || !d_uy) return fail(LB_EINVAL, "a field pointer is NULL");
    if (!g || !out) return fail(LB_EINVAL, "g or out is NULL");
    if (nx < 1 || ny < 3) return fail(LB_EINVAL, "nx = %d, ny = %d must be >= 1 and >= 3", nx, ny);
    if (ny > LB_NOALLOC_MAX_NY)
        return fail(LB_EINVAL, "ny = %d exceeds LB_NOALLOC_MAX_NY = %d (the fixed scratch holds that many rows)", ny,
                    LB_NOALLOC_MAX_NY);
    if (trim < 1 || ny <= 2 * trim) return fail(LB_EINVAL, "trim = %d must be >= 1 and leave rows of ny = %d", trim, ny);
    double *ptr = nullptr;
    int32_t rc = scratch_on_current_device(&ptr);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    double *part = ptr, *red = ptr + NOALLOC_PART;
    // every partial and result read below is written first by these kernels:
    // nothing needs to start at zero
    hipLaunchKernelGGL(k_reduce_rows, dim3(ny), dim3(RED_THREADS), 0, s, d_rhoA, d_rhoB, d_ux, d_uy, nx, ny, trim, g[0],
                       g[1], g[2], g[3], part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_THREADS), 0, s, (const double *)part, nx, ny, red,
                       red + RED_NQ);
    HIP_TRY(hipGetLastError());
    double host[RED_NQ];
    HIP_TRY(hipMemcpyAsync(host, red, sizeof host, hipMemcpyDeviceToHost, s));
    if (phi_profile)
        HIP_TRY(hipMemcpyAsync(phi_profile, red + RED_NQ, (size_t)ny * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double nd = (double)nx * (double)(ny - 2 * trim);
    out->t = 0;
    out->mass[0] = host[0];
    out->mass[1] = host[1];
    out->Ek = host[3] / nd;
    out->Ep = host[4] / nd;
    out->buoyancy = host[5] / nd;
    out->omega2 = host[6] / nd;
    out->umax = host[7];
    out->finite = host[8] == 0.0 ? 1 : 0;
    if (!out->finite) return fail(LB_ENONFINITE, "%.0f non-finite densities or velocities", host[8]);
    return LB_OK;
}

}  // extern "C"
