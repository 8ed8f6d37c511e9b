// Host side of liblbm: the C-ABI declared in include/lbm.h.
//
// Device layout of a context (one allocation, or a caller workspace):
//   buffer A | buffer B | flag | partial sums | staging
// Each population buffer holds every box in turn, each box as 41 q-blocks
// of N_box values ([q][s][z][y][x], x fastest). A step reads the current
// buffer and writes the other (ping-pong), so streaming never races.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/lbm.h"
#include "kernels_io.hpp"
#include "layout.hpp"
#include "step_launch.hpp"

using namespace lbm;

namespace {

constexpr uint64_t STAGING_MAX = 256ull << 20;  // bytes of the host<->device staging area

int elem_bytes(int storage)
{
    switch (storage) {
        case LBM_F64: return 8;
        case LBM_F32:
        case LBM_F32_SHIFT: return 4;
        case LBM_F16_SHIFT:
        case LBM_BF16_SHIFT: return 2;
        default: return 0;
    }
}

struct BoxDev {
    Geom g;
    double omega;
    uint64_t offset;  // element offset of this box in a population buffer
    uint64_t nodes;
    uint64_t node0;   // index of the box's first node in the context
    double* wall_dev = nullptr;  // device: the box's two walls, 41 deviations and the kind each
};

struct Layout {
    uint64_t elems = 0;      // elements per population buffer
    uint64_t buf_bytes = 0;  // bytes per population buffer (aligned)
    uint64_t flag_off = 0, partial_off = 0, staging_off = 0, staging_bytes = 0, total = 0;
    uint64_t table_off = 0;          // BatchBox per box
    uint64_t wall_off = 0;           // 2 x (41 + 1) doubles per box (kinetic walls)
    uint64_t tiles_off[NBLK] = {};   // (box, tile) pairs per block size
    uint64_t ntiles[NBLK] = {};
    uint64_t max_nodes = 0;
};

// In the flag area: the non-finite flag at byte 0, the device step counter
// of graph replays at byte COUNTER_OFF.
constexpr uint64_t COUNTER_OFF = 64;

// Kernel model (equilibrium in the low bits, MODEL_ENTROPIC) of validated flags.
uint32_t model_of(uint32_t flags)
{
    const uint32_t base = (flags & LBM_FLAG_ISOTHERMAL) ? uint32_t(MODEL_ISO)
                          : (flags & LBM_FLAG_SERIES_EQUILIBRIUM) ? uint32_t(MODEL_SERIES) : uint32_t(MODEL_E2);
    return base | ((flags & LBM_FLAG_ENTROPIC) ? uint32_t(MODEL_ENTROPIC) : 0u) |
           ((flags & LBM_FLAG_WALLS) ? uint32_t(MODEL_WALLS) : 0u);
}

int check_boxes(const lbm_box* boxes, int32_t nboxes, const lbm_opts* opts)
{
    if (!boxes || !opts || nboxes < 1) return LBM_E_ARG;
    const int eb = elem_bytes(opts->storage);
    if (eb == 0) return LBM_E_ARG;
    if (opts->tau_conv != LBM_TAU_LB && opts->tau_conv != LBM_TAU_PAPER) return LBM_E_ARG;
    if (opts->newton_iters < 0 || opts->newton_iters > 4) return LBM_E_ARG;
    if (opts->flags & ~uint32_t(LBM_FLAG_STOCHASTIC_ROUNDING | LBM_FLAG_ISOTHERMAL | LBM_FLAG_SERIES_EQUILIBRIUM |
                                LBM_FLAG_ENTROPIC | LBM_FLAG_WALLS))
        return LBM_E_ARG;
    if ((opts->flags & LBM_FLAG_WALLS) && (opts->flags & LBM_FLAG_SERIES_EQUILIBRIUM)) return LBM_E_UNSUPPORTED;
    if ((opts->flags & LBM_FLAG_ISOTHERMAL) && (opts->flags & LBM_FLAG_SERIES_EQUILIBRIUM)) return LBM_E_ARG;
    if ((opts->flags & LBM_FLAG_ENTROPIC) && (opts->flags & LBM_FLAG_SERIES_EQUILIBRIUM)) return LBM_E_ARG;
    if ((opts->flags & LBM_FLAG_STOCHASTIC_ROUNDING) &&
        !(opts->storage == LBM_F32 || opts->storage == LBM_F16_SHIFT || opts->storage == LBM_BF16_SHIFT))
        return LBM_E_ARG;
    if (!(opts->rho0 >= 0.0) || !std::isfinite(opts->rho0)) return LBM_E_ARG;
    if (opts->shift_exp != LBM_SHIFT_AUTO && (opts->shift_exp < -60 || opts->shift_exp > 60)) return LBM_E_ARG;
    uint64_t tiles = 0;
    for (int b = 0; b < nboxes; ++b) {
        const lbm_box& x = boxes[b];
        if (x.nx < 1 || x.ny < 1 || x.nz < 1 || x.reserved != 0) return LBM_E_ARG;
        const uint64_t nodes = 2ull * uint64_t(x.nx) * uint64_t(x.ny) * uint64_t(x.nz);
        // node ids and in-q-block byte offsets are 32-bit
        if (nodes >= (1ull << 32) || nodes * uint64_t(eb) > 0xffffffffull - (QPAD_16 + 256)) return LBM_E_ARG;
        if (!std::isfinite(x.tau)) return LBM_E_ARG;
        if ((opts->flags & LBM_FLAG_WALLS) && x.ny < 2) return LBM_E_ARG;
        if (opts->tau_conv == LBM_TAU_LB && !(x.tau > 0.5)) return LBM_E_ARG;
        if (opts->tau_conv == LBM_TAU_PAPER && !(x.tau > 0.0)) return LBM_E_ARG;
        tiles += (nodes + 127) / 128;
    }
    // the batched launch has one block per (box, 128-node tile)
    if (tiles >= (1ull << 31)) return LBM_E_ARG;
    return LBM_OK;
}

Layout plan(const lbm_box* boxes, int32_t nboxes, const lbm_opts* opts)
{
    Layout L;
    const int eb = elem_bytes(opts->storage);
    for (int b = 0; b < nboxes; ++b) {
        const uint64_t nodes = 2ull * uint64_t(boxes[b].nx) * boxes[b].ny * boxes[b].nz;
        L.elems += uint64_t(Q) * qstride(nodes, eb);
        L.max_nodes = std::max(L.max_nodes, nodes);
    }
    L.buf_bytes = align_up(L.elems * eb);
    L.flag_off = 2 * L.buf_bytes;
    L.table_off = L.flag_off + ALIGN;
    L.wall_off = L.table_off + align_up(uint64_t(nboxes) * sizeof(BatchBox));
    uint64_t off = L.wall_off + align_up(uint64_t(nboxes) * 2 * WALL_STRIDE * sizeof(double));
    for (int i = 0; i < NBLK; ++i) {
        for (int b = 0; b < nboxes; ++b) {
            const uint64_t nodes = 2ull * uint64_t(boxes[b].nx) * boxes[b].ny * boxes[b].nz;
            L.ntiles[i] += (nodes + BLK_SIZES[i] - 1) / BLK_SIZES[i];
        }
        L.tiles_off[i] = off;
        off += align_up(L.ntiles[i] * sizeof(uint2));
    }
    L.partial_off = off;
    // partial sums: up to TOTAL_BLOCKS blocks of 2*PROJ_FIELDS doubles, then the result
    L.staging_off = L.partial_off + align_up(uint64_t(TOTAL_BLOCKS + 1) * 2 * PROJ_FIELDS * sizeof(double));
    // staging holds chunks of FP64 node fields (5 per node) or populations
    const uint64_t want = std::max<uint64_t>(L.max_nodes * 8 * uint64_t(Q), 4096);
    L.staging_bytes = align_up(std::min(want, STAGING_MAX));
    L.total = L.staging_off + L.staging_bytes;
    return L;
}

}  // namespace

struct lbm_ctx {
    std::vector<BoxDev> boxes;
    int storage = 0;
    int newton = 1;
    int kamp = 0;
    double rho0 = 1.0;
    Layout L;
    char* mem = nullptr;
    bool own_mem = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int cur = 0;  // population buffer holding the current state
    StepParams base{};  // per-context part of the kernel parameters
    uint32_t* flag = nullptr;
    double* partials = nullptr;
    char* staging = nullptr;
    int variant = 0;
    double rho_ref_storage = 0.0;  // rho0 for shifted storage, else 0
    bool stochastic = false;       // stochastic rounding of the stored values
    uint32_t steps_done = 0;       // counter feeding the stochastic rounding
    int schedule = LBM_SCHEDULE_PER_BOX;
    int graph_steps = 0;           // 0: eager launches; else steps per captured graph
    BatchBox* table = nullptr;     // device: per-box parameters of the batched launch
    uint2* tiles[NBLK] = {};       // device: (box, tile) lists per block size
    uint32_t* step_ctr = nullptr;  // device: step base read by graph replays
    struct Graph {
        int cur;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;     // captured step sequences for the current tuning
    hipStream_t capture = nullptr; // private stream the graphs are captured on

    char* buf(int i) const { return mem + uint64_t(i) * L.buf_bytes; }
    StepParams params(const BoxDev& b) const
    {
        StepParams p = base;
        p.g = b.g;
        p.omega = b.omega;
        p.node0 = uint32_t(b.node0);
        p.wall_dev = b.wall_dev;
        p.step = steps_done;
        // the kernel's reference weights are the FP32-rounded ones
        for (int s = 0; s < 6; ++s)
            p.omw[s] = float(b.omega * double(float(SHELL_W[s])) * rho_ref_storage * double(p.scale[s]));
        return p;
    }
};

#define HIPCHK(expr)                                  \
    do {                                              \
        if ((expr) != hipSuccess) return LBM_E_HIP;   \
    } while (0)

namespace {

template <class F>
int dispatch_storage(int storage, F&& f)
{
    switch (storage) {
        case LBM_F64: return f(StoreF64{});
        case LBM_F32: return f(StoreF32{});
        case LBM_F16_SHIFT: return f(StoreF16S{});
        case LBM_BF16_SHIFT: return f(StoreBF16S{});
        case LBM_F32_SHIFT: return f(StoreF32S{});
        default: return LBM_E_ARG;
    }
}

uint32_t nblocks(uint64_t n) { return uint32_t((n + BLOCK - 1) / BLOCK); }

// Enqueue one step of every box from buffer `from` into the other buffer on
// stream s. The stochastic-rounding step is `step`, plus *step_base when
// step_base is not null (graph replays).
int enqueue_step(lbm_ctx* ctx, int from, uint32_t step, const uint32_t* step_base, hipStream_t s)
{
#if defined(LBM_HOST_CHECK)
    // host-code check build (the sanitizer on the host code, no device):
    // the step kernels are not built and a step is refused
    (void)ctx;
    (void)from;
    (void)step;
    (void)step_base;
    (void)s;
    return LBM_E_UNSUPPORTED;
#else
    StepLaunch L{};
    L.in = ctx->buf(from);
    L.out = ctx->buf(1 - from);
    L.newton = ctx->newton;
    L.schedule = ctx->schedule;
    L.variant = ctx->variant;
    L.model = ctx->base.model;
    L.xcd_remap = ctx->base.xcd_remap;
    L.step = step;
    L.step_base = step_base;
    L.stream = s;
    L.table = ctx->table;
    for (int i = 0; i < NBLK; ++i) {
        L.tiles[i] = ctx->tiles[i];
        L.ntiles[i] = ctx->L.ntiles[i];
    }
    std::vector<StepParams> params;
    std::vector<uint64_t> offset, nodes;
    if (ctx->schedule != LBM_SCHEDULE_BATCHED) {
        for (const BoxDev& b : ctx->boxes) {
            params.push_back(ctx->params(b));
            offset.push_back(b.offset);
            nodes.push_back(b.nodes);
        }
        L.nboxes = int(ctx->boxes.size());
        L.params = params.data();
        L.offset = offset.data();
        L.nodes = nodes.data();
    }
    // stochastic rounding exists for the FP32-arithmetic forms whose
    // rounding is coarse: FP32 of f, FP16 and BF16 of the shift
    const bool sr = ctx->stochastic;
    int rc;
    switch (ctx->storage) {
        case LBM_F64: rc = enqueue_step_f64(L); break;
        case LBM_F32: rc = sr ? enqueue_step_f32_sr(L) : enqueue_step_f32(L); break;
        case LBM_F32_SHIFT: rc = enqueue_step_f32s(L); break;
        case LBM_F16_SHIFT: rc = sr ? enqueue_step_f16s_sr(L) : enqueue_step_f16s(L); break;
        case LBM_BF16_SHIFT: rc = sr ? enqueue_step_bf16s_sr(L) : enqueue_step_bf16s(L); break;
        default: rc = LBM_E_ARG; break;
    }
    return rc;
#endif
}

// Device tables of the batched launch: per-box parameters and, per block
// size, the (box, tile) list. Called once the storage scales are final.
int upload_tables(lbm_ctx* ctx)
{
    std::vector<BatchBox> tab(ctx->boxes.size());
    for (size_t b = 0; b < ctx->boxes.size(); ++b) {
        tab[b].p = ctx->params(ctx->boxes[b]);
        tab[b].p.step = 0;
        tab[b].p.step_base = nullptr;
        tab[b].offset = ctx->boxes[b].offset;
    }
    HIPCHK(hipMemcpyAsync(ctx->table, tab.data(), tab.size() * sizeof(BatchBox), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < NBLK; ++i) {
        std::vector<uint2> t;
        t.reserve(ctx->L.ntiles[i]);
        for (size_t b = 0; b < ctx->boxes.size(); ++b) {
            const uint64_t nt = (ctx->boxes[b].nodes + BLK_SIZES[i] - 1) / BLK_SIZES[i];
            for (uint64_t k = 0; k < nt; ++k) t.push_back(make_uint2(uint32_t(b), uint32_t(k)));
        }
        if (t.size() != ctx->L.ntiles[i]) return LBM_E_ARG;
        HIPCHK(hipMemcpyAsync(ctx->tiles[i], t.data(), t.size() * sizeof(uint2), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return LBM_OK;
}

void drop_graphs(lbm_ctx* ctx)
{
    for (auto& g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
    ctx->graphs.clear();
}

// The executable graph of graph_steps steps starting from buffer ctx->cur
// (graph_steps is even, so a replay ends on the same buffer), captured on
// the private stream the first time it is asked for.
int graph_for(lbm_ctx* ctx, hipGraphExec_t* out)
{
    for (auto& g : ctx->graphs)
        if (g.cur == ctx->cur) {
            *out = g.exec;
            return LBM_OK;
        }
    if (!ctx->capture) HIPCHK(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
    int rc = LBM_OK;
    int from = ctx->cur;
    for (int i = 0; i < ctx->graph_steps && rc == LBM_OK; ++i) {
        rc = enqueue_step(ctx, from, uint32_t(i), ctx->step_ctr, ctx->capture);
        from ^= 1;
    }
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(ctx->capture, &graph);
    if (rc != LBM_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return rc != LBM_OK ? rc : LBM_E_HIP;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) return LBM_E_HIP;
    ctx->graphs.push_back({ctx->cur, exec});
    *out = exec;
    return LBM_OK;
}

// Run the init kernel over box b chunk by chunk. Host fields are copied
// through the staging area; device fields (device_fields) are read in place.
int run_init(lbm_ctx* ctx, const BoxDev& b, uint64_t node_base, const double* const fields[5], bool device_fields,
             int mode, float* maxdev)
{
    const uint64_t chunk = device_fields ? uint64_t(1) << 30 : ctx->L.staging_bytes / (5 * sizeof(double));
    double* stage = reinterpret_cast<double*>(ctx->staging);
    for (uint64_t n0 = 0; n0 < b.nodes; n0 += chunk) {
        const uint64_t cnt = std::min(chunk, b.nodes - n0);
        InitFields in;
        const double** dst[5] = {&in.rho, &in.ux, &in.uy, &in.uz, &in.th};
        for (int k = 0; k < 5; ++k) {
            if (device_fields) {
                *dst[k] = fields[k] + node_base + n0;
            } else {
                HIPCHK(hipMemcpyAsync(stage + k * cnt, fields[k] + node_base + n0, cnt * sizeof(double),
                                      hipMemcpyHostToDevice, ctx->stream));
                *dst[k] = stage + k * cnt;
            }
        }
        const StepParams p = ctx->params(b);
        int rc = dispatch_storage(ctx->storage, [&](auto st) {
            using ST = decltype(st);
            using T = typename ST::T;
            T* f = reinterpret_cast<T*>(ctx->buf(ctx->cur)) + b.offset;
            hipLaunchKernelGGL((k_init<ST>), dim3(nblocks(cnt)), dim3(BLOCK), 0, ctx->stream, f, b.g.qs,
                               uint32_t(n0), uint32_t(cnt), in, p, mode, maxdev);
            return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
        });
        if (rc) return rc;
        // the staging area is reused by the next chunk
        if (!device_fields) HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    // the caller reads the flag and the measured deviation next
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

void set_shift(lbm_ctx* ctx)
{
    for (int s = 0; s < 6; ++s) {
        const int k = ctx->storage == LBM_F32_SHIFT ? 0 : ctx->kamp + SHELL_K[s];
        ctx->base.scale[s] = std::ldexp(1.0f, k);
        ctx->base.inv_scale[s] = std::ldexp(1.0f, -k);
    }
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// Autotuner: times launch configurations of the step on the context's own
// boxes without changing the held state, and keeps the fastest.
// ---------------------------------------------------------------------------

// Tuning choices already made in this process (and optionally a file),
// keyed by what the step's speed depends on: the device architecture, the
// storage form, the kernel model, the rounding, the Newton count and the
// box shapes. Thread-safe.
class TuneCache {
public:
    bool find(const std::string& key, lbm_tuning* t)
    {
        std::lock_guard<std::mutex> g(mu_);
        auto it = map_.find(key);
        if (it == map_.end()) return false;
        *t = it->second;
        return true;
    }
    void insert(const std::string& key, const lbm_tuning& t)
    {
        std::lock_guard<std::mutex> g(mu_);
        map_[key] = t;
        if (!file_.empty()) {
            if (FILE* f = std::fopen(file_.c_str(), "a")) {
                std::fprintf(f, "%s %d %d %d %d\n", key.c_str(), t.variant, t.xcd_remap, t.schedule, t.graph_steps);
                std::fclose(f);
            }
        }
    }
    // Entries of the file are loaded (malformed lines are skipped); new
    // entries are appended to it. NULL: in-process only.
    int set_file(const char* path)
    {
        std::lock_guard<std::mutex> g(mu_);
        if (!path) {
            file_.clear();
            return LBM_OK;
        }
        FILE* f = std::fopen(path, "a+");
        if (!f) return LBM_E_ARG;
        std::rewind(f);
        // one entry per line: key and four integers; other lines are skipped
        char line[8192], key[4096], extra[2];
        lbm_tuning t;
        while (std::fgets(line, sizeof line, f)) {
            if (!std::strchr(line, '\n') && !std::feof(f)) {
                int c;  // over-long line: drop its remainder
                while ((c = std::fgetc(f)) != EOF && c != '\n') {
                }
                continue;
            }
            if (std::sscanf(line, "%4095s %d %d %d %d %1s", key, &t.variant, &t.xcd_remap, &t.schedule,
                            &t.graph_steps, extra) == 5 &&
                tuning_valid(t))
                map_[key] = t;
        }
        std::fclose(f);
        file_ = path;
        return LBM_OK;
    }
    void clear()
    {
        std::lock_guard<std::mutex> g(mu_);
        map_.clear();
    }
    int count()
    {
        std::lock_guard<std::mutex> g(mu_);
        return int(map_.size());
    }
    static bool tuning_valid(const lbm_tuning& t)
    {
        return t.variant >= 0 && t.variant < NVARIANTS && (t.xcd_remap == 0 || t.xcd_remap == 1) &&
               (t.schedule == LBM_SCHEDULE_PER_BOX || t.schedule == LBM_SCHEDULE_BATCHED) && t.graph_steps >= 0 &&
               t.graph_steps <= LBM_GRAPH_STEPS_MAX && t.graph_steps % 2 == 0;
    }

private:
    std::mutex mu_;
    std::map<std::string, lbm_tuning> map_;
    std::string file_;
};

TuneCache& tune_cache()
{
    static TuneCache c;
    return c;
}

// Cache key of a context: architecture, storage, model, rounding, Newton
// steps and the box shapes (listed for up to four boxes, else their count
// and a 64-bit FNV-1a hash of the shapes). No spaces.
int tune_key(lbm_ctx* ctx, uint32_t flags, std::string* key)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    char arch[64];
    std::snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
    for (char* c = arch; *c; ++c)
        if (*c == ' ' || *c == ':') *c = '_';
    char head[256];
    std::snprintf(head, sizeof(head), "%s|st%d|m%u|sr%d|nw%d|f%u|nb%zu", arch, ctx->storage, ctx->base.model,
                  ctx->stochastic ? 1 : 0, ctx->newton, flags & (LBM_TUNE_SCHEDULE | LBM_TUNE_GRAPH),
                  ctx->boxes.size());
    std::string k = head;
    if (ctx->boxes.size() <= 4) {
        for (const BoxDev& b : ctx->boxes) {
            char d[64];
            std::snprintf(d, sizeof(d), "|%ux%ux%u", b.g.nx, b.g.ny, b.g.nz);
            k += d;
        }
    } else {
        uint64_t h = 1469598103934665603ull;
        for (const BoxDev& b : ctx->boxes) {
            for (uint32_t v : {b.g.nx, b.g.ny, b.g.nz}) {
                for (int i = 0; i < 4; ++i) {
                    h ^= (v >> (8 * i)) & 0xffu;
                    h *= 1099511628211ull;
                }
            }
        }
        char d[32];
        std::snprintf(d, sizeof(d), "|h%016llx", static_cast<unsigned long long>(h));
        k += d;
    }
    *key = k;
    return LBM_OK;
}

// Mean time per step of one launch configuration: `reps` steps (after one
// untimed step), or for graph_steps G > 0 whole replays of a captured
// graph of G steps (at least `reps` steps). Every timed launch reads the
// current buffer and writes the other one: the held state is unchanged.
int time_config(lbm_ctx* ctx, const lbm_tuning& t, int32_t reps, hipEvent_t e0, hipEvent_t e1, float* ms)
{
    const int sv = ctx->variant, ss = ctx->schedule;
    const uint32_t sx = ctx->base.xcd_remap;
    ctx->variant = t.variant;
    ctx->base.xcd_remap = uint32_t(t.xcd_remap);
    ctx->schedule = t.schedule;
    int rc = LBM_OK;
    float el = 0.f;
    int steps = 0;
    if (t.graph_steps == 0) {
        for (int r = -1; r < reps && rc == LBM_OK; ++r) {
            if (r == 0 && hipEventRecord(e0, ctx->stream) != hipSuccess) rc = LBM_E_HIP;
            if (rc == LBM_OK) rc = enqueue_step(ctx, ctx->cur, ctx->steps_done, nullptr, ctx->stream);
        }
        steps = reps;
    } else {
        if (!ctx->capture && hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking) != hipSuccess)
            rc = LBM_E_HIP;
        hipGraphExec_t exec = nullptr;
        if (rc == LBM_OK && hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
            rc = LBM_E_HIP;
        if (rc == LBM_OK) {
            int crc = LBM_OK;
            for (int i = 0; i < t.graph_steps && crc == LBM_OK; ++i)
                crc = enqueue_step(ctx, ctx->cur, uint32_t(i), ctx->step_ctr, ctx->capture);
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(ctx->capture, &graph);
            if (crc == LBM_OK && e == hipSuccess && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
                crc = LBM_E_HIP;
            if (graph) (void)hipGraphDestroy(graph);
            if (e != hipSuccess) crc = LBM_E_HIP;
            rc = crc;
            (void)hipGetLastError();
        }
        const int replays = std::max(1, (reps + t.graph_steps - 1) / t.graph_steps);
        for (int r = -1; r < replays && rc == LBM_OK; ++r) {
            if (r == 0 && hipEventRecord(e0, ctx->stream) != hipSuccess) rc = LBM_E_HIP;
            if (rc == LBM_OK && hipGraphLaunch(exec, ctx->stream) != hipSuccess) rc = LBM_E_HIP;
        }
        steps = replays * t.graph_steps;
        if (rc == LBM_OK && hipEventRecord(e1, ctx->stream) != hipSuccess) rc = LBM_E_HIP;
        if (rc == LBM_OK && hipEventSynchronize(e1) != hipSuccess) rc = LBM_E_HIP;
        if (rc == LBM_OK && hipEventElapsedTime(&el, e0, e1) != hipSuccess) rc = LBM_E_HIP;
        if (exec) {
            (void)hipStreamSynchronize(ctx->stream);
            (void)hipGraphExecDestroy(exec);
        }
        ctx->variant = sv;
        ctx->base.xcd_remap = sx;
        ctx->schedule = ss;
        if (rc == LBM_OK) *ms = el / float(steps);
        return rc;
    }
    if (rc == LBM_OK && hipEventRecord(e1, ctx->stream) != hipSuccess) rc = LBM_E_HIP;
    if (rc == LBM_OK && hipEventSynchronize(e1) != hipSuccess) rc = LBM_E_HIP;
    if (rc == LBM_OK && hipEventElapsedTime(&el, e0, e1) != hipSuccess) rc = LBM_E_HIP;
    ctx->variant = sv;
    ctx->base.xcd_remap = sx;
    ctx->schedule = ss;
    if (rc == LBM_OK) *ms = el / float(steps);
    return rc;
}

// Timing noise below which configurations count as tied (relative).
constexpr float TUNE_TIE = 0.005f;
// graph_steps candidates besides eager launches.
constexpr int TUNE_GRAPH_STEPS[] = {16, 64};

// The search: every (variant, XCD remap) pair with the context's schedule,
// eager, in three interleaved rounds (each configuration keeps its fastest
// round); then, on request, the schedule and graph_steps with the chosen
// pair. Among configurations within TUNE_TIE of the fastest, the one with
// the XCD remap on is preferred (it moves no more than the algorithmic HBM
// bytes), then eager launches. The choice is applied to the context.
int autotune_impl(lbm_ctx* ctx, int32_t reps, uint32_t flags, float* ms, lbm_tune_result* res)
{
    if (!ctx || reps < 1) return LBM_E_ARG;
    std::string key;
    if (flags & LBM_TUNE_CACHE) {
        int rc = tune_key(ctx, flags, &key);
        if (rc) return rc;
        lbm_tuning t;
        if (tune_cache().find(key, &t)) {
            rc = lbm_set_tuning(ctx, &t);
            if (rc) return rc;
            res->best = t;
            res->best_ms = 0.f;
            res->from_cache = 1;
            res->timed = 0;
            if (ms)
                for (int k = 0; k < 2 * NVARIANTS; ++k) ms[k] = 0.f;
            return LBM_OK;
        }
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return LBM_E_HIP;
    }
    // captured graphs of the old configuration are dropped when the choice
    // differs (lbm_set_tuning below); the stream is idle after timing
    int rc = LBM_OK;
    int timed = 0;
    constexpr int ROUNDS = 3;
    // variant x remap (the models other than E2 run one launch shape, so
    // only the remap is timed for them)
    const int nvar = ctx->base.model == MODEL_E2 ? NVARIANTS : 1;
    float tmin[2 * NVARIANTS];
    for (int k = 0; k < 2 * NVARIANTS; ++k) tmin[k] = 0.f;
    for (int round = 0; round < ROUNDS && rc == LBM_OK; ++round)
        for (int v = 0; v < nvar && rc == LBM_OK; ++v)
            for (int x = 0; x < 2 && rc == LBM_OK; ++x) {
                float t = 0.f;
                rc = time_config(ctx, lbm_tuning{v, x, ctx->schedule, 0}, reps, e0, e1, &t);
                if (rc == LBM_OK && (tmin[2 * v + x] == 0.f || t < tmin[2 * v + x])) tmin[2 * v + x] = t;
                ++timed;
            }
    lbm_tuning bt{ctx->variant, int32_t(ctx->base.xcd_remap), ctx->schedule, 0};
    float best_ms = 0.f;
    if (rc == LBM_OK) {
        for (int k = 0; k < 2 * nvar; ++k)
            if (best_ms == 0.f || tmin[k] < best_ms) best_ms = tmin[k];
        // ties (within noise) go to the remap, then to the lower index
        int pick = -1;
        for (int pass = 0; pass < 2 && pick < 0; ++pass)
            for (int k = 0; k < 2 * nvar && pick < 0; ++k)
                if ((pass == 1 || k % 2 == 1) && tmin[k] <= best_ms * (1.f + TUNE_TIE)) pick = k;
        bt.variant = pick / 2;
        bt.xcd_remap = pick % 2;
        best_ms = tmin[pick];
        if (ms)
            for (int k = 0; k < 2 * NVARIANTS; ++k) ms[k] = k < 2 * nvar ? tmin[k] : 0.f;
    }
    // schedule (only meaningful with several boxes)
    if (rc == LBM_OK && (flags & LBM_TUNE_SCHEDULE) && ctx->boxes.size() > 1) {
        float ts[2] = {0.f, 0.f};
        for (int round = 0; round < ROUNDS && rc == LBM_OK; ++round)
            for (int sc = 0; sc < 2 && rc == LBM_OK; ++sc) {
                float t = 0.f;
                rc = time_config(ctx, lbm_tuning{bt.variant, bt.xcd_remap, sc, 0}, reps, e0, e1, &t);
                if (rc == LBM_OK && (ts[sc] == 0.f || t < ts[sc])) ts[sc] = t;
                ++timed;
            }
        if (rc == LBM_OK) {
            // the current schedule unless the other is faster beyond noise
            const int other = 1 - bt.schedule;
            if (ts[other] < ts[bt.schedule] * (1.f - TUNE_TIE)) bt.schedule = other;
            best_ms = ts[bt.schedule];
        }
    }
    // graph replays of G steps against eager launches
    if (rc == LBM_OK && (flags & LBM_TUNE_GRAPH)) {
        constexpr int NG = int(sizeof(TUNE_GRAPH_STEPS) / sizeof(TUNE_GRAPH_STEPS[0]));
        float tg[NG + 1];
        for (int k = 0; k <= NG; ++k) tg[k] = 0.f;
        for (int round = 0; round < ROUNDS && rc == LBM_OK; ++round)
            for (int k = 0; k <= NG && rc == LBM_OK; ++k) {
                const int g = k == 0 ? 0 : TUNE_GRAPH_STEPS[k - 1];
                float t = 0.f;
                rc = time_config(ctx, lbm_tuning{bt.variant, bt.xcd_remap, bt.schedule, g}, reps, e0, e1, &t);
                if (rc == LBM_OK && (tg[k] == 0.f || t < tg[k])) tg[k] = t;
                ++timed;
            }
        if (rc == LBM_OK) {
            int pick = 0;
            for (int k = 1; k <= NG; ++k)
                if (tg[k] < tg[pick] * (1.f - TUNE_TIE)) pick = k;
            bt.graph_steps = pick == 0 ? 0 : TUNE_GRAPH_STEPS[pick - 1];
            best_ms = tg[pick];
        }
    } else {
        bt.graph_steps = ctx->graph_steps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LBM_OK) return rc;
    rc = lbm_set_tuning(ctx, &bt);
    if (rc) return rc;
    if (flags & LBM_TUNE_CACHE) tune_cache().insert(key, bt);
    res->best = bt;
    res->best_ms = best_ms;
    res->from_cache = 0;
    res->timed = timed;
    return LBM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of lbm_totals_noalloc: the per-block partial sums of its FP64
// totals live in this fixed device array (one copy per device, held until
// the process ends) instead of a context workspace.
// ---------------------------------------------------------------------------
namespace {
constexpr uint32_t NOALLOC_BLOCKS = TOTAL_BLOCKS;                 // partial-sum blocks
constexpr size_t SCRATCH_DOUBLES = size_t(NOALLOC_BLOCKS) * 5;   // 40 KiB
}  // namespace

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device (with that device current) and kept: in host code the array's
// name is not a device address.
int scratch_on_current_device(double** out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return LBM_E_UNSUPPORTED;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return LBM_E_HIP;
        }
        g_scratch[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch[dev];
    return LBM_OK;
}
}  // namespace

namespace {
template <typename R, int NEWTON>
void collide_host(double omega, int model, const double* in, double* out)
{
    CollideConst<R> cc;
    cc.om = R(omega);
    cc.rho_ref = R(1);
    for (int s = 0; s < 6; ++s) {
        cc.inv_scale[s] = R(1);
        cc.omw[s] = cc.om * R(SHELL_W[s]);
    }
    R x[Q], y[Q], rho, theta;
    for (int q = 0; q < Q; ++q) x[q] = R(in[q]);
    switch (model) {
        case MODEL_ISO: collide<R, false, NEWTON, MODEL_ISO>(x, y, cc, rho, theta); break;
        case MODEL_SERIES: collide<R, false, NEWTON, MODEL_SERIES>(x, y, cc, rho, theta); break;
        case MODEL_E2 | MODEL_ENTROPIC: collide<R, false, NEWTON, MODEL_E2 | MODEL_ENTROPIC>(x, y, cc, rho, theta); break;
        case MODEL_ISO | MODEL_ENTROPIC:
            collide<R, false, NEWTON, MODEL_ISO | MODEL_ENTROPIC>(x, y, cc, rho, theta);
            break;
        default: collide<R, false, NEWTON, MODEL_E2>(x, y, cc, rho, theta); break;
    }
    for (int q = 0; q < Q; ++q)
        out[q] = DEV_IN_PLACE<R> ? double(R((x[q] + R(SHELL_W[VEL[q].shell])) + y[q]))  // x holds f - w
                                 : double(R(x[q] + y[q]));
}
}  // namespace


extern "C" {

int lbm_lattice(double* c, double* w, double* theta0)
{
    for (int q = 0; q < Q; ++q) {
        if (c) {
            c[3 * q + 0] = 0.5 * VEL[q].x;
            c[3 * q + 1] = 0.5 * VEL[q].y;
            c[3 * q + 2] = 0.5 * VEL[q].z;
        }
        if (w) w[q] = SHELL_W[VEL[q].shell];
    }
    if (theta0) *theta0 = THETA0;
    return LBM_OK;
}

int lbm_workspace_size(const lbm_box* boxes, int32_t nboxes, const lbm_opts* opts, uint64_t* bytes)
{
    if (!bytes) return LBM_E_ARG;
    int rc = check_boxes(boxes, nboxes, opts);
    if (rc) return rc;
    *bytes = plan(boxes, nboxes, opts).total;
    return LBM_OK;
}

static int init_impl(lbm_ctx** out, const lbm_box* boxes, int32_t nboxes, const lbm_opts* opts, const double* rho,
                     const double* ux, const double* uy, const double* uz, const double* theta, bool device_fields,
                     void* stream, void* workspace, uint64_t workspace_bytes)
{
    if (!out) return LBM_E_ARG;
    *out = nullptr;
    int rc = check_boxes(boxes, nboxes, opts);
    if (rc) return rc;
    if (!rho || !ux || !uy || !uz || !theta) return LBM_E_ARG;

    lbm_ctx* ctx = new (std::nothrow) lbm_ctx();
    if (!ctx) return LBM_E_NOMEM;
    ctx->storage = opts->storage;
    ctx->newton = opts->newton_iters ? opts->newton_iters : (opts->storage == LBM_F64 ? 3 : 1);
    ctx->rho0 = opts->rho0 > 0 ? opts->rho0 : 1.0;
    ctx->L = plan(boxes, nboxes, opts);
    ctx->stochastic = (opts->flags & LBM_FLAG_STOCHASTIC_ROUNDING) != 0;
    const bool shifted = opts->storage == LBM_F16_SHIFT || opts->storage == LBM_BF16_SHIFT ||
                         opts->storage == LBM_F32_SHIFT;

    uint64_t off = 0, node0 = 0;
    for (int b = 0; b < nboxes; ++b) {
        BoxDev d;
        d.g = make_geom(uint32_t(boxes[b].nx), uint32_t(boxes[b].ny), uint32_t(boxes[b].nz));
        d.nodes = d.g.N;
        d.g.qs = qstride(d.nodes, elem_bytes(opts->storage));
        d.offset = off;
        d.node0 = node0;
        off += uint64_t(Q) * d.g.qs;
        node0 += d.nodes;
        d.omega = opts->tau_conv == LBM_TAU_LB ? 1.0 / boxes[b].tau : 2.0 / (2.0 * boxes[b].tau + 1.0);
        ctx->boxes.push_back(d);
    }

    // domain check of host fields before any device work (device fields are
    // checked by the init kernel, which raises the flag read below)
    const uint64_t total = device_fields ? 0 : node0;
    for (uint64_t i = 0; i < total; ++i) {
        if (!(rho[i] > 0.0) || !(theta[i] > 0.0) || !std::isfinite(rho[i]) || !std::isfinite(theta[i]) ||
            !std::isfinite(ux[i]) || !std::isfinite(uy[i]) || !std::isfinite(uz[i])) {
            delete ctx;
            return LBM_E_DOMAIN;
        }
    }

    auto fail = [&](int code) {
        lbm_free(ctx);
        return code;
    };

    if (stream) {
        ctx->stream = reinterpret_cast<hipStream_t>(stream);
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) return fail(LBM_E_HIP);
        ctx->own_stream = true;
    }
    if (workspace) {
        if (workspace_bytes < ctx->L.total || (reinterpret_cast<uintptr_t>(workspace) % ALIGN) != 0)
            return fail(LBM_E_NOMEM);
        ctx->mem = reinterpret_cast<char*>(workspace);
    } else {
        hipError_t e = hipMalloc(reinterpret_cast<void**>(&ctx->mem), ctx->L.total);
        if (e != hipSuccess) {
            ctx->mem = nullptr;
            (void)hipGetLastError();
            return fail(e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation ? LBM_E_NOMEM : LBM_E_HIP);
        }
        ctx->own_mem = true;
    }
    ctx->flag = reinterpret_cast<uint32_t*>(ctx->mem + ctx->L.flag_off);
    ctx->step_ctr = reinterpret_cast<uint32_t*>(ctx->mem + ctx->L.flag_off + COUNTER_OFF);
    ctx->table = reinterpret_cast<BatchBox*>(ctx->mem + ctx->L.table_off);
    for (size_t b = 0; b < ctx->boxes.size(); ++b)
        ctx->boxes[b].wall_dev = reinterpret_cast<double*>(ctx->mem + ctx->L.wall_off) + b * 2 * WALL_STRIDE;
    for (int i = 0; i < NBLK; ++i) ctx->tiles[i] = reinterpret_cast<uint2*>(ctx->mem + ctx->L.tiles_off[i]);
    ctx->schedule = nboxes > 1 ? LBM_SCHEDULE_BATCHED : LBM_SCHEDULE_PER_BOX;
    ctx->partials = reinterpret_cast<double*>(ctx->mem + ctx->L.partial_off);
    ctx->staging = ctx->mem + ctx->L.staging_off;

    ctx->base.flag = ctx->flag;
    ctx->base.xcd_remap = 1;
    ctx->base.model = model_of(opts->flags);
    ctx->base.seed = opts->seed;
    ctx->base.rho_ref = shifted ? ctx->rho0 : 0.0;
    ctx->rho_ref_storage = ctx->base.rho_ref;
    double e2 = 0.0;  // sum_q w_q c_q^2 rho_ref
    for (int q = 0; q < Q; ++q)
        e2 += SHELL_W[VEL[q].shell] * 0.25 * (VEL[q].x * VEL[q].x + VEL[q].y * VEL[q].y + VEL[q].z * VEL[q].z);
    ctx->base.e2_ref = shifted ? e2 * ctx->rho0 : 0.0;
    ctx->kamp = 0;
    set_shift(ctx);

    if (hipMemsetAsync(ctx->flag, 0, ALIGN, ctx->stream) != hipSuccess) return fail(LBM_E_HIP);
    // kinetic walls start at rest at theta0: their equilibrium is w_q
    if (hipMemsetAsync(ctx->mem + ctx->L.wall_off, 0, ctx->boxes.size() * 2 * WALL_STRIDE * sizeof(double),
                       ctx->stream) != hipSuccess)
        return fail(LBM_E_HIP);
    const double* fields[5] = {rho, ux, uy, uz, theta};

    if (shifted && ctx->storage != LBM_F32_SHIFT) {
        if (opts->shift_exp == LBM_SHIFT_AUTO) {
            // largest |f - w rho0| 2^k_shell of the initial state, then k_amp
            // so that it becomes about 2^10 (FP16 max is 65504: ~64x headroom)
            float* maxdev = reinterpret_cast<float*>(ctx->partials);
            if (hipMemsetAsync(maxdev, 0, sizeof(float), ctx->stream) != hipSuccess) return fail(LBM_E_HIP);
            uint64_t base = 0;
            for (const BoxDev& b : ctx->boxes) {
                rc = run_init(ctx, b, base, fields, device_fields, 0, maxdev);
                if (rc) return fail(rc);
                base += b.nodes;
            }
            float m = 0.f;
            if (hipMemcpy(&m, maxdev, sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) return fail(LBM_E_HIP);
            int k = 10;
            if (m > 0.f && std::isfinite(m)) k = int(std::floor(std::log2(1024.0 / double(m))));
            ctx->kamp = std::max(-40, std::min(40, k));
        } else {
            ctx->kamp = opts->shift_exp;
        }
        set_shift(ctx);
    }

    uint64_t base = 0;
    for (const BoxDev& b : ctx->boxes) {
        rc = run_init(ctx, b, base, fields, device_fields, 1, nullptr);
        if (rc) return fail(rc);
        base += b.nodes;
    }
    uint32_t flag = 0;
    if (hipMemcpy(&flag, ctx->flag, sizeof(flag), hipMemcpyDeviceToHost) != hipSuccess) return fail(LBM_E_HIP);
    if (flag) return fail(LBM_E_DOMAIN);
    rc = upload_tables(ctx);
    if (rc) return fail(rc);
    *out = ctx;
    return LBM_OK;
}

int lbm_init(lbm_ctx** out, const lbm_box* boxes, int32_t nboxes, const lbm_opts* opts, const double* rho,
             const double* ux, const double* uy, const double* uz, const double* theta, void* stream,
             void* workspace, uint64_t workspace_bytes)
{
    return init_impl(out, boxes, nboxes, opts, rho, ux, uy, uz, theta, false, stream, workspace, workspace_bytes);
}

int lbm_init_device(lbm_ctx** out, const lbm_box* boxes, int32_t nboxes, const lbm_opts* opts, const double* rho,
                    const double* ux, const double* uy, const double* uz, const double* theta, void* stream,
                    void* workspace, uint64_t workspace_bytes)
{
    return init_impl(out, boxes, nboxes, opts, rho, ux, uy, uz, theta, true, stream, workspace, workspace_bytes);
}

int lbm_step(lbm_ctx* ctx, int32_t n)
{
    if (!ctx || n < 0) return LBM_E_ARG;
    // whole graphs first (each ends on the buffer it started from), then
    // the remaining steps as eager launches
    while (ctx->graph_steps > 0 && n >= ctx->graph_steps) {
        hipGraphExec_t exec = nullptr;
        int rc = graph_for(ctx, &exec);
        if (rc) return rc;
        hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, ctx->stream, ctx->step_ctr, ctx->steps_done);
        HIPCHK(hipGetLastError());
        HIPCHK(hipGraphLaunch(exec, ctx->stream));
        ctx->steps_done += uint32_t(ctx->graph_steps);
        n -= ctx->graph_steps;
    }
    for (int32_t i = 0; i < n; ++i) {
        int rc = enqueue_step(ctx, ctx->cur, ctx->steps_done, nullptr, ctx->stream);
        if (rc) return rc;
        ctx->cur ^= 1;
        ++ctx->steps_done;
    }
    return LBM_OK;
}

int lbm_stream_free(lbm_ctx* ctx, int32_t n)
{
    if (!ctx || n < 0) return LBM_E_ARG;
    if (ctx->base.model & MODEL_WALLS) return LBM_E_UNSUPPORTED;
#if defined(LBM_HOST_CHECK)
    return n == 0 ? LBM_OK : LBM_E_UNSUPPORTED;
#else
    // the launch shape of the energy-conserving step: the context's variant
    // and tile mapping (other models run 256 threads without hints)
    const int v = ctx->base.model == MODEL_E2 ? ctx->variant : 0;
    for (int32_t i = 0; i < n; ++i) {
        const int eb = elem_bytes(ctx->storage);
        int rc = LBM_OK;
        auto launch = [&](auto tag, auto blk, auto fl) {
            using T = decltype(tag);
            constexpr int BLK = decltype(blk)::value;
            constexpr int FL = decltype(fl)::value;
            const T* in = reinterpret_cast<const T*>(ctx->buf(ctx->cur));
            T* out = reinterpret_cast<T*>(ctx->buf(1 - ctx->cur));
            for (const BoxDev& b : ctx->boxes) {
                const StepParams p = ctx->params(b);
                hipLaunchKernelGGL((k_stream_free<T, BLK, FL>), dim3(uint32_t((b.nodes + BLK - 1) / BLK)), dim3(BLK), 0,
                                   ctx->stream, in + b.offset, out + b.offset, p);
            }
        };
        auto by_type = [&](auto blk, auto fl) {
            if (eb == 8) launch(double{}, blk, fl);
            else if (eb == 4) launch(float{}, blk, fl);
            else launch(uint16_t{}, blk, fl);
        };
        using std::integral_constant;
        switch (v) {
            case 0: by_type(integral_constant<int, 256>{}, integral_constant<int, 0>{}); break;
            case 1: by_type(integral_constant<int, 256>{}, integral_constant<int, FL_NT_LOAD | FL_NT_STORE>{}); break;
            case 2: by_type(integral_constant<int, 512>{}, integral_constant<int, 0>{}); break;
            case 3: by_type(integral_constant<int, 128>{}, integral_constant<int, 0>{}); break;
            case 4: by_type(integral_constant<int, 256>{}, integral_constant<int, FL_NT_STORE>{}); break;
            case 5: by_type(integral_constant<int, 1024>{}, integral_constant<int, 0>{}); break;
            case 6: by_type(integral_constant<int, 256>{}, integral_constant<int, 0>{}); break;  // plain pulls
            default: rc = LBM_E_ARG; break;
        }
        if (rc) return rc;
        HIPCHK(hipGetLastError());
        ctx->cur ^= 1;
    }
    return LBM_OK;
#endif
}

int lbm_device_copy(const void* src, void* dst, uint64_t bytes, void* stream)
{
    const uintptr_t s = reinterpret_cast<uintptr_t>(src), d = reinterpret_cast<uintptr_t>(dst);
    if (!src || !dst || bytes % 16 != 0 || (s | d) % 16 != 0) return LBM_E_ARG;
    if (bytes == 0) return LBM_OK;
    if (s < d + bytes && d < s + bytes) return LBM_E_ARG;  // overlapping ranges
    const uint64_t n = bytes / 16;
    const uint64_t blocks = (n + BLOCK - 1) / BLOCK;
    if (blocks > 0x7fffffffull) return LBM_E_ARG;
    hipLaunchKernelGGL(k_copy16, dim3(uint32_t(blocks)), dim3(BLOCK), 0, static_cast<hipStream_t>(stream),
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), n);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
}

int lbm_synchronize(lbm_ctx* ctx)
{
    if (!ctx) return LBM_E_ARG;
    return hipStreamSynchronize(ctx->stream) == hipSuccess ? LBM_OK : LBM_E_HIP;
}

int lbm_moments(lbm_ctx* ctx, double* rho, double* jx, double* jy, double* jz, double* energy)
{
    if (!ctx) return LBM_E_ARG;
    double* outs[5] = {rho, jx, jy, jz, energy};
    const uint64_t chunk = ctx->L.staging_bytes / (5 * sizeof(double));
    double* stage = reinterpret_cast<double*>(ctx->staging);
    uint64_t base = 0;
    for (const BoxDev& b : ctx->boxes) {
        const StepParams p = ctx->params(b);
        for (uint64_t n0 = 0; n0 < b.nodes; n0 += chunk) {
            const uint64_t cnt = std::min(chunk, b.nodes - n0);
            int rc = dispatch_storage(ctx->storage, [&](auto st) {
                using ST = decltype(st);
                using T = typename ST::T;
                const T* f = reinterpret_cast<const T*>(ctx->buf(ctx->cur)) + b.offset;
                hipLaunchKernelGGL((k_moments<ST>), dim3(nblocks(cnt)), dim3(BLOCK), 0, ctx->stream, f,
                                   b.g.qs, uint32_t(n0), uint32_t(cnt), p, stage);
                return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
            });
            if (rc) return rc;
            for (int k = 0; k < 5; ++k)
                if (outs[k])
                    HIPCHK(hipMemcpyAsync(outs[k] + base + n0, stage + k * cnt, cnt * sizeof(double),
                                          hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
        }
        base += b.nodes;
    }
    return LBM_OK;
}

int lbm_status(lbm_ctx* ctx)
{
    if (!ctx) return LBM_E_ARG;
    uint32_t flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, ctx->flag, sizeof(flag), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return flag ? LBM_E_NONFINITE : LBM_OK;
}

int lbm_totals(lbm_ctx* ctx, double* out)
{
    if (!ctx || !out) return LBM_E_ARG;
    double* res = ctx->partials + TOTAL_BLOCKS * 2 * PROJ_FIELDS;
    for (size_t bi = 0; bi < ctx->boxes.size(); ++bi) {
        const BoxDev& b = ctx->boxes[bi];
        const StepParams p = ctx->params(b);
        const uint32_t nblk = std::min<uint32_t>(TOTAL_BLOCKS, nblocks(b.nodes));
        int rc = dispatch_storage(ctx->storage, [&](auto st) {
            using ST = decltype(st);
            using T = typename ST::T;
            const T* f = reinterpret_cast<const T*>(ctx->buf(ctx->cur)) + b.offset;
            hipLaunchKernelGGL((k_totals<ST>), dim3(nblk), dim3(BLOCK), 0, ctx->stream, f, uint32_t(b.nodes), p,
                               ctx->partials, uint32_t(ctx->stochastic));
            hipLaunchKernelGGL(k_reduce_partials<5>, dim3(1), dim3(BLOCK), 0, ctx->stream, ctx->partials, nblk, res);
            return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
        });
        if (rc) return rc;
        HIPCHK(hipMemcpyAsync(out + 5 * bi, res, 5 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return lbm_status(ctx);
}

int lbm_totals_noalloc(const void* f, int32_t storage, const lbm_box* box, uint64_t qstride, double rho0,
                       int32_t shift_exp, void* stream, double* out)
{
    if (!f || !box || !out) return LBM_E_ARG;
    const int eb = elem_bytes(storage);
    if (eb == 0) return LBM_E_ARG;
    if (box->nx < 1 || box->ny < 1 || box->nz < 1) return LBM_E_ARG;
    const uint64_t nodes = 2ull * uint64_t(box->nx) * uint64_t(box->ny) * uint64_t(box->nz);
    // the largest box: 32-bit node ids and q-block strides
    if (nodes >= (1ull << 32) || qstride < nodes || qstride >= (1ull << 32)) return LBM_E_ARG;
    const bool shifted = storage == LBM_F16_SHIFT || storage == LBM_BF16_SHIFT || storage == LBM_F32_SHIFT;
    if (!(rho0 >= 0.0) || !std::isfinite(rho0)) return LBM_E_ARG;
    if (rho0 == 0.0) rho0 = 1.0;
    if ((storage == LBM_F16_SHIFT || storage == LBM_BF16_SHIFT) && (shift_exp < -60 || shift_exp > 60))
        return LBM_E_ARG;
    StepParams p{};
    p.g = make_geom(uint32_t(box->nx), uint32_t(box->ny), uint32_t(box->nz));
    p.g.qs = uint32_t(qstride);
    for (int sh = 0; sh < 6; ++sh) {
        const int k = storage == LBM_F32_SHIFT ? 0 : shift_exp + SHELL_K[sh];
        p.scale[sh] = std::ldexp(1.0f, k);
        p.inv_scale[sh] = std::ldexp(1.0f, -k);
    }
    double e2 = 0.0;  // sum_q w_q c_q^2 / 2 per unit reference density
    for (int q = 0; q < Q; ++q)
        e2 += SHELL_W[VEL[q].shell] * 0.25 * (VEL[q].x * VEL[q].x + VEL[q].y * VEL[q].y + VEL[q].z * VEL[q].z);
    p.rho_ref = shifted ? rho0 : 0.0;
    p.e2_ref = shifted ? e2 * rho0 : 0.0;
    double* part = nullptr;
    int rc = scratch_on_current_device(&part);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const uint32_t nblk = std::min<uint32_t>(NOALLOC_BLOCKS, nblocks(nodes));
    return dispatch_storage(storage, [&](auto st) {
        using ST = decltype(st);
        using T = typename ST::T;
        // every partial the reduction reads is written by k_totals first
        hipLaunchKernelGGL((k_totals<ST>), dim3(nblk), dim3(BLOCK), 0, s, reinterpret_cast<const T*>(f),
                           uint32_t(nodes), p, part, 0u);
        hipLaunchKernelGGL(k_reduce_partials<5>, dim3(1), dim3(BLOCK), 0, s, part, nblk, out);
        return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
    });
}

int lbm_project(lbm_ctx* ctx, int32_t box, const double* k, double* out)
{
    if (!ctx || !k || !out || box < 0 || box >= int32_t(ctx->boxes.size())) return LBM_E_ARG;
    const BoxDev& b = ctx->boxes[box];
    const StepParams p = ctx->params(b);
    const uint32_t nblk = std::min<uint32_t>(TOTAL_BLOCKS, nblocks(b.nodes));
    double* res = ctx->partials + TOTAL_BLOCKS * 2 * PROJ_FIELDS;
    int rc = dispatch_storage(ctx->storage, [&](auto st) {
        using ST = decltype(st);
        using T = typename ST::T;
        const T* f = reinterpret_cast<const T*>(ctx->buf(ctx->cur)) + b.offset;
        hipLaunchKernelGGL((k_project<ST>), dim3(nblk), dim3(BLOCK), 0, ctx->stream, f, p, k[0], k[1], k[2],
                           ctx->partials);
        hipLaunchKernelGGL(k_reduce_partials<2 * PROJ_FIELDS>, dim3(1), dim3(BLOCK), 0, ctx->stream, ctx->partials,
                           nblk, res);
        return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
    });
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(out, res, 2 * PROJ_FIELDS * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < 2 * PROJ_FIELDS; ++i) out[i] /= double(b.nodes);
    return LBM_OK;
}

int lbm_get_populations(lbm_ctx* ctx, double* f)
{
    if (!ctx || !f) return LBM_E_ARG;
    const uint64_t chunk = ctx->L.staging_bytes / sizeof(double);
    double* stage = reinterpret_cast<double*>(ctx->staging);
    uint64_t host_off = 0;
    for (const BoxDev& b : ctx->boxes) {
        for (int q = 0; q < Q; ++q) {
            const int sh = VEL[q].shell;
            for (uint64_t n0 = 0; n0 < b.nodes; n0 += chunk) {
                const uint64_t cnt = std::min(chunk, b.nodes - n0);
                int rc = dispatch_storage(ctx->storage, [&](auto st) {
                    using ST = decltype(st);
                    using T = typename ST::T;
                    const T* fq = reinterpret_cast<const T*>(ctx->buf(ctx->cur)) + b.offset + uint64_t(q) * b.g.qs + n0;
                    hipLaunchKernelGGL((k_get<ST>), dim3(nblocks(cnt)), dim3(BLOCK), 0, ctx->stream, fq,
                                       uint32_t(cnt), ctx->base.inv_scale[sh], SHELL_W[sh] * ctx->base.rho_ref, stage);
                    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
                });
                if (rc) return rc;
                HIPCHK(hipMemcpyAsync(f + host_off + uint64_t(q) * b.nodes + n0, stage, cnt * sizeof(double),
                                      hipMemcpyDeviceToHost, ctx->stream));
                HIPCHK(hipStreamSynchronize(ctx->stream));
            }
        }
        host_off += uint64_t(Q) * b.nodes;
    }
    return LBM_OK;
}

int lbm_set_populations(lbm_ctx* ctx, const double* f)
{
    if (!ctx || !f) return LBM_E_ARG;
    const uint64_t chunk = ctx->L.staging_bytes / sizeof(double);
    double* stage = reinterpret_cast<double*>(ctx->staging);
    uint64_t host_off = 0;
    for (const BoxDev& b : ctx->boxes) {
        for (int q = 0; q < Q; ++q) {
            const int sh = VEL[q].shell;
            for (uint64_t n0 = 0; n0 < b.nodes; n0 += chunk) {
                const uint64_t cnt = std::min(chunk, b.nodes - n0);
                HIPCHK(hipMemcpyAsync(stage, f + host_off + uint64_t(q) * b.nodes + n0, cnt * sizeof(double),
                                      hipMemcpyHostToDevice, ctx->stream));
                int rc = dispatch_storage(ctx->storage, [&](auto st) {
                    using ST = decltype(st);
                    using T = typename ST::T;
                    T* fq = reinterpret_cast<T*>(ctx->buf(ctx->cur)) + b.offset + uint64_t(q) * b.g.qs + n0;
                    hipLaunchKernelGGL((k_set<ST>), dim3(nblocks(cnt)), dim3(BLOCK), 0, ctx->stream, fq,
                                       uint32_t(cnt), ctx->base.scale[sh], SHELL_W[sh] * ctx->base.rho_ref, stage);
                    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
                });
                if (rc) return rc;
                HIPCHK(hipStreamSynchronize(ctx->stream));
            }
        }
        host_off += uint64_t(Q) * b.nodes;
    }
    return LBM_OK;
}

int lbm_gather(lbm_ctx* ctx, int32_t box, const int64_t* idx, int64_t count, double* out)
{
    if (!ctx || box < 0 || box >= int32_t(ctx->boxes.size()) || count < 0) return LBM_E_ARG;
    if (count == 0) return LBM_OK;
    if (!idx || !out) return LBM_E_ARG;
    const BoxDev& b = ctx->boxes[box];
    const int64_t lim = int64_t(Q) * int64_t(b.nodes);
    for (int64_t i = 0; i < count; ++i)
        if (idx[i] < 0 || idx[i] >= lim) return LBM_E_ARG;
    const uint64_t chunk = ctx->L.staging_bytes / (2 * sizeof(double));
    int64_t* sidx = reinterpret_cast<int64_t*>(ctx->staging);
    double* sout = reinterpret_cast<double*>(ctx->staging + chunk * sizeof(int64_t));
    const StepParams p = ctx->params(b);
    for (int64_t i0 = 0; i0 < count; i0 += int64_t(chunk)) {
        const uint64_t cnt = std::min<uint64_t>(chunk, uint64_t(count - i0));
        HIPCHK(hipMemcpyAsync(sidx, idx + i0, cnt * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
        int rc = dispatch_storage(ctx->storage, [&](auto st) {
            using ST = decltype(st);
            using T = typename ST::T;
            const T* f = reinterpret_cast<const T*>(ctx->buf(ctx->cur)) + b.offset;
            hipLaunchKernelGGL((k_gather<ST>), dim3(nblocks(cnt)), dim3(BLOCK), 0, ctx->stream, f, uint32_t(b.nodes),
                               sidx, uint32_t(cnt), p, sout);
            return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_HIP;
        });
        if (rc) return rc;
        HIPCHK(hipMemcpyAsync(out + i0, sout, cnt * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return LBM_OK;
}

int lbm_debug_pull_map(lbm_ctx* ctx, int32_t box, int64_t* src)
{
    if (!ctx || !src || box < 0 || box >= int32_t(ctx->boxes.size())) return LBM_E_ARG;
    const BoxDev& b = ctx->boxes[box];
    const uint64_t chunk = ctx->L.staging_bytes / (uint64_t(Q) * sizeof(int64_t));
    int64_t* stage = reinterpret_cast<int64_t*>(ctx->staging);
    for (uint64_t n0 = 0; n0 < b.nodes; n0 += chunk) {
        const uint64_t cnt = std::min(chunk, b.nodes - n0);
        hipLaunchKernelGGL(k_pull_map, dim3(nblocks(cnt)), dim3(BLOCK), 0, ctx->stream, b.g, uint32_t(n0),
                           uint32_t(cnt), stage);
        HIPCHK(hipGetLastError());
        for (int q = 0; q < Q; ++q)
            HIPCHK(hipMemcpyAsync(src + uint64_t(q) * b.nodes + n0, stage + uint64_t(q) * cnt, cnt * sizeof(int64_t),
                                  hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return LBM_OK;
}

int lbm_set_step_counter(lbm_ctx* ctx, uint32_t steps_done)
{
    if (!ctx) return LBM_E_ARG;
    ctx->steps_done = steps_done;
    return LBM_OK;
}

int lbm_get_info(lbm_ctx* ctx, lbm_info* info)
{
    if (!ctx || !info) return LBM_E_ARG;
    std::memset(info, 0, sizeof(*info));
    info->storage = ctx->storage;
    info->newton_iters = ctx->newton;
    info->shift_exp = (ctx->storage == LBM_F16_SHIFT || ctx->storage == LBM_BF16_SHIFT) ? ctx->kamp : 0;
    const uint32_t base = ctx->base.model & MODEL_BASE_MASK;
    info->flags = (ctx->stochastic ? LBM_FLAG_STOCHASTIC_ROUNDING : 0u) |
                  (base == MODEL_ISO ? LBM_FLAG_ISOTHERMAL : 0u) |
                  (base == MODEL_SERIES ? LBM_FLAG_SERIES_EQUILIBRIUM : 0u) |
                  ((ctx->base.model & MODEL_ENTROPIC) ? LBM_FLAG_ENTROPIC : 0u) |
                  ((ctx->base.model & MODEL_WALLS) ? LBM_FLAG_WALLS : 0u);
    info->steps_done = ctx->steps_done;
    info->nboxes = int32_t(ctx->boxes.size());
    uint64_t nodes = 0;
    for (const BoxDev& b : ctx->boxes) nodes += b.nodes;
    info->nodes = int64_t(nodes);
    info->bytes_per_step = int64_t(2 * uint64_t(Q) * nodes * uint64_t(elem_bytes(ctx->storage)));
    info->block_threads = ctx->base.model != MODEL_E2 ? 256 : VARIANTS[ctx->variant].blk;
    info->variant = ctx->variant;
    info->device_bytes = ctx->L.total;
    return LBM_OK;
}

int lbm_num_variants(void) { return NVARIANTS; }

int lbm_variant_desc(int32_t variant, int32_t* block_threads, uint32_t* flags)
{
    if (variant < 0 || variant >= NVARIANTS) return LBM_E_ARG;
    if (block_threads) *block_threads = VARIANTS[variant].blk;
    if (flags) *flags = uint32_t(VARIANTS[variant].fl);
    return LBM_OK;
}

int lbm_set_tuning(lbm_ctx* ctx, const lbm_tuning* t)
{
    if (!ctx || !t || t->variant < 0 || t->variant >= NVARIANTS || (t->xcd_remap != 0 && t->xcd_remap != 1) ||
        (t->schedule != LBM_SCHEDULE_PER_BOX && t->schedule != LBM_SCHEDULE_BATCHED) || t->graph_steps < 0 ||
        t->graph_steps > LBM_GRAPH_STEPS_MAX || (t->graph_steps % 2) != 0)
        return LBM_E_ARG;
    if (t->variant != ctx->variant || uint32_t(t->xcd_remap) != ctx->base.xcd_remap ||
        t->schedule != ctx->schedule || t->graph_steps != ctx->graph_steps) {
        // captured graphs hold the old launch configuration
        if (!ctx->graphs.empty()) HIPCHK(hipStreamSynchronize(ctx->stream));
        drop_graphs(ctx);
    }
    ctx->variant = t->variant;
    ctx->base.xcd_remap = uint32_t(t->xcd_remap);
    ctx->schedule = t->schedule;
    ctx->graph_steps = t->graph_steps;
    return LBM_OK;
}

int lbm_get_tuning(lbm_ctx* ctx, lbm_tuning* t)
{
    if (!ctx || !t) return LBM_E_ARG;
    t->variant = ctx->variant;
    t->xcd_remap = int32_t(ctx->base.xcd_remap);
    t->schedule = ctx->schedule;
    t->graph_steps = ctx->graph_steps;
    return LBM_OK;
}

int lbm_autotune(lbm_ctx* ctx, int32_t reps, float* ms, lbm_tuning* best)
{
    lbm_tune_result r{};
    const int rc = autotune_impl(ctx, reps, 0u, ms, &r);
    if (rc == LBM_OK && best) *best = r.best;
    return rc;
}

int lbm_autotune_ex(lbm_ctx* ctx, int32_t reps, uint32_t flags, float* ms, lbm_tune_result* res)
{
    if (flags & ~uint32_t(LBM_TUNE_SCHEDULE | LBM_TUNE_GRAPH | LBM_TUNE_CACHE)) return LBM_E_ARG;
    lbm_tune_result r{};
    const int rc = autotune_impl(ctx, reps, flags, ms, &r);
    if (rc == LBM_OK && res) *res = r;
    return rc;
}

int lbm_tune_cache_file(const char* path) { return tune_cache().set_file(path); }

int lbm_tune_cache_clear(void)
{
    tune_cache().clear();
    return LBM_OK;
}

int lbm_tune_cache_count(void) { return tune_cache().count(); }

void* lbm_stream(lbm_ctx* ctx) { return ctx ? reinterpret_cast<void*>(ctx->stream) : nullptr; }

void lbm_free(lbm_ctx* ctx)
{
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    drop_graphs(ctx);
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    if (ctx->own_mem && ctx->mem) (void)hipFree(ctx->mem);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char* lbm_strerror(int code)
{
    switch (code) {
        case LBM_OK: return "ok";
        case LBM_E_ARG: return "invalid argument";
        case LBM_E_NOMEM: return "out of memory (or workspace too small)";
        case LBM_E_DOMAIN: return "unrealisable input state (rho <= 0, theta <= 0 or non-finite)";
        case LBM_E_NONFINITE: return "a step produced a non-finite or unrealisable node";
        case LBM_E_HIP: return "HIP runtime error";
        case LBM_E_UNSUPPORTED: return "unsupported request";
        default: return "unknown error";
    }
}

int lbm_set_walls_kind(lbm_ctx* ctx, int32_t box, const double* wall, const int32_t* kind)
{
    if (!ctx || !wall || !kind || box < 0 || box >= int32_t(ctx->boxes.size())) return LBM_E_ARG;
    if (!(ctx->base.model & MODEL_WALLS)) return LBM_E_ARG;
    if ((kind[0] != LBM_WALL_DIFFUSE && kind[0] != LBM_WALL_SPECULAR) ||
        (kind[1] != LBM_WALL_DIFFUSE && kind[1] != LBM_WALL_SPECULAR))
        return LBM_E_ARG;
    const int model = int(ctx->base.model & MODEL_BASE_MASK);
    double dev[2 * WALL_STRIDE];
    for (int w = 0; w < 2; ++w) {
        const double* u = wall + 4 * w;
        for (int k = 0; k < 4; ++k)
            if (!std::isfinite(u[k])) return LBM_E_DOMAIN;
        if (model != MODEL_ISO && !(u[3] > 0.0)) return LBM_E_DOMAIN;
        // the wall's equilibrium at unit density, as deviations f_w,q / w_q - 1
        equilibrium_dev_f64(1.0, u[0], u[1], u[2], model == MODEL_ISO ? THETA0 : u[3], 1.0, model,
                            dev + w * WALL_STRIDE);
        for (int q = 0; q < Q; ++q)
            if (!(dev[w * WALL_STRIDE + q] > -1.0) || !std::isfinite(dev[w * WALL_STRIDE + q])) return LBM_E_DOMAIN;
        dev[w * WALL_STRIDE + Q] = kind[w] == LBM_WALL_SPECULAR ? 1.0 : 0.0;
    }
    HIPCHK(hipMemcpyAsync(ctx->boxes[box].wall_dev, dev, sizeof(dev), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return LBM_OK;
}

int lbm_set_walls(lbm_ctx* ctx, int32_t box, const double* wall)
{
    const int32_t diffuse[2] = {LBM_WALL_DIFFUSE, LBM_WALL_DIFFUSE};
    return lbm_set_walls_kind(ctx, box, wall, diffuse);
}

int lbm_collide_host(int32_t precision, int32_t newton, uint32_t flags, double omega, const double* f_in,
                     double* f_out)
{
    if (!f_in || !f_out || (precision != 0 && precision != 1) || newton < 0 || newton > 4 ||
        (flags & ~uint32_t(LBM_FLAG_ISOTHERMAL | LBM_FLAG_SERIES_EQUILIBRIUM | LBM_FLAG_ENTROPIC)) ||
        ((flags & LBM_FLAG_ISOTHERMAL) && (flags & LBM_FLAG_SERIES_EQUILIBRIUM)) ||
        ((flags & LBM_FLAG_ENTROPIC) && (flags & LBM_FLAG_SERIES_EQUILIBRIUM)))
        return LBM_E_ARG;
    const int iso = int(model_of(flags));
    if (precision == 0) {
        switch (newton) {
            case 0: collide_host<double, 0>(omega, iso, f_in, f_out); break;
            case 1: collide_host<double, 1>(omega, iso, f_in, f_out); break;
            case 2: collide_host<double, 2>(omega, iso, f_in, f_out); break;
            case 3: collide_host<double, 3>(omega, iso, f_in, f_out); break;
            default: collide_host<double, 4>(omega, iso, f_in, f_out); break;
        }
    } else {
        switch (newton) {
            case 0: collide_host<float, 0>(omega, iso, f_in, f_out); break;
            case 1: collide_host<float, 1>(omega, iso, f_in, f_out); break;
            case 2: collide_host<float, 2>(omega, iso, f_in, f_out); break;
            case 3: collide_host<float, 3>(omega, iso, f_in, f_out); break;
            default: collide_host<float, 4>(omega, iso, f_in, f_out); break;
        }
    }
    return LBM_OK;
}

int lbm_selftest(void)
{
    // division by invariant integers: all small divisors on a spread of n,
    // plus the extremes of the 32-bit range
    uint64_t state = 0x9e3779b97f4a7c15ull;
    for (uint32_t d = 1; d <= 4096; ++d) {
        const FastDiv f = make_fastdiv(d);
        for (int i = 0; i < 256; ++i) {
            state = state * 6364136223846793005ull + 1442695040888963407ull;
            const uint32_t n = i < 4 ? (i == 0 ? 0u : i == 1 ? 0xffffffffu : i == 2 ? d - 1 : d) : uint32_t(state >> 32);
            if (fdiv(n, f) != n / d) return LBM_E_ARG;
        }
    }
    for (uint32_t d : {1000003u, 1u << 20, (1u << 31) + 7u, 0xffffffffu}) {
        const FastDiv f = make_fastdiv(d);
        for (uint32_t n : {0u, d - 1, d, 2 * d - 1, 0xfffffffeu, 0xffffffffu})
            if (fdiv(n, f) != n / d) return LBM_E_ARG;
    }
    return LBM_OK;
}

}  // extern "C"
