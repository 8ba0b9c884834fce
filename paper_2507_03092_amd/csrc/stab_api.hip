// stab_api.hip -- host side of libstab: argument validation, compilation of an op stream into
// gate/noise segments and measurement layers, device buffers and the C ABI of include/stab.h.
//
// Execution order of one stream (the race-safe order of Fig. 2 of the paper): all gates and
// noise up to a measurement layer run in one segment kernel per 64-row band; a measurement
// layer then runs classify -> deterministic batch -> in-order random chain -> reset/record.
#include "stab_kernels.hip"
#include "stab_batch.hip"
#include "stab_commute.hip"
#include "stab.h"

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

using namespace stabdev;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

constexpr int kLdsBytes = 160 * 1024;     // LDS of one gfx950 compute unit
constexpr int kSegThreads = 1024;
constexpr int kRedWords = 16;
constexpr int kMaxShots = 65535;          // grid y dimension of the reset kernel
constexpr int kReplayThreads = 512;
constexpr int kReplayStatic = 512;        // bound on k_replay's static LDS
constexpr int kNumKernels = 10;           // timing ids (include/stab.h)

// 32-bit words of the segment kernel's LDS for one half-band (before the per-shot accumulators)
int seg_lds_words(int RS) { return 64 * (RS + 1) + kRedWords; }

int max_qubits_for_lds(int lds_bytes)
{
    // a staged half-band, 64 * (2*Wc + 1) + kRedWords 32-bit words, must fit
    const int words = lds_bytes / 4 - kRedWords;
    const int wc = (words / 64 - 1) / 2;
    // register-resident limits: column words per lane (deterministic wave), band words per lane
    // (chain analysis: 2 * wc <= 64 * kMaxBandsPerLane)
    return std::min(std::min(wc, 64 * kMaxWordsPerLane), 32 * kMaxBandsPerLane) * 64;
}

// STAB_REVERSE_BLOCKS set (and not "0") in the environment: kernels take their workgroups in
// reverse order, a check that results do not depend on the order in which work runs.
int reverse_blocks()
{
    const char* v = std::getenv("STAB_REVERSE_BLOCKS");
    return (v && v[0] && !(v[0] == '0' && v[1] == 0)) ? 1 : 0;
}

Geom make_geom(int n, int shots, int mode)
{
    Geom g{};
    g.rev = reverse_blocks();
    g.n = n;
    g.Wc = (n + 63) / 64;
    g.Wr = g.Wc;
    g.NR = 64 * g.Wr;
    g.RS = 2 * g.Wc;
    g.NB = 2 * g.Wr;
    g.B = shots;
    g.S = (mode == STAB_MODE_SHARED) ? 1 : shots;
    g.bpc = g.B / g.S;
    return g;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
    size_t tab, rs, rd, total;
};

Layout layout_of(const Geom& g)
{
    Layout L{};
    L.tab = 0;
    L.rs = align256(L.tab + (size_t)g.S * 2 * g.NR * g.RS * 8);
    L.rd = align256(L.rs + (size_t)g.S * g.NB * 8);
    L.total = align256(L.rd + (size_t)g.B * g.NB * 8);
    return L;
}

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    bool arena = false;   // carved from the static scratch array (never freed)
};

}  // namespace

struct stab_ctx {
    Geom g{};
    int mode = 0;
    uint64_t seed = 0, first_shot = 0, instr_counter = 0;
    hipStream_t stream = nullptr;
    uint64_t* tab = nullptr;
    uint64_t* rs = nullptr;
    uint64_t* rd = nullptr;
    bool poisoned = false;
    int max_lds = kLdsBytes;
    // stab_sample_noalloc and the server's shared lane: every buffer of the context (and of its
    // program) is carved from caller-owned scratch (arena != NULL), nothing is allocated or freed
    char* arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    int* d_err = nullptr;
    unsigned long long* d_counters = nullptr;
    DevBuf xcol, zcol, cls, obuf, events, record, packed, pend;
    DevBuf plog_p, plog_row, plog_rs, plog_rd, ran;   // pivot log of the random chain
    DevBuf plist, pcnt, povf;                        // pending targets with x in each pivot
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // per-kernel timing (stab_set_timing)
    bool timing = false;
    // captured launch sequence of the last program executed with graphs on, and its key
    bool graph_on = false;
    hipStream_t cap_stream = nullptr;   // capture happens here (the context's stream may be the null stream)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    uint64_t gkey[5] = {0, 0, 0, 0, 0};
    uint32_t tmask = 0;           // kernel ids timed (bit k = kernel k)
    std::vector<hipEvent_t> evpool;
    std::vector<int> evkind;      // kernel id of each recorded pair
    size_t evused = 0;            // events used in the current execution
    double kms[kNumKernels] = {0};
    unsigned long long klaunch[kNumKernels] = {0};
};

namespace {

struct SegPlan {
    int item_begin = 0, item_count = 0;
    int modifies = 0;
    int noise_begin = 0, noise_count = 0;
    int units = 0;
    int max_units = 0;     // largest noise instruction of the segment (units)
    long long ev_cap = 0;
    long long ev_global = 0;   // first event slot of the segment when the whole program is drawn at once
    int meas = -1;
    long long gate_count = 0;
};

struct MeasPlan {
    uint64_t instr;   // relative instruction index
    int kind;
    int pos_base;     // position of the first target within its instruction
    int tq_begin;
    int K;
    long long rec_off;
};

}  // namespace

struct stab_program {
    int ninstr = 0;
    long long nrec = 0;
    int Kmax = 0;
    long long ev_cap_max = 0;
    long long ev_total = 0;    // event slots of all segments
    int max_units = 0;         // largest noise instruction of the program (units)
    int nnoise = 0;
    std::vector<SegPlan> segs;
    std::vector<MeasPlan> meas;
    std::vector<std::pair<int, int>> steps;   // (0, segment) or (1, measurement layer)
    // device copies
    void* dev = nullptr;
    bool dev_arena = false;   // dev lies in the static scratch (stab_sample_noalloc)
    int4* d_items = nullptr;
    uint2* d_gates = nullptr;
    NoiseDesc* d_noise = nullptr;
    int* d_noise_tg = nullptr;
    int* d_unit_start = nullptr;
    int* d_ev_base = nullptr;
    int* d_ev_count = nullptr;
    long long* d_noise_seg = nullptr;   // per noise instruction: its segment's first event slot
    int* d_mran = nullptr;              // per measurement layer: a target ran (learning execution)
    // Per measurement layer, whether a target of it ran in an execution that started from
    // |0...0> (instruction counter 0).  x|z never depends on outcomes or Pauli noise, so this is
    // the same in every such execution: later ones skip the chain, the replay, the column
    // refresh and the second deterministic pass of the layers where nothing ran.
    std::vector<int> mran;
    bool mran_known = false;
    int* d_mtq = nullptr;
    // geometry it was compiled for
    int n = 0, B = 0;
    uint64_t serial = 0;   // distinct for every program of the process (keys captured graphs)
};

namespace {

// Carve `bytes` (256-byte aligned) from the context's static scratch; STAB_ERANGE past its end.
int arena_take(stab_ctx* ctx, size_t bytes, void** out)
{
    const size_t at = align256(ctx->arena_used);
    bytes = std::max<size_t>(align256(bytes), 256);
    if (at + bytes > ctx->arena_cap)
        return fail(STAB_ERANGE, "the workload needs more than the " + std::to_string(ctx->arena_cap) +
                                     " bytes of scratch given to the context");
    *out = ctx->arena + at;
    ctx->arena_used = at + bytes;
    return STAB_OK;
}

int ensure(DevBuf& b, size_t bytes);

int ensure(stab_ctx* ctx, DevBuf& b, size_t bytes)
{
    if (!ctx->arena) return ensure(b, bytes);
    if (bytes <= b.cap) return STAB_OK;
    // an outgrown piece of the scratch stays unused until the call ends
    void* p = nullptr;
    const int rc = arena_take(ctx, bytes, &p);
    if (rc) return rc;
    b.p = p;
    b.cap = bytes;
    b.arena = true;
    return STAB_OK;
}

// Grow b (device memory of its own) to at least `bytes`.
int ensure(DevBuf& b, size_t bytes)
{
    if (bytes <= b.cap) return STAB_OK;
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
    }
    bytes = std::max<size_t>(bytes, 256);
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
        b.p = nullptr;
        return fail(STAB_ENOMEM, "device allocation failed");
    }
    b.cap = bytes;
    return STAB_OK;
}

#define HIP_CHECK(ctx, call)                                                                   \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            (ctx)->poisoned = true;                                                            \
            return fail(STAB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
        }                                                                                      \
    } while (0)

bool valid_kind(uint32_t k) { return k <= STAB_T1T2; }

// Timing brackets: tstart(kind) before a launch, tstop(kind) after it (no-ops unless that
// kernel id is timed).
int tstart(stab_ctx* ctx, int kind)
{
    if (!((ctx->tmask >> kind) & 1u)) return STAB_OK;
    if (ctx->evused + 2 > ctx->evpool.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            HIP_CHECK(ctx, hipEventCreate(&e));
            ctx->evpool.push_back(e);
        }
    }
    HIP_CHECK(ctx, hipEventRecord(ctx->evpool[ctx->evused], ctx->stream));
    return STAB_OK;
}

int tstop(stab_ctx* ctx, int kind)
{
    if (!((ctx->tmask >> kind) & 1u)) return STAB_OK;
    HIP_CHECK(ctx, hipEventRecord(ctx->evpool[ctx->evused + 1], ctx->stream));
    ctx->evkind.push_back(kind);
    ctx->evused += 2;
    return STAB_OK;
}

// After the stream has synchronized: add the recorded pairs to the totals.
int tcollect(stab_ctx* ctx)
{
    for (size_t i = 0; i < ctx->evkind.size(); ++i) {
        float ms = 0.f;
        HIP_CHECK(ctx, hipEventElapsedTime(&ms, ctx->evpool[2 * i], ctx->evpool[2 * i + 1]));
        ctx->kms[ctx->evkind[i]] += ms;
        ctx->klaunch[ctx->evkind[i]] += 1;
    }
    ctx->evkind.clear();
    ctx->evused = 0;
    return STAB_OK;
}

// The classify/product pass, the chain and the replay instantiated for the row's words per lane.
using DetFn = decltype(&k_det<1>);
static DetFn det_kernel(int Wc)
{
    const int wpl = (Wc + 63) / 64;
    return wpl <= 1 ? k_det<1> : wpl == 2 ? k_det<2> : wpl == 3 ? k_det<3> : k_det<4>;
}

using ChainFn = decltype(&k_chain<1>);
static ChainFn chain_kernel(int Wc)
{
    const int wpl = (Wc + 63) / 64;
    return wpl <= 1 ? k_chain<1> : wpl == 2 ? k_chain<2> : wpl == 3 ? k_chain<3> : k_chain<4>;
}

// The replay instantiated for the row's words per lane.
using ReplayFn = decltype(&k_replay<1>);
static ReplayFn replay_kernel(int Wc)
{
    const int wpl = (Wc + 63) / 64;
    return wpl <= 1 ? k_replay<1> : wpl == 2 ? k_replay<2> : wpl == 3 ? k_replay<3> : k_replay<4>;
}

#define TIMED(ctx, kind, launch)                 \
    do {                                         \
        int rc_ = tstart(ctx, kind);             \
        if (rc_) return rc_;                     \
        launch;                                  \
        HIP_CHECK(ctx, hipGetLastError());       \
        rc_ = tstop(ctx, kind);                  \
        if (rc_) return rc_;                     \
    } while (0)

// Split an op stream into segments (gate layers on disjoint qubits and noise layers) and
// measurement layers (disjoint qubits); see the file header.
int compile_stream(const Geom& g, const stab_instr* ins, int ninstr, const int32_t* tg,
                   int64_t ntg, stab_program& P, std::vector<int4>& items,
                   std::vector<uint2>& gates, std::vector<NoiseDesc>& noise,
                   std::vector<int>& noise_tg, std::vector<int>& unit_start,
                   std::vector<int>& ev_base, std::vector<int>& mtq)
{
    if (ninstr < 0 || ntg < 0) return fail(STAB_EINVAL, "negative count");
    if ((ninstr > 0 && !ins) || (ntg > 0 && !tg)) return fail(STAB_EINVAL, "null stream");
    const int n = g.n;
    // gate and noise targets are stored as the word index of the qubit's column in the segment
    // kernel's staged tile, (q mod 64) * (RS + 1) + q / 64
    const uint32_t RSP = (uint32_t)g.RS + 1u;
    auto tile_index = [&](int q) { return (uint32_t)(q & 63) * RSP + (uint32_t)(q >> 6); };
    std::vector<int> stamp(n, -1), mstamp(n, -1);
    int layer_id = 0, mlayer_id = 0;
    SegPlan seg;
    int open_begin = -1;
    long long rec_off = 0;

    auto close_layer = [&]() {
        if (open_begin >= 0) {
            const int cnt = (int)gates.size() - open_begin;
            if (cnt > 0) {
                items.push_back(make_int4(0, open_begin, cnt, -1));
                seg.item_count++;
                seg.gate_count += cnt;
            }
            open_begin = -1;
        }
        ++layer_id;
    };
    auto close_seg = [&](int meas_index) {
        close_layer();
        seg.meas = meas_index;
        P.steps.push_back({0, (int)P.segs.size()});
        P.ev_cap_max = std::max(P.ev_cap_max, seg.ev_cap);
        seg.ev_global = P.ev_total;
        P.ev_total += seg.ev_cap;
        P.max_units = std::max(P.max_units, seg.max_units);
        P.segs.push_back(seg);
        seg = SegPlan();
        seg.item_begin = (int)items.size();
        seg.noise_begin = (int)noise.size();
    };

    int64_t off = 0;
    for (int k = 0; k < ninstr; ++k) {
        const uint32_t kind = ins[k].kind, nt = ins[k].ntargets;
        if (!valid_kind(kind)) return fail(STAB_EINVAL, "instruction " + std::to_string(k) + ": unknown kind");
        if (off + (int64_t)nt > ntg) return fail(STAB_EINVAL, "instruction " + std::to_string(k) + ": targets run past the target array");
        if ((kind == STAB_CX || kind == STAB_DEP2) && (nt & 1u))
            return fail(STAB_EINVAL, "instruction " + std::to_string(k) + ": odd target count for a two-qubit kind");
        const int32_t* t = tg + off;
        for (uint32_t q = 0; q < nt; ++q)
            if (t[q] < 0 || t[q] >= n)
                return fail(STAB_EINVAL, "instruction " + std::to_string(k) + ": target " + std::to_string(t[q]) + " out of range");
        switch (kind) {
        case STAB_TICK:
            break;
        case STAB_T1T2:
            return fail(STAB_EINVAL, "instruction " + std::to_string(k) +
                                         ": T1T2 resets change x|z shot by shot; run it with stab_batch_*");
        case STAB_H: case STAB_S: case STAB_X: case STAB_Y: case STAB_Z:
            for (uint32_t q = 0; q < nt; ++q) {
                if (stamp[t[q]] == layer_id) close_layer();
                if (open_begin < 0) open_begin = (int)gates.size();
                stamp[t[q]] = layer_id;
                gates.push_back(make_uint2(kind | (tile_index(t[q]) << 4), 0u));
                if (kind == STAB_H || kind == STAB_S) seg.modifies = 1;
            }
            break;
        case STAB_CX:
            for (uint32_t q = 0; q < nt; q += 2) {
                const int c = t[q], d = t[q + 1];
                if (c == d) return fail(STAB_EINVAL, "instruction " + std::to_string(k) + ": CX with equal qubits");
                if (stamp[c] == layer_id || stamp[d] == layer_id) close_layer();
                if (open_begin < 0) open_begin = (int)gates.size();
                stamp[c] = stamp[d] = layer_id;
                gates.push_back(make_uint2(kind | (tile_index(c) << 4), tile_index(d)));
                seg.modifies = 1;
            }
            break;
        case STAB_DEP1: case STAB_DEP2: case STAB_PAULI1: {
            close_layer();
            const int units = (kind == STAB_DEP2) ? (int)nt / 2 : (int)nt;
            if (units == 0) break;
            NoiseDesc d{};
            d.instr = (uint64_t)k;
            d.t0 = ins[k].t0;
            d.t1 = ins[k].t1;
            d.t2 = ins[k].t2;
            d.kind = (int)kind;
            d.toff = (int)noise_tg.size();
            d.units = units;
            // noise layers with no gate between them act on the same tableau: they share one
            // event bucket (their events commute) and one item of the segment kernel
            const bool join = seg.item_count > 0 && items.back().x == 1;
            d.bucket = join ? items.back().w : (int)ev_base.size();
            for (uint32_t q = 0; q < nt; ++q) noise_tg.push_back((int)tile_index(t[q]));
            unit_start.push_back(seg.units);
            seg.units += units;
            seg.max_units = std::max(seg.max_units, units);
            if (!join) ev_base.push_back((int)seg.ev_cap);
            const long long cap = (long long)units * (kind == STAB_DEP2 ? 2 : 1) * g.B;
            seg.ev_cap += cap;
            if (seg.ev_cap > (1ll << 31) - 1) return fail(STAB_ERANGE, "too many noise locations in one segment");
            noise.push_back(d);
            seg.noise_count++;
            if (join) {
                items.back().z += (int)cap;
            } else {
                // {1, first event slot, event capacity, bucket}
                items.push_back(make_int4(1, ev_base.back(), (int)cap, d.bucket));
                seg.item_count++;
            }
        } break;
        case STAB_M: case STAB_MR: case STAB_R: {
            uint32_t q = 0;
            while (q < nt) {
                ++mlayer_id;
                const uint32_t begin = q;
                while (q < nt && mstamp[t[q]] != mlayer_id) mstamp[t[q++]] = mlayer_id;
                MeasPlan m{};
                m.instr = (uint64_t)k;
                m.kind = (int)kind;
                m.pos_base = (int)begin;
                m.tq_begin = (int)mtq.size();
                m.K = (int)(q - begin);
                m.rec_off = rec_off;
                mtq.insert(mtq.end(), t + begin, t + q);
                if (kind != STAB_R) rec_off += m.K;
                close_seg((int)P.meas.size());
                P.steps.push_back({1, (int)P.meas.size()});
                P.Kmax = std::max(P.Kmax, m.K);
                P.meas.push_back(m);
            }
        } break;
        default:
            return fail(STAB_EINVAL, "unknown kind");
        }
        off += nt;
    }
    if (off != ntg) return fail(STAB_EINVAL, "target array longer than the instructions consume");
    close_seg(-1);
    P.ninstr = ninstr;
    P.nrec = rec_off;
    P.nnoise = (int)noise.size();
    return STAB_OK;
}

template <typename T>
size_t put(std::vector<char>& blob, const std::vector<T>& v)
{
    const size_t at = align256(blob.size());
    blob.resize(at + std::max<size_t>(v.size() * sizeof(T), 1));
    if (!v.empty()) std::memcpy(blob.data() + at, v.data(), v.size() * sizeof(T));
    return at;
}

int launch_init(stab_ctx* ctx)
{
    const Geom& g = ctx->g;
    const size_t words = (size_t)g.S * 2 * g.NR * g.RS;
    const int blocks = (int)std::min<size_t>((words + 255) / 256, 65536);
    TIMED(ctx, 0, (k_init<<<blocks, 256, 0, ctx->stream>>>(g, ctx->tab, ctx->rs, ctx->rd)));
    HIP_CHECK(ctx, hipMemsetAsync(ctx->d_err, 0, sizeof(int), ctx->stream));
    return STAB_OK;
}

}  // namespace

// =============================================================================================
// C ABI
// =============================================================================================
extern "C" {

const char* stab_last_error(void) { return g_err.c_str(); }

int32_t stab_max_qubits(void) { return max_qubits_for_lds(kLdsBytes); }

int stab_tableau_bytes(int32_t n, int32_t shots, int32_t mode, uint64_t* bytes_out)
{
    if (!bytes_out) return fail(STAB_EINVAL, "bytes_out is NULL");
    if (n < 1 || shots < 1) return fail(STAB_EINVAL, "n and shots must be >= 1");
    if (shots > kMaxShots) return fail(STAB_ERANGE, "shots exceeds 65535");
    if (mode != STAB_MODE_SHARED && mode != STAB_MODE_FULL) return fail(STAB_EINVAL, "bad mode");
    if (n > stab_max_qubits()) return fail(STAB_ERANGE, "n exceeds stab_max_qubits()");
    *bytes_out = layout_of(make_geom(n, shots, mode)).total;
    return STAB_OK;
}

}  // extern "C"

namespace {

// stab_create; with arena != NULL the context's own device memory (error flag, counters and,
// later, every execution buffer) is carved from arena[0, arena_cap) and no event is created.
int create_ctx(int32_t n, int32_t shots, int32_t mode, uint64_t seed, uint64_t first_shot, void* dev_buf,
               uint64_t buf_bytes, void* hip_stream, char* arena, size_t arena_cap, stab_ctx** out,
               bool wait_init = true)
{
    if (!out) return fail(STAB_EINVAL, "out is NULL");
    *out = nullptr;
    uint64_t need = 0;
    int rc = stab_tableau_bytes(n, shots, mode, &need);
    if (rc) return rc;
    if (!dev_buf) return fail(STAB_EINVAL, "dev_buf is NULL");
    if (((uintptr_t)dev_buf & 255u) != 0) return fail(STAB_EINVAL, "dev_buf must be 256-byte aligned");
    if (buf_bytes < need) return fail(STAB_ENOMEM, "dev_buf smaller than stab_tableau_bytes()");

    stab_ctx* ctx = new stab_ctx();
    ctx->g = make_geom(n, shots, mode);
    ctx->mode = mode;
    ctx->seed = seed;
    ctx->first_shot = first_shot;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->arena = arena;
    ctx->arena_cap = arena ? arena_cap : 0;
    const Layout L = layout_of(ctx->g);
    char* base = (char*)dev_buf;
    ctx->tab = (uint64_t*)(base + L.tab);
    ctx->rs = (uint64_t*)(base + L.rs);
    ctx->rd = (uint64_t*)(base + L.rd);

    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        delete ctx;
        return fail(STAB_EDEVICE, "no HIP device");
    }
    ctx->max_lds = lds;
    const int seg_bytes = seg_lds_words(ctx->g.RS) * 4;
    if (seg_bytes > lds) {
        delete ctx;
        return fail(STAB_ERANGE, "a half-band of the tableau does not fit in this device's LDS");
    }
    (void)hipFuncSetAttribute((const void*)k_segment, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_chain<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_chain<2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_chain<3>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_chain<4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_det<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_det<2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_det<3>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_det<4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_replay<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_replay<2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_replay<3>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_replay<4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipGetLastError();

    const size_t counter_bytes = kNumCounters * kCounterStripes * sizeof(unsigned long long);
    if (arena) {
        if ((rc = arena_take(ctx, sizeof(int), (void**)&ctx->d_err)) ||
            (rc = arena_take(ctx, counter_bytes, (void**)&ctx->d_counters))) {
            delete ctx;
            return rc;
        }
    } else {
        bool ok = hipMalloc((void**)&ctx->d_err, sizeof(int)) == hipSuccess &&
                  hipMalloc((void**)&ctx->d_counters, counter_bytes) == hipSuccess &&
                  hipEventCreate(&ctx->ev0) == hipSuccess && hipEventCreate(&ctx->ev1) == hipSuccess;
        if (!ok) {
            stab_destroy(ctx);
            return fail(STAB_ENOMEM, "device allocation failed");
        }
    }
    if (hipMemsetAsync(ctx->d_counters, 0, counter_bytes, ctx->stream) != hipSuccess) {
        stab_destroy(ctx);
        return fail(STAB_EDEVICE, "memset failed");
    }
    rc = launch_init(ctx);
    if (rc == STAB_OK && wait_init && hipStreamSynchronize(ctx->stream) != hipSuccess)
        rc = fail(STAB_EDEVICE, "init failed");
    if (rc) {
        stab_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return STAB_OK;
}

}  // namespace

extern "C" {

int stab_create(int32_t n, int32_t shots, int32_t mode, uint64_t seed, uint64_t first_shot,
                void* dev_buf, uint64_t buf_bytes, void* hip_stream, stab_ctx** out)
{
    return create_ctx(n, shots, mode, seed, first_shot, dev_buf, buf_bytes, hip_stream, nullptr, 0, out);
}

void stab_destroy(stab_ctx* ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    DevBuf* bufs[] = {&ctx->xcol, &ctx->zcol, &ctx->cls, &ctx->obuf,
                      &ctx->events, &ctx->record, &ctx->packed, &ctx->pend, &ctx->plog_p,
                      &ctx->plog_row, &ctx->plog_rs, &ctx->plog_rd, &ctx->ran, &ctx->plist,
                      &ctx->pcnt, &ctx->povf};
    for (DevBuf* b : bufs)
        if (b->p && !b->arena) (void)hipFree(b->p);
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (!ctx->arena) {
        if (ctx->d_err) (void)hipFree(ctx->d_err);
        if (ctx->d_counters) (void)hipFree(ctx->d_counters);
    }
    for (hipEvent_t e : ctx->evpool) (void)hipEventDestroy(e);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    delete ctx;
}

int stab_set_rng(stab_ctx* ctx, uint64_t seed, uint64_t first_shot)
{
    if (!ctx) return fail(STAB_EINVAL, "ctx is NULL");
    if (ctx->poisoned) return fail(STAB_EDEVICE, "context poisoned by an earlier device error");
    ctx->seed = seed;
    ctx->first_shot = first_shot;
    return STAB_OK;
}

int stab_reset(stab_ctx* ctx, uint64_t seed, uint64_t first_shot)
{
    if (!ctx) return fail(STAB_EINVAL, "ctx is NULL");
    if (ctx->poisoned) return fail(STAB_EDEVICE, "context poisoned by an earlier device error");
    ctx->seed = seed;
    ctx->first_shot = first_shot;
    ctx->instr_counter = 0;
    int rc = launch_init(ctx);
    if (rc) return rc;
    HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->timing && (rc = tcollect(ctx))) return rc;
    return STAB_OK;
}

}  // extern "C"

namespace {

// Byte offsets of the device arrays of a program inside its uploaded blob.
struct ProgramBlob {
    std::vector<char> bytes;
    size_t items, gates, noise, ntg, us, eb, ec, nseg, mran, mtq;
};

// Host half of stab_compile: validate and split the stream for geometry g into P's plan and
// the blob of device arrays.  Touches no device.
int compile_host(const Geom& g, const stab_instr* instrs, int32_t ninstr, const int32_t* targets,
                 int64_t ntargets, stab_program& P, ProgramBlob& B)
{
    std::vector<int4> items;
    std::vector<uint2> gates;
    std::vector<NoiseDesc> noise;
    std::vector<int> noise_tg, unit_start, ev_base, mtq;
    int rc = compile_stream(g, instrs, ninstr, targets, ntargets, P, items, gates, noise, noise_tg,
                            unit_start, ev_base, mtq);
    if (rc) return rc;
    P.n = g.n;
    P.B = g.B;
    std::vector<char>& blob = B.bytes;
    B.items = put(blob, items);
    B.gates = put(blob, gates);
    B.noise = put(blob, noise);
    B.ntg = put(blob, noise_tg);
    B.us = put(blob, unit_start);
    B.eb = put(blob, ev_base);
    B.ec = put(blob, std::vector<int>(std::max<int>(P.nnoise, 1), 0));
    std::vector<long long> nseg(std::max<size_t>(noise.size(), 1), 0);
    for (const SegPlan& sp : P.segs)
        for (int i = 0; i < sp.noise_count; ++i) nseg[sp.noise_begin + i] = sp.ev_global;
    B.nseg = put(blob, nseg);
    B.mran = put(blob, std::vector<int>(std::max<size_t>(P.meas.size(), 1), 0));
    B.mtq = put(blob, mtq);
    return STAB_OK;
}

// Device half: the blob goes to device memory (the context's static scratch when it has one).
// On failure P is left without device memory.
int upload_program(stab_ctx* ctx, stab_program& P, const ProgramBlob& B)
{
    const std::vector<char>& blob = B.bytes;
    if (ctx->arena) {
        const int rc = arena_take(ctx, blob.size(), &P.dev);
        if (rc) return rc;
        P.dev_arena = true;
    } else if (hipMalloc(&P.dev, blob.size()) != hipSuccess) {
        P.dev = nullptr;
        return fail(STAB_ENOMEM, "device allocation failed");
    }
    if (hipMemcpy(P.dev, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
        if (!P.dev_arena) (void)hipFree(P.dev);
        P.dev = nullptr;
        ctx->poisoned = true;
        return fail(STAB_EDEVICE, "program upload failed");
    }
    char* d = (char*)P.dev;
    P.d_items = (int4*)(d + B.items);
    P.d_gates = (uint2*)(d + B.gates);
    P.d_noise = (NoiseDesc*)(d + B.noise);
    P.d_noise_tg = (int*)(d + B.ntg);
    P.d_unit_start = (int*)(d + B.us);
    P.d_ev_base = (int*)(d + B.eb);
    P.d_ev_count = (int*)(d + B.ec);
    P.d_noise_seg = (long long*)(d + B.nseg);
    P.d_mran = (int*)(d + B.mran);
    P.d_mtq = (int*)(d + B.mtq);
    return STAB_OK;
}

}  // namespace

extern "C" {

int stab_compile(stab_ctx* ctx, const stab_instr* instrs, int32_t ninstr, const int32_t* targets,
                 int64_t ntargets, stab_program** out)
{
    if (!ctx || !out) return fail(STAB_EINVAL, "null argument");
    *out = nullptr;
    if (ctx->poisoned) return fail(STAB_EDEVICE, "context poisoned by an earlier device error");
    stab_program* P = new stab_program();
    static std::atomic<uint64_t> program_serial{0};
    P->serial = ++program_serial;
    ProgramBlob B;
    int rc = compile_host(ctx->g, instrs, ninstr, targets, ntargets, *P, B);
    if (rc == STAB_OK) rc = upload_program(ctx, *P, B);
    if (rc) {
        delete P;
        return rc;
    }
    *out = P;
    return STAB_OK;
}

int64_t stab_program_records(const stab_program* prog) { return prog ? prog->nrec : -1; }

int stab_plan_describe(int32_t n, int32_t shots, int32_t mode, const stab_instr* instrs, int32_t ninstr,
                       const int32_t* targets, int64_t ntargets, int64_t* out, int32_t nout)
{
    if (nout < 0 || nout > STAB_PLAN_FIELDS || (nout > 0 && !out)) return fail(STAB_EINVAL, "bad output array");
    uint64_t bytes = 0;
    int rc = stab_tableau_bytes(n, shots, mode, &bytes);
    if (rc) return rc;
    stab_program P;
    std::vector<int4> items;
    std::vector<uint2> gates;
    std::vector<NoiseDesc> noise;
    std::vector<int> noise_tg, unit_start, ev_base, mtq;
    rc = compile_stream(make_geom(n, shots, mode), instrs, ninstr, targets, ntargets, P, items, gates, noise,
                        noise_tg, unit_start, ev_base, mtq);
    if (rc) return rc;
    long long gate_layers = 0, units = 0;
    for (const int4& it : items) gate_layers += it.x == 0 ? 1 : 0;
    for (const NoiseDesc& d : noise) units += d.units;
    const int64_t v[STAB_PLAN_FIELDS] = {(int64_t)P.segs.size(), (int64_t)P.meas.size(), gate_layers,
                                         (int64_t)gates.size(), (int64_t)noise.size(), units, P.nrec, P.Kmax};
    for (int i = 0; i < nout; ++i) out[i] = v[i];
    return STAB_OK;
}

void stab_program_destroy(stab_program* prog)
{
    if (!prog) return;
    if (prog->dev && !prog->dev_arena) (void)hipFree(prog->dev);   // implicitly waits for work that uses it
    delete prog;
}

}  // extern "C"

namespace {

// Bytes of the device buffers one execution of P needs, in the order xcol, zcol, cls, pend,
// obuf, events, record, packed, plog_p, plog_rs, plog_row, plog_rd, ran, plist, pcnt, povf.
constexpr int kExecBufs = 16;
void exec_sizes(const Geom& g, const stab_program& P, bool draw_all, size_t* sizes)
{
    const size_t K = (size_t)std::max(P.Kmax, 1);
    const size_t nrec = (size_t)std::max<long long>(P.nrec, 1);
    const size_t v[kExecBufs] = {(size_t)g.S * g.NB * K * 8, (size_t)g.S * g.NB * K * 8, (size_t)g.S * K * 4,
                                 (size_t)g.S * K * 4, (size_t)g.B * K,
                                 (size_t)std::max<long long>(draw_all ? P.ev_total : P.ev_cap_max, 1) * 8,
                                 (size_t)g.B * nrec, (size_t)g.B * ((nrec + 7) / 8), (size_t)g.S * K * 4,
                                 (size_t)g.S * K * 4, (size_t)g.S * K * g.RS * 8,
                                 (size_t)g.S * K * ((g.bpc + 63) / 64) * 8, 4, (size_t)g.S * K * kPListCap * 2,
                                 (size_t)g.S * K * 4, (size_t)g.S * 4};
    for (int i = 0; i < kExecBufs; ++i) sizes[i] = v[i];
}

// Device buffers of one execution of P, grown (or carved from the context's scratch) before
// anything is enqueued.  The noise of every segment is drawn by one launch at the start when its
// event slots fit (the draws depend on the RNG key only, not on the tableau), else segment by
// segment; *draw_all_out says which.
int exec_prepare(stab_ctx* ctx, const stab_program* P, bool allow_draw_all, bool* draw_all_out)
{
    const Geom& g = ctx->g;
    bool draw_all = allow_draw_all && P->nnoise > 0 && P->nnoise <= 65535 && P->ev_total <= kDrawAllEvents;
    int rc;
    DevBuf* bufs[kExecBufs] = {&ctx->xcol, &ctx->zcol, &ctx->cls, &ctx->pend, &ctx->obuf, &ctx->events,
                               &ctx->record, &ctx->packed, &ctx->plog_p, &ctx->plog_rs, &ctx->plog_row,
                               &ctx->plog_rd, &ctx->ran, &ctx->plist, &ctx->pcnt, &ctx->povf};
    size_t sizes[kExecBufs];
    exec_sizes(g, *P, draw_all, sizes);
    if (ctx->arena && draw_all) {
        // in the static scratch the whole program's noise is drawn at once only if it fits
        size_t at = ctx->arena_used;
        for (int i = 0; i < kExecBufs; ++i)
            if (bufs[i]->cap < sizes[i]) at = align256(at) + std::max<size_t>(align256(sizes[i]), 256);
        if (at > ctx->arena_cap) {
            draw_all = false;
            exec_sizes(g, *P, draw_all, sizes);
        }
    }
    for (int i = 0; i < kExecBufs; ++i)
        if ((rc = ensure(ctx, *bufs[i], sizes[i]))) return rc;
    *draw_all_out = draw_all;
    return STAB_OK;
}

// Launch shapes of one execution that depend on the geometry and the device's LDS.
struct ExecLds {
    int lds_rd = 0;           // per-shot sign accumulators of the segment kernel in LDS
    size_t seg_lds = 0, chain_lds = 0, replay_lds = 0;
    int ent_cap = -1;         // replay list entries in LDS (-1: the replay's small form)
};

int exec_lds(const Geom& g, const stab_program& P, int max_lds, ExecLds* out)
{
    ExecLds E;
    const size_t K = (size_t)std::max(P.Kmax, 1);
    // per-shot sign accumulators in LDS only where they keep two half-band blocks per compute
    // unit (or where even one block without them would not get two)
    const int seg_base = seg_lds_words(g.RS) * 4, seg_acc = (seg_lds_words(g.RS) + g.bpc) * 4;
    E.lds_rd = (seg_acc <= max_lds / 2 || (seg_base > max_lds / 2 && seg_acc <= max_lds)) ? 1 : 0;
    E.seg_lds = (size_t)(seg_lds_words(g.RS) + (E.lds_rd ? g.bpc : 0)) * 4;
    E.chain_lds = (size_t)chain_lds_layout(g).total;
    if (E.chain_lds + kReplayStatic > (size_t)max_lds)   // (a bound on its static LDS too)
        return fail(STAB_ERANGE, "too many shots per copy for the chain kernel");
    // the replay's list form when its fixed part leaves room for list entries in LDS
    const ReplayLds RL = replay_lds_layout((int)K, (g.bpc + 63) / 64, kReplayThreads / 64);
    // (kReplayStatic bytes of the block's LDS are its own __shared__ variables)
    E.replay_lds = (size_t)RL.small_bytes;
    const int replay_room = max_lds - kReplayStatic;
    if (replay_walk_fits((int)K) && RL.fixed_bytes + 2 * 1024 <= replay_room) {
        E.ent_cap = std::min((replay_room - RL.fixed_bytes) / 2, (int)K * kPListCap);
        E.replay_lds = (size_t)RL.fixed_bytes + 2 * (size_t)E.ent_cap;
    }
    if (E.replay_lds > (size_t)replay_room) return fail(STAB_ERANGE, "too many shots per copy for the replay kernel");
    *out = E;
    return STAB_OK;
}

// Every launch of one execution of P on ctx->stream, eagerly or into a graph (a fill kernel
// clears the event counts: no memset node in a captured graph).  use_mran skips the launches of
// measurement layers where nothing ran in an earlier execution from |0...0>; learn_mran marks,
// in P->d_mran, the layers where something runs.
int exec_enqueue(stab_ctx* ctx, stab_program* P, bool draw_all, bool use_mran, bool learn_mran)
{
    const Geom& g = ctx->g;
    uint64_t* Xcol = (uint64_t*)ctx->xcol.p;
    uint64_t* Zcol = (uint64_t*)ctx->zcol.p;
    int* cls = (int*)ctx->cls.p;
    uint8_t* obuf = (uint8_t*)ctx->obuf.p;
    uint2* events = (uint2*)ctx->events.p;
    uint8_t* record = (uint8_t*)ctx->record.p;
    const uint64_t base = ctx->instr_counter;

    ExecLds E;
    int rc = exec_lds(g, *P, ctx->max_lds, &E);
    if (rc) return rc;
    const int lds_rd = E.lds_rd, ent_cap = E.ent_cap;
    const size_t seg_lds = E.seg_lds, chain_lds = E.chain_lds, replay_lds = E.replay_lds;
    int* plog_p = (int*)ctx->plog_p.p;
    int* plog_rs = (int*)ctx->plog_rs.p;
    uint64_t* plog_row = (uint64_t*)ctx->plog_row.p;
    uint64_t* plog_rd = (uint64_t*)ctx->plog_rd.p;
    int* ran = (int*)ctx->ran.p;

    const long long nbytes = (P->nrec + 7) / 8;
    if (P->nnoise > 0)
        k_zero32<<<1, 256, 0, ctx->stream>>>((uint32_t*)P->d_ev_count, (long long)P->nnoise);
    if (draw_all) {
        const long long most = (long long)P->max_units * g.B;
        const dim3 grid((unsigned)((most + kNoiseUnitsPerBlock - 1) / kNoiseUnitsPerBlock), (unsigned)P->nnoise);
        TIMED(ctx, 1, (k_noise_draw<<<grid, kNoiseThreads, 0, ctx->stream>>>(
            P->d_noise, P->d_noise_tg, g.B, ctx->seed, ctx->first_shot, base, events, P->d_noise_seg,
            P->d_ev_base, P->d_ev_count, ctx->d_counters, g.rev)));
    }
    for (const auto& st : P->steps) {
        if (st.first == 0) {
            const SegPlan& sp = P->segs[st.second];
            if (sp.noise_count > 0 && !draw_all) {
                const long long most = (long long)sp.max_units * g.B;
                const dim3 grid((unsigned)((most + kNoiseUnitsPerBlock - 1) / kNoiseUnitsPerBlock),
                                (unsigned)sp.noise_count);
                TIMED(ctx, 1, (k_noise_draw<<<grid, kNoiseThreads, 0, ctx->stream>>>(
                    P->d_noise + sp.noise_begin, P->d_noise_tg, g.B, ctx->seed, ctx->first_shot, base, events,
                    nullptr, P->d_ev_base, P->d_ev_count, ctx->d_counters, g.rev)));
            }
            if (sp.item_count > 0 || sp.meas >= 0) {
                SegArgs a{};
                a.items = P->d_items + sp.item_begin;
                a.nitems = sp.item_count;
                a.gates = P->d_gates;
                a.events = events + (draw_all ? sp.ev_global : 0);
                a.ev_count = P->d_ev_count;
                a.ev_base = P->d_ev_base;
                a.write_back = sp.modifies;
                a.lds_rd = lds_rd;
                if (sp.meas >= 0) {
                    const MeasPlan& m = P->meas[sp.meas];
                    a.ext_q = P->d_mtq + m.tq_begin;
                    a.K = m.K;
                } else {
                    a.ext_q = nullptr;
                    a.K = 0;
                }
                a.Xcol = Xcol;
                a.Zcol = Zcol;
                TIMED(ctx, 2, (k_segment<<<dim3(2 * g.NB, g.S), kSegThreads, seg_lds, ctx->stream>>>(
                                  g, ctx->tab, ctx->rs, ctx->rd, a)));
            }
        } else {
            const MeasPlan& m = P->meas[st.second];
            const int K2 = m.K;
            // classes of the targets and the outcomes of the deterministic ones (also clears ran)
            const int dt = det_targets((g.Wc + 63) / 64);
            const dim3 dgrid((K2 + dt - 1) / dt, g.S);
            const size_t det_lds = (size_t)dt * (g.NB + (g.bpc + 63) / 64) * 8;
            TIMED(ctx, 3, (det_kernel(g.Wc)<<<dgrid, 64 * dt, det_lds, ctx->stream>>>(g, ctx->tab, ctx->rs, ctx->rd, Xcol, K2, cls,
                                                                       obuf, ran, ctx->d_err, ctx->d_counters, 0, nullptr)));
            // a layer where nothing ran in an earlier execution from |0...0>: the next four
            // launches would return at once
            if (!use_mran || P->mran[st.second]) {
            TIMED(ctx, 5, (chain_kernel(g.Wc)<<<g.S, chain_threads((g.Wc + 63) / 64), chain_lds, ctx->stream>>>(
                              g, ctx->tab, ctx->rs, ctx->rd, Xcol, Zcol, K2, cls, P->d_mtq + m.tq_begin,
                              (int*)ctx->pend.p, ctx->seed, ctx->first_shot, base + m.instr,
                              m.pos_base, plog_p, plog_row, plog_rs, plog_rd, ran, (uint16_t*)ctx->plist.p,
                              (int*)ctx->pcnt.p, (int*)ctx->povf.p, obuf, ctx->d_err, ctx->d_counters)));
            // destabilizer updates of the run targets, then fresh columns of the final tableau
            // (skipped on the device when nothing ran)
            TIMED(ctx, 8, (replay_kernel(g.Wc)<<<dim3(g.Wr, g.S), kReplayThreads, replay_lds, ctx->stream>>>(
                              g, ctx->tab, ctx->rs, ctx->rd, Xcol, K2, P->d_mtq + m.tq_begin, plog_p, plog_row,
                              plog_rs, plog_rd, (const uint16_t*)ctx->plist.p, (const int*)ctx->pcnt.p,
                              (const int*)ctx->povf.p, ran, ent_cap, ctx->d_err, ctx->d_counters)));
            {
                SegArgs a{};
                a.items = P->d_items;
                a.nitems = 0;
                a.gates = P->d_gates;
                a.events = events;
                a.ev_count = P->d_ev_count;
                a.ev_base = P->d_ev_base;
                a.write_back = 0;
                a.lds_rd = 0;
                a.ext_q = P->d_mtq + m.tq_begin;
                a.K = K2;
                a.Xcol = Xcol;
                a.Zcol = Zcol;
                a.gate = ran;
                TIMED(ctx, 9, (k_segment<<<dim3(2 * g.NB, g.S), kSegThreads, (size_t)seg_lds_words(g.RS) * 4,
                                           ctx->stream>>>(g, ctx->tab, ctx->rs, ctx->rd, a)));
            }
            // targets the chain found deterministic: reduced in parallel on the final tableau
            TIMED(ctx, 4, (det_kernel(g.Wc)<<<dgrid, 64 * dt, det_lds, ctx->stream>>>(g, ctx->tab, ctx->rs, ctx->rd, Xcol, K2, cls,
                                                                       obuf, ran, ctx->d_err, ctx->d_counters, 1,
                                                                       learn_mran ? P->d_mran + st.second : nullptr)));
            }
            const int do_reset = m.kind != STAB_M, do_record = m.kind != STAB_R;
            const int rshots = std::min(g.B, kResetShots);
            const dim3 rgrid(g.NB, (g.B + rshots - 1) / rshots, std::max(1, (K2 + kResetChunk - 1) / kResetChunk));
            TIMED(ctx, 6, (k_reset_record<<<rgrid, 64 * rshots, 0, ctx->stream>>>(
                              g, ctx->rd, Zcol, obuf, K2, do_reset, record, (long long)P->nrec, m.rec_off,
                              do_record)));
        }
    }
    if (P->nrec > 0) {
        const long long total = nbytes * g.B;
        const int blocks = (int)std::min<long long>((total + 255) / 256, 1 << 16);
        TIMED(ctx, 7, (k_pack<<<blocks, 256, 0, ctx->stream>>>(record, P->nrec, g.B, (uint8_t*)ctx->packed.p)));
    }
    HIP_CHECK(ctx, hipGetLastError());
    return STAB_OK;
}

}  // namespace

extern "C" {

int stab_execute(stab_ctx* ctx, stab_program* P, uint8_t* out_bits, float* elapsed_ms)
{
    if (!ctx || !P) return fail(STAB_EINVAL, "null argument");
    if (ctx->poisoned) return fail(STAB_EDEVICE, "context poisoned by an earlier device error");
    const Geom& g = ctx->g;
    if (P->n != g.n || P->B != g.B) return fail(STAB_EINVAL, "program compiled for another geometry");
    if (P->nrec > 0 && !out_bits) return fail(STAB_EINVAL, "out_bits is NULL but the stream records outcomes");
    bool draw_all = false;
    int rc;
    if ((rc = exec_prepare(ctx, P, true, &draw_all))) return rc;
    const long long nbytes = (P->nrec + 7) / 8;
    // layers where nothing ran are known once the program has run from |0...0>
    const uint64_t base = ctx->instr_counter;
    const bool use_mran = base == 0 && P->mran_known;
    const bool learn_mran = base == 0 && !P->mran_known && !P->meas.empty();
    auto enqueue = [&]() -> int { return exec_enqueue(ctx, P, draw_all, use_mran, learn_mran); };

    if (ctx->ev0) HIP_CHECK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    if (ctx->graph_on && !ctx->timing && !learn_mran) {
        // the launches depend on the program, the RNG key, the instruction counter and the
        // buffers: replay the captured graph while they are unchanged, capture again otherwise
        uint64_t bufsig = 0;
        const DevBuf* bufs[] = {&ctx->xcol, &ctx->zcol, &ctx->cls, &ctx->obuf, &ctx->events, &ctx->record,
                                &ctx->packed, &ctx->pend, &ctx->plog_p, &ctx->plog_row, &ctx->plog_rs,
                                &ctx->plog_rd, &ctx->ran, &ctx->plist, &ctx->pcnt, &ctx->povf};
        for (const DevBuf* b : bufs) bufsig = bufsig * 1099511628211ull ^ (uint64_t)(uintptr_t)b->p;
        const uint64_t key[5] = {P->serial, ctx->seed, ctx->first_shot, base, bufsig};
        if (!ctx->gexec || std::memcmp(key, ctx->gkey, sizeof(key)) != 0) {
            if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
            if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
            ctx->gexec = nullptr;
            ctx->graph = nullptr;
            if (!ctx->cap_stream) HIP_CHECK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
            HIP_CHECK(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
            hipStream_t run_stream = ctx->stream;
            ctx->stream = ctx->cap_stream;          // the launches below are recorded, not run
            const int erc = enqueue();
            hipGraph_t gr = nullptr;
            const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &gr);
            ctx->stream = run_stream;
            if (erc || ec != hipSuccess) {
                if (gr) (void)hipGraphDestroy(gr);
                ctx->poisoned = true;
                return erc ? erc : fail(STAB_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
            }
            ctx->graph = gr;
            HIP_CHECK(ctx, hipGraphInstantiate(&ctx->gexec, gr, nullptr, nullptr, 0));
            std::memcpy(ctx->gkey, key, sizeof(key));
        }
        HIP_CHECK(ctx, hipGraphLaunch(ctx->gexec, ctx->stream));
    } else if ((rc = enqueue())) {
        return rc;
    }
    std::vector<uint8_t> host;
    if (P->nrec > 0) {
        const long long total = nbytes * g.B;
        host.resize((size_t)total);
        HIP_CHECK(ctx, hipMemcpyAsync(host.data(), ctx->packed.p, (size_t)total, hipMemcpyDeviceToHost, ctx->stream));
    }
    if (ctx->ev1) HIP_CHECK(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    int err = 0;
    HIP_CHECK(ctx, hipMemcpy(&err, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost));
    if (err) {
        ctx->poisoned = true;
        return fail(STAB_EINTERNAL, "device consistency check failed (code " + std::to_string(err) + ")");
    }
    if (elapsed_ms && ctx->ev0) HIP_CHECK(ctx, hipEventElapsedTime(elapsed_ms, ctx->ev0, ctx->ev1));
    if (ctx->timing && (rc = tcollect(ctx))) return rc;
    if (learn_mran) {
        P->mran.assign(P->meas.size(), 1);
        HIP_CHECK(ctx, hipMemcpy(P->mran.data(), P->d_mran, P->meas.size() * sizeof(int), hipMemcpyDeviceToHost));
        P->mran_known = true;
    }
    if (P->nrec > 0) std::memcpy(out_bits, host.data(), host.size());
    ctx->instr_counter += (uint64_t)P->ninstr;
    return STAB_OK;
}

int stab_run(stab_ctx* ctx, const stab_instr* instrs, int32_t ninstr, const int32_t* targets,
             int64_t ntargets, uint8_t* out_bits)
{
    stab_program* P = nullptr;
    int rc = stab_compile(ctx, instrs, ninstr, targets, ntargets, &P);
    if (rc) return rc;
    rc = stab_execute(ctx, P, out_bits, nullptr);
    stab_program_destroy(P);
    return rc;
}

int stab_apply_layer(stab_ctx* ctx, const stab_instr* instrs, int32_t ninstr,
                     const int32_t* targets, int64_t ntargets)
{
    for (int32_t k = 0; k < ninstr && instrs; ++k)
        if (instrs[k].kind == STAB_M || instrs[k].kind == STAB_MR || instrs[k].kind == STAB_R)
            return fail(STAB_EINVAL, "stab_apply_layer takes no measurement instructions");
    return stab_run(ctx, instrs, ninstr, targets, ntargets, nullptr);
}

int stab_measure(stab_ctx* ctx, uint32_t kind, const int32_t* qubits, int32_t k, uint8_t* out_bits)
{
    if (kind != STAB_M && kind != STAB_MR && kind != STAB_R) return fail(STAB_EINVAL, "kind must be M, MR or R");
    if (k < 0) return fail(STAB_EINVAL, "negative count");
    stab_instr in{};
    in.kind = kind;
    in.ntargets = (uint32_t)k;
    return stab_run(ctx, &in, 1, qubits, k, out_bits);
}

int stab_get_tableau(stab_ctx* ctx, int32_t shot, uint8_t* x, uint8_t* z, uint8_t* r)
{
    if (!ctx) return fail(STAB_EINVAL, "ctx is NULL");
    if (ctx->poisoned) return fail(STAB_EDEVICE, "context poisoned by an earlier device error");
    const Geom& g = ctx->g;
    if (shot < 0 || shot >= g.B) return fail(STAB_EINVAL, "shot out of range");
    const int s = shot / g.bpc;
    std::vector<uint64_t> tab((size_t)2 * g.NR * g.RS), rs(g.NB), rd(g.NB);
    HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    HIP_CHECK(ctx, hipMemcpy(tab.data(), ctx->tab + (size_t)s * 2 * g.NR * g.RS, tab.size() * 8, hipMemcpyDeviceToHost));
    HIP_CHECK(ctx, hipMemcpy(rs.data(), ctx->rs + (size_t)s * g.NB, g.NB * 8, hipMemcpyDeviceToHost));
    HIP_CHECK(ctx, hipMemcpy(rd.data(), ctx->rd + (size_t)shot * g.NB, g.NB * 8, hipMemcpyDeviceToHost));
    const int n = g.n;
    for (int half = 0; half < 2; ++half) {
        for (int i = 0; i < n; ++i) {
            const int row = half * g.NR + i;
            const int out = half * n + i;
            const uint64_t* w = &tab[(size_t)row * g.RS];
            for (int j = 0; j < n; ++j) {
                if (x) x[(size_t)out * n + j] = (uint8_t)((w[j >> 6] >> (j & 63)) & 1ull);
                if (z) z[(size_t)out * n + j] = (uint8_t)((w[g.Wc + (j >> 6)] >> (j & 63)) & 1ull);
            }
            if (r) r[out] = (uint8_t)(((rs[row >> 6] ^ rd[row >> 6]) >> (row & 63)) & 1ull);
        }
    }
    return STAB_OK;
}

int stab_get_counters(stab_ctx* ctx, uint64_t* counters, int32_t ncounters)
{
    if (!ctx || !counters || ncounters < 0 || ncounters > kNumCounters) return fail(STAB_EINVAL, "bad arguments");
    unsigned long long c[kNumCounters * kCounterStripes];
    HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    HIP_CHECK(ctx, hipMemcpy(c, ctx->d_counters, sizeof(c), hipMemcpyDeviceToHost));
    for (int i = 0; i < ncounters; ++i) {
        uint64_t v = 0;
        for (int j = 0; j < kCounterStripes; ++j) v += c[i * kCounterStripes + j];
        counters[i] = v;
    }
    return STAB_OK;
}

int stab_set_timing(stab_ctx* ctx, int32_t kernel_mask)
{
    if (!ctx) return fail(STAB_EINVAL, "ctx is NULL");
    HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->tmask = (uint32_t)kernel_mask & ((1u << kNumKernels) - 1u);
    ctx->timing = ctx->tmask != 0;
    ctx->evkind.clear();
    ctx->evused = 0;
    for (int i = 0; i < kNumKernels; ++i) {
        ctx->kms[i] = 0.0;
        ctx->klaunch[i] = 0;
    }
    return STAB_OK;
}

int stab_set_graph(stab_ctx* ctx, int32_t enable)
{
    if (!ctx) return fail(STAB_EINVAL, "null context");
    ctx->graph_on = enable != 0;
    return STAB_OK;
}

int stab_get_kernel_times(stab_ctx* ctx, double* ms, uint64_t* launches, int32_t nkernels)
{
    if (!ctx || nkernels < 0 || nkernels > kNumKernels) return fail(STAB_EINVAL, "bad arguments");
    for (int i = 0; i < nkernels; ++i) {
        if (ms) ms[i] = ctx->kms[i];
        if (launches) launches[i] = ctx->klaunch[i];
    }
    return STAB_OK;
}

int stab_sample(const stab_instr* instrs, int32_t ninstr, const int32_t* targets, int64_t ntargets,
                int32_t n, int32_t shots, int32_t mode, uint64_t seed, void* dev_buf, uint64_t buf_bytes,
                void* hip_stream, uint8_t* out_bits, float* elapsed_ms)
{
    stab_ctx* ctx = nullptr;
    int rc = stab_create(n, shots, mode, seed, 0, dev_buf, buf_bytes, hip_stream, &ctx);
    if (rc) return rc;
    stab_program* P = nullptr;
    rc = stab_compile(ctx, instrs, ninstr, targets, ntargets, &P);
    if (rc == STAB_OK) rc = stab_execute(ctx, P, out_bits, elapsed_ms);
    stab_program_destroy(P);
    stab_destroy(ctx);
    return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// stab_sample without device allocation.  Every buffer the library would allocate (error flag,
// counters, the uploaded program, target columns, noise events, pivot log, records) is carved
// from `scratch`, a static device array each GPU holds for the life of the process.  Its name
// is a host-side stand-in in host code: the device address of each GPU's copy is looked up
// once per device with hipGetSymbolAddress and only that address is handed to kernels and
// copies.  Calls on one GPU share the array, so calls that overlap on one GPU race.
// ---------------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[STAB_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;   // device ordinal -> address of its copy of scratch

// Address of the current device's copy of scratch (looked up on the first call per device).
int scratch_address(char** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(STAB_EDEVICE, "no HIP device");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return STAB_OK;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(STAB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)ptr;
    *out = (char*)ptr;
    return STAB_OK;
}

// Scratch bytes stab_sample_noalloc carves for this program (noise drawn segment by segment),
// in the order the context takes them.
size_t noalloc_bytes(const Geom& g, const stab_program& P, size_t blob_bytes)
{
    auto piece = [](size_t b) { return std::max<size_t>(align256(b), 256); };
    size_t total = piece(sizeof(int)) + piece(kNumCounters * kCounterStripes * sizeof(unsigned long long)) +
                   piece(blob_bytes);
    size_t sizes[kExecBufs];
    exec_sizes(g, P, false, sizes);
    for (size_t b : sizes) total += piece(b);
    return total;
}

}  // namespace

extern "C" int stab_sample_noalloc(const stab_instr* instrs, int32_t ninstr, const int32_t* targets,
                                   int64_t ntargets, int32_t n, int32_t shots, int32_t mode, uint64_t seed,
                                   void* dev_buf, uint64_t buf_bytes, void* hip_stream, uint8_t* out_bits)
{
    // everything that can be checked on the host is checked before the device is touched
    uint64_t need = 0;
    int rc = stab_tableau_bytes(n, shots, mode, &need);
    if (rc) return rc;
    if (!dev_buf) return fail(STAB_EINVAL, "dev_buf is NULL");
    if (((uintptr_t)dev_buf & 255u) != 0) return fail(STAB_EINVAL, "dev_buf must be 256-byte aligned");
    if (buf_bytes < need) return fail(STAB_ENOMEM, "dev_buf smaller than stab_tableau_bytes()");
    const Geom g = make_geom(n, shots, mode);
    stab_program P;
    ProgramBlob B;
    if ((rc = compile_host(g, instrs, ninstr, targets, ntargets, P, B))) return rc;
    if (P.nrec > 0 && !out_bits) return fail(STAB_EINVAL, "out_bits is NULL but the stream records outcomes");
    const size_t want = noalloc_bytes(g, P, B.bytes.size());
    if (want > (size_t)STAB_NOALLOC_SCRATCH_BYTES)
        return fail(STAB_ERANGE, "stab_sample_noalloc: this workload needs " + std::to_string(want) +
                                     " bytes of scratch; the static scratch holds " +
                                     std::to_string((size_t)STAB_NOALLOC_SCRATCH_BYTES) + " (use stab_sample)");
    char* arena = nullptr;
    if ((rc = scratch_address(&arena))) return rc;
    stab_ctx* ctx = nullptr;
    if ((rc = create_ctx(n, shots, mode, seed, 0, dev_buf, buf_bytes, hip_stream, arena,
                         (size_t)STAB_NOALLOC_SCRATCH_BYTES, &ctx)))
        return rc;
    rc = upload_program(ctx, P, B);
    if (rc == STAB_OK) rc = stab_execute(ctx, &P, out_bits, nullptr);
    P.dev = nullptr;   // (in the scratch: nothing to free)
    stab_destroy(ctx);
    return rc;
}

// Pauli-string commutation (Sec. 3.2)
extern "C" int stab_commute(const uint64_t* A, int32_t na, const uint64_t* B, int32_t nb, int32_t n,
                            uint64_t* gc, uint64_t* qwc, void* hip_stream)
{
    if (na < 0 || nb < 0 || n < 1) return fail(STAB_EINVAL, "need n >= 1 and na, nb >= 0");
    if ((na > 0 && !A) || (nb > 0 && !B)) return fail(STAB_EINVAL, "string array is NULL");
    if (!gc && !qwc) return fail(STAB_EINVAL, "both outputs are NULL");
    if (((uintptr_t)A | (uintptr_t)B | (uintptr_t)gc | (uintptr_t)qwc) & 7u)
        return fail(STAB_EINVAL, "arrays must be 8-byte aligned");
    if (na == 0 || nb == 0) return STAB_OK;
    const int W = (n + 63) / 64;
    const long long rows = ((long long)na + kCommRows - 1) / kCommRows;
    if (rows > 65535) return fail(STAB_ERANGE, "too many strings in A (at most 65535 * 64)");
    const dim3 grid((unsigned)((nb + 63) / 64), (unsigned)rows);
    k_commute<<<grid, kCommThreads, 0, (hipStream_t)hip_stream>>>(A, na, B, nb, W, gc, qwc);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(STAB_EDEVICE, std::string("k_commute: ") + hipGetErrorString(e));
    return STAB_OK;
}

// multi-circuit batches
#include "stab_batch_api.hip"

// continuous batching of sampling requests
#include "stab_server_api.hip"
