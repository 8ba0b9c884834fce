// stab_server_api.hip -- continuous batching of sampling requests (include/stab.h,
// stab_server_*).  Included at the end of stab_api.hip, after the batch code it runs on.
//
// A request is an op stream with a shot count and a seed; its records are those of the stream
// run alone with RNG key (seed, shot) per shot, whatever else is resident.  Requests are
// admitted in arrival order while their bytes fit in the caller's arena, into one of two lanes:
//
//  * batch lane: each shot is one circuit of the batch kernel (its own tableau).  Every step()
//    runs one launch that advances every resident shot of the lane by one measurement step (a
//    round of a memory experiment), so rounds of all resident requests share each launch, new
//    requests join at the next step and finished ones leave.  Any stream runs here, T1T2 too.
//  * shared lane (streams whose noise is all Pauli): the shots of a request share one x|z
//    tableau and keep their own sign bits (the shared mode; Sec. 3.1 of the paper keeps one
//    tableau per circuit).  Admission enqueues the request's whole program on one of a few
//    device streams, followed by the copy of its records to pinned host memory and an event;
//    step() retires the requests whose event has fired.  Requests on different streams run at
//    the same time on the device and none waits for a step boundary.
//
// Streams are compiled and uploaded once (stab_server_program; the shared lane's compile per
// power-of-two shot bucket at the first request of that bucket) and submitted by program id.

namespace {

// Growable device array mirrored on the host.
template <typename T>
struct DevVec {
    std::vector<T> host;
    T* dev = nullptr;
    size_t cap = 0;
    size_t synced = 0;   // host entries already on the device
};

template <typename T>
int devvec_sync(DevVec<T>& v, hipStream_t stream)
{
    if (v.host.size() > v.cap) {
        const size_t cap = std::max(v.host.size() * 2, (size_t)1024);
        T* p = nullptr;
        if (hipMalloc((void**)&p, cap * sizeof(T)) != hipSuccess) return fail(STAB_ENOMEM, "device allocation failed");
        if (v.dev) {
            if (hipStreamSynchronize(stream) != hipSuccess) return fail(STAB_EDEVICE, "stream synchronize failed");
            (void)hipFree(v.dev);
        }
        v.dev = p;
        v.cap = cap;
        v.synced = 0;
    }
    if (v.synced < v.host.size()) {
        if (hipMemcpyAsync(v.dev + v.synced, v.host.data() + v.synced, (v.host.size() - v.synced) * sizeof(T),
                           hipMemcpyHostToDevice, stream) != hipSuccess)
            return fail(STAB_EDEVICE, "program upload failed");
        if (hipStreamSynchronize(stream) != hipSuccess) return fail(STAB_EDEVICE, "stream synchronize failed");
        v.synced = v.host.size();
    }
    return STAB_OK;
}

// First-fit list of the free byte ranges of a buffer (the arena, the pinned staging).
struct FreeList {
    std::map<size_t, size_t> blocks;   // offset -> size
    size_t in_use = 0;

    void reset(size_t bytes)
    {
        blocks.clear();
        in_use = 0;
        if (bytes) blocks[0] = bytes;
    }

    bool take(size_t bytes, size_t* off)
    {
        for (auto it = blocks.begin(); it != blocks.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                blocks.erase(it);
                if (rest) blocks[at] = rest;
                in_use += bytes;
                return true;
            }
        }
        return false;
    }

    void give(size_t off, size_t bytes)
    {
        in_use -= bytes;
        auto it = blocks.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != blocks.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            blocks.erase(nx);
        }
        if (it != blocks.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                blocks.erase(it);
            }
        }
    }
};

constexpr int kSrvStreams = 4;                      // shared-lane device streams
constexpr int kSrvIdleQuota = 4;                    // batch-lane rounds per launch while none waits
constexpr size_t kSrvPinnedBytes = 64ull << 20;     // pinned staging of shared-lane records

// Shared-mode compile of a program for one shot bucket: the host plan and its device arrays
// (uploaded once, never written by a kernel; each request brings its own event counts and
// layer flags).
struct SrvVariant {
    stab_program plan;
    size_t tab_bytes = 0;       // the context's tableau and signs
    size_t scratch_bytes = 0;   // everything else the context carves (see srv_scratch_bytes)
};

struct SrvProgram {
    int n = 0;
    long long nrec = 0;
    int ninstr = 0;
    int step_base = 0, nsteps = 0;
    int kfast = 0;                // column scratch targets per band
    bool pauli_only = true;       // no T1T2: the shared lane can run it
    int lane = STAB_LANE_AUTO;
    std::vector<stab_instr> instrs;
    std::vector<int32_t> targets;
    std::map<int, std::unique_ptr<SrvVariant>> variants;   // by shot bucket
    // measurement layers where a target ran, learned by the first shared-lane request (x|z and
    // therefore which layers have random outcomes do not depend on the seed or the shot count)
    std::vector<int> mran;
    bool mran_known = false, mran_pending = false;
};

struct SrvRequest {
    int64_t id = 0;
    int prog = 0;
    int shots = 0;
    uint64_t seed = 0;
    size_t off = 0, bytes = 0;    // arena block
    bool cancelled = false;
    std::vector<uint8_t> result;
    // batch lane
    size_t rec_off = 0;           // byte offset of the records inside the arena
    std::vector<int> cursor;      // per shot: next program step
    int remaining = 0;            // shots not finished
    // shared lane
    bool shared = false;
    int bucket = 0;               // shots the context runs (a power of two >= shots)
    stab_ctx* ctx = nullptr;
    stab_program P;               // the variant's plan with this request's counters
    int stream = -1;
    hipEvent_t ev = nullptr;
    size_t pin_off = 0, pin_bytes = 0;
    bool learn = false;
};

int shot_bucket(int shots)
{
    int b = 1;
    while (b < shots) b <<= 1;
    return b;
}

// Pinned bytes of a shared-lane request: its records, the error flag, the layer flags.
size_t srv_pin_bytes(const stab_program& P, int shots)
{
    return align256((size_t)shots * (size_t)((P.nrec + 7) / 8)) + 256 +
           align256(std::max<size_t>(P.meas.size(), 1) * 4);
}

// Bytes a shared-lane context carves after its tableau, in the order it takes them: the error
// flag and the work counters (create_ctx), the event counts and layer flags of its copy of the
// program, the execution buffers with the noise drawn segment by segment (exec_prepare).
size_t srv_scratch_bytes(const Geom& g, const stab_program& P)
{
    auto piece = [](size_t b) { return std::max<size_t>(align256(b), 256); };
    size_t total = piece(sizeof(int)) + piece(kNumCounters * kCounterStripes * sizeof(unsigned long long)) +
                   piece(std::max<size_t>(P.nnoise, 1) * 4) + piece(std::max<size_t>(P.meas.size(), 1) * 4);
    size_t sizes[kExecBufs];
    exec_sizes(g, P, false, sizes);
    for (size_t b : sizes) total += piece(b);
    return total;
}

// per shot: tableau, signs, column scratch [2][NB][kfast]
size_t srv_shot_bytes(int n, int kfast)
{
    const int Wc = (n + 63) / 64;
    return align256((size_t)2 * 64 * Wc * 2 * Wc * 8) + align256((size_t)2 * Wc * 8) +
           align256((size_t)2 * 2 * Wc * kfast * 8);
}

size_t srv_request_bytes(int n, int kfast, int shots, long long nrec)
{
    return (size_t)shots * srv_shot_bytes(n, kfast) + align256((size_t)shots * (size_t)((nrec + 7) / 8));
}

}  // namespace

struct stab_server {
    hipStream_t stream = nullptr;
    char* base = nullptr;
    size_t bytes = 0;
    int max_lds = 0;
    bool poisoned = false;
    FreeList arena;
    // program arena (all cached programs, indices global)
    std::vector<SrvProgram> progs;
    DevVec<int4> steps;
    DevVec<uint2> gates;
    DevVec<NoiseDesc> noise;
    DevVec<int> noise_tg;
    DevVec<BatchMeas> meas;
    DevVec<int> meas_tg;
    // requests
    int64_t next_id = 1;
    std::deque<SrvRequest> queue;
    std::vector<SrvRequest> resident;
    std::map<int64_t, SrvRequest> done;
    std::deque<int64_t> finished;                    // ids not yet returned by poll
    long long iterations = 0, completed = 0, cancelled = 0;
    // per-step device tables of the batch lane
    DevBuf d_circ, d_order, d_keys, d_ibase, d_init;
    int* d_err = nullptr;
    unsigned long long* d_counters = nullptr;
    // shared lane
    hipStream_t lanes[kSrvStreams] = {};
    int lane_busy[kSrvStreams] = {};                 // requests in flight per stream
    int lane_next = 0;
    char* pinned = nullptr;                          // hipHostMalloc'd at the first shared request
    FreeList pin;
    std::vector<hipEvent_t> evfree;
    int in_flight = 0;
};

namespace {

#define SHIP_CHECK(s, call)                                                                    \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            (s)->poisoned = true;                                                              \
            return fail(STAB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
        }                                                                                      \
    } while (0)

// Circuit table entry of shot `shot` of batch-lane request r starting at program step `cursor`.
BatchCirc srv_circ(const stab_server* s, const SrvRequest& r, int shot, int cursor)
{
    const SrvProgram& P = s->progs[r.prog];
    BatchCirc C{};
    C.n = P.n;
    C.Wc = (P.n + 63) / 64;
    C.RS = 2 * C.Wc;
    C.NR = 64 * C.Wc;
    const size_t shot_b = srv_shot_bytes(P.n, P.kfast);
    const size_t tab_b = align256((size_t)2 * C.NR * C.RS * 8);
    const size_t sg_b = align256((size_t)2 * C.Wc * 8);
    C.tab_off = (long long)((r.off + (size_t)shot * shot_b) / 8);
    C.rs_off = (long long)((r.off + (size_t)shot * shot_b + tab_b) / 8);
    C.col_off = (long long)((r.off + (size_t)shot * shot_b + tab_b + sg_b) / 8);
    C.col_k = P.kfast;
    C.step_begin = P.step_base + cursor;
    C.step_count = P.nsteps - cursor;
    C.rec_bit_off = (long long)(r.rec_off + (size_t)shot * (size_t)((P.nrec + 7) / 8)) * 8;
    return C;
}

// Lane a program's next requests go to.
bool srv_shared_lane(const SrvProgram& P) { return P.lane == STAB_LANE_SHARED || (P.lane == STAB_LANE_AUTO && P.pauli_only); }

// The shared-mode compile of program `prog` for `bucket` shots (compiled and uploaded on first
// use).
int srv_variant(stab_server* s, int prog, int bucket, SrvVariant** out)
{
    SrvProgram& G = s->progs[prog];
    auto it = G.variants.find(bucket);
    if (it != G.variants.end()) {
        *out = it->second.get();
        return STAB_OK;
    }
    uint64_t tab = 0;
    int rc = stab_tableau_bytes(G.n, bucket, STAB_MODE_SHARED, &tab);
    if (rc) return rc;
    std::unique_ptr<SrvVariant> V(new SrvVariant());
    const Geom g = make_geom(G.n, bucket, STAB_MODE_SHARED);
    ProgramBlob B;
    if ((rc = compile_host(g, G.instrs.data(), (int32_t)G.instrs.size(), G.targets.data(),
                           (int64_t)G.targets.size(), V->plan, B)))
        return rc;
    ExecLds E;
    if ((rc = exec_lds(g, V->plan, s->max_lds, &E))) return rc;
    stab_ctx up;   // (no scratch: the arrays go to device memory of their own)
    if ((rc = upload_program(&up, V->plan, B))) {
        s->poisoned = true;
        return rc;
    }
    V->tab_bytes = align256(tab);
    V->scratch_bytes = srv_scratch_bytes(g, V->plan);
    *out = V.get();
    G.variants.emplace(bucket, std::move(V));
    return STAB_OK;
}

// Enqueue shared-lane request r (its arena and pinned blocks already taken) on the least busy
// stream: context set-up, the whole program, the copies of its records, error flag and layer
// flags to pinned memory, then its completion event.
int srv_launch_shared(stab_server* s, SrvRequest& r)
{
    SrvProgram& G = s->progs[r.prog];
    const SrvVariant& V = *G.variants.at(r.bucket);
    int k = s->lane_next;
    for (int j = 0; j < kSrvStreams; ++j) {
        const int c = (s->lane_next + j) % kSrvStreams;
        if (s->lane_busy[c] < s->lane_busy[k]) k = c;
    }
    s->lane_next = (k + 1) % kSrvStreams;
    hipStream_t st = s->lanes[k];
    char* blk = s->base + r.off;
    stab_ctx* ctx = nullptr;
    int rc = create_ctx(G.n, r.bucket, STAB_MODE_SHARED, r.seed, 0, blk, V.tab_bytes, st, blk + V.tab_bytes,
                        V.scratch_bytes, &ctx, false);
    if (rc) {
        s->poisoned = true;
        return rc;
    }
    r.ctx = ctx;
    r.stream = k;
    r.P = V.plan;
    r.P.dev = nullptr;   // the arrays belong to the variant
    r.P.dev_arena = true;
    const size_t nmeas = std::max<size_t>(r.P.meas.size(), 1);
    void* evc = nullptr;
    void* mr = nullptr;
    if ((rc = arena_take(ctx, std::max<size_t>(r.P.nnoise, 1) * 4, &evc)) || (rc = arena_take(ctx, nmeas * 4, &mr))) {
        s->poisoned = true;
        return rc;
    }
    r.P.d_ev_count = (int*)evc;
    r.P.d_mran = (int*)mr;
    r.learn = !G.mran_known && !G.mran_pending && !r.P.meas.empty();
    if (r.learn) {
        G.mran_pending = true;
        k_zero32<<<1, 256, 0, st>>>((uint32_t*)mr, (long long)nmeas);
        SHIP_CHECK(s, hipGetLastError());
    }
    if (G.mran_known) {
        r.P.mran = G.mran;
        r.P.mran_known = true;
    }
    bool draw_all = false;
    if ((rc = exec_prepare(ctx, &r.P, false, &draw_all)) || (rc = exec_enqueue(ctx, &r.P, draw_all, G.mran_known, r.learn))) {
        s->poisoned = true;
        return rc;
    }
    char* pin = s->pinned + r.pin_off;
    const size_t rec_b = (size_t)r.shots * (size_t)((r.P.nrec + 7) / 8);
    if (rec_b) SHIP_CHECK(s, hipMemcpyAsync(pin, ctx->packed.p, rec_b, hipMemcpyDeviceToHost, st));
    SHIP_CHECK(s, hipMemcpyAsync(pin + align256(rec_b), ctx->d_err, sizeof(int), hipMemcpyDeviceToHost, st));
    if (r.learn)
        SHIP_CHECK(s, hipMemcpyAsync(pin + align256(rec_b) + 256, mr, r.P.meas.size() * 4, hipMemcpyDeviceToHost, st));
    if (s->evfree.empty()) {
        hipEvent_t e = nullptr;
        SHIP_CHECK(s, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        s->evfree.push_back(e);
    }
    r.ev = s->evfree.back();
    s->evfree.pop_back();
    SHIP_CHECK(s, hipEventRecord(r.ev, st));
    ++s->lane_busy[k];
    ++s->in_flight;
    return STAB_OK;
}

// Release what a shared-lane request holds once its event has fired (its stream may already
// run later requests: nothing here waits for the stream).
void srv_release_shared(stab_server* s, SrvRequest& r)
{
    delete r.ctx;   // every buffer of it lies in the arena block
    r.ctx = nullptr;
    s->evfree.push_back(r.ev);
    r.ev = nullptr;
    s->pin.give(r.pin_off, r.pin_bytes);
    s->arena.give(r.off, r.bytes);
    --s->lane_busy[r.stream];
    --s->in_flight;
}

// Admit queued requests in order while they fit: batch-lane ones get |0...0> tableaux and
// cleared records (run at the next launch), shared-lane ones are enqueued whole.
int srv_admit(stab_server* s)
{
    std::vector<BatchCirc> init;
    std::vector<std::pair<size_t, size_t>> clear;   // record byte ranges
    while (!s->queue.empty()) {
        SrvRequest& r = s->queue.front();
        size_t off = 0;
        if (r.shared) {
            size_t pin_off = 0;
            if (!s->pin.take(r.pin_bytes, &pin_off)) break;
            if (!s->arena.take(r.bytes, &off)) {
                s->pin.give(pin_off, r.pin_bytes);
                break;
            }
            r.off = off;
            r.pin_off = pin_off;
            s->resident.push_back(std::move(r));
            s->queue.pop_front();
            const int rc = srv_launch_shared(s, s->resident.back());
            if (rc) return rc;
            continue;
        }
        if (!s->arena.take(r.bytes, &off)) break;
        r.off = off;
        r.rec_off = off + (size_t)r.shots * srv_shot_bytes(s->progs[r.prog].n, s->progs[r.prog].kfast);
        for (int sh = 0; sh < r.shots; ++sh) init.push_back(srv_circ(s, r, sh, 0));
        clear.push_back({r.rec_off, r.off + r.bytes - r.rec_off});
        s->resident.push_back(std::move(r));
        s->queue.pop_front();
    }
    if (init.empty()) return STAB_OK;
    int rc = ensure(s->d_init, init.size() * sizeof(BatchCirc));
    if (rc) return rc;
    SHIP_CHECK(s, hipMemcpyAsync(s->d_init.p, init.data(), init.size() * sizeof(BatchCirc), hipMemcpyHostToDevice,
                                 s->stream));
    k_batch_init<<<(unsigned)init.size(), 256, 0, s->stream>>>((const BatchCirc*)s->d_init.p, (uint64_t*)s->base,
                                                               (uint64_t*)s->base);
    SHIP_CHECK(s, hipGetLastError());
    for (const auto& c : clear) {
        const long long words = (long long)(c.second / 4);
        if (words > 0) {
            k_zero32<<<(unsigned)std::min<long long>((words + 255) / 256, 1024), 256, 0, s->stream>>>(
                (uint32_t*)(s->base + c.first), words);
            SHIP_CHECK(s, hipGetLastError());
        }
    }
    // the init table must stay valid until the kernels ran
    SHIP_CHECK(s, hipStreamSynchronize(s->stream));
    return STAB_OK;
}

// Retire the shared-lane requests whose completion event has fired.
int srv_retire_shared(stab_server* s, int* nfin)
{
    for (size_t i = 0; i < s->resident.size();) {
        SrvRequest& r = s->resident[i];
        if (!r.shared) {
            ++i;
            continue;
        }
        const hipError_t q = hipEventQuery(r.ev);
        if (q == hipErrorNotReady) {
            (void)hipGetLastError();   // (not an error: leave nothing behind for later checks)
            ++i;
            continue;
        }
        SHIP_CHECK(s, q);
        SrvProgram& G = s->progs[r.prog];
        const char* pin = s->pinned + r.pin_off;
        const size_t rec_b = (size_t)r.shots * (size_t)((r.P.nrec + 7) / 8);
        int err = 0;
        std::memcpy(&err, pin + align256(rec_b), sizeof(int));
        if (err) {
            s->poisoned = true;
            return fail(STAB_EINTERNAL, "device consistency check failed (code " + std::to_string(err) + ")");
        }
        if (r.learn) {
            G.mran.assign(r.P.meas.size(), 1);
            std::memcpy(G.mran.data(), pin + align256(rec_b) + 256, r.P.meas.size() * 4);
            G.mran_known = true;
            G.mran_pending = false;
        }
        if (!r.cancelled) r.result.assign(pin, pin + rec_b);
        srv_release_shared(s, r);
        if (!r.cancelled) {
            s->finished.push_back(r.id);
            const int64_t id = r.id;
            s->done.emplace(id, std::move(r));
            ++s->completed;
            ++*nfin;
        }
        s->resident.erase(s->resident.begin() + (long)i);
    }
    return STAB_OK;
}

// One launch of the batch kernel over every unfinished batch-lane shot, then the retirement of
// the batch-lane requests that finished.  A launch advances each shot by one measurement step,
// or by kSrvIdleQuota of them while no request waits for admission (fewer launches and host
// round trips per request; a request that arrives meanwhile waits up to that many rounds).
int srv_batch_step(stab_server* s, int* nfin)
{
    const int quota = s->queue.empty() ? kSrvIdleQuota : 1;
    std::vector<BatchCirc> circ;
    std::vector<ulonglong2> keys;
    int maxwc = 1;
    for (auto& r : s->resident) {
        if (r.shared) continue;
        for (int sh = 0; sh < r.shots; ++sh) {
            if (r.cursor[sh] >= s->progs[r.prog].nsteps) continue;
            circ.push_back(srv_circ(s, r, sh, r.cursor[sh]));
            ulonglong2 k;
            k.x = r.seed;
            k.y = (uint64_t)sh;
            keys.push_back(k);
            maxwc = std::max(maxwc, circ.back().Wc);
        }
    }
    const int nc = (int)circ.size();
    int rc;
    if (nc > 0) {
        std::vector<int> order(nc);
        for (int i = 0; i < nc; ++i) order[i] = reverse_blocks() ? nc - 1 - i : i;
        std::vector<uint64_t> ib(nc, 0ull);
        if ((rc = ensure(s->d_circ, (size_t)nc * sizeof(BatchCirc))) || (rc = ensure(s->d_order, (size_t)nc * 4)) ||
            (rc = ensure(s->d_keys, (size_t)nc * sizeof(ulonglong2))) || (rc = ensure(s->d_ibase, (size_t)nc * 8)))
            return rc;
        SHIP_CHECK(s, hipMemcpyAsync(s->d_circ.p, circ.data(), (size_t)nc * sizeof(BatchCirc), hipMemcpyHostToDevice,
                                     s->stream));
        SHIP_CHECK(s, hipMemcpyAsync(s->d_order.p, order.data(), (size_t)nc * 4, hipMemcpyHostToDevice, s->stream));
        SHIP_CHECK(s, hipMemcpyAsync(s->d_keys.p, keys.data(), (size_t)nc * sizeof(ulonglong2), hipMemcpyHostToDevice,
                                     s->stream));
        SHIP_CHECK(s, hipMemcpyAsync(s->d_ibase.p, ib.data(), (size_t)nc * 8, hipMemcpyHostToDevice, s->stream));
        BatchArgs A{};
        A.circ = (const BatchCirc*)s->d_circ.p;
        A.order = (const int*)s->d_order.p;
        A.steps = s->steps.dev;
        A.gates = s->gates.dev;
        A.noise = s->noise.dev;
        A.noise_tg = s->noise_tg.dev;
        A.meas = s->meas.dev;
        A.meas_tg = s->meas_tg.dev;
        A.tab = (uint64_t*)s->base;
        A.rs = (uint64_t*)s->base;
        A.rec = (uint32_t*)s->base;
        A.ibase = (const uint64_t*)s->d_ibase.p;
        A.keys = (const ulonglong2*)s->d_keys.p;
        A.cols = (uint64_t*)s->base;
        A.meas_quota = quota;
        A.seed = 0;
        A.err = s->d_err;
        A.counters = s->d_counters;
        const size_t lds = (size_t)batch_lds_words(maxwc) * 8;
        if (maxwc <= 64) k_batch<1, 4><<<nc, kBatchThreads, lds, s->stream>>>(A);
        else k_batch<2, 4><<<nc, kBatchThreads, lds, s->stream>>>(A);
        SHIP_CHECK(s, hipGetLastError());
        int err = 0;
        SHIP_CHECK(s, hipMemcpyAsync(&err, s->d_err, sizeof(int), hipMemcpyDeviceToHost, s->stream));
        SHIP_CHECK(s, hipStreamSynchronize(s->stream));
        if (err) {
            s->poisoned = true;
            return fail(STAB_EINTERNAL, "device consistency check failed");
        }
        ++s->iterations;
    }
    // the kernel ran each shot to just after its next `quota` measurement steps (or to the end)
    for (size_t i = 0; i < s->resident.size();) {
        SrvRequest& r = s->resident[i];
        if (r.shared) {
            ++i;
            continue;
        }
        const SrvProgram& P = s->progs[r.prog];
        for (int sh = 0; sh < r.shots && nc > 0; ++sh) {
            int& cur = r.cursor[sh];
            if (cur >= P.nsteps) continue;
            for (int q = 0; q < quota && cur < P.nsteps; ++q) {
                while (cur < P.nsteps && s->steps.host[P.step_base + cur].x != 2) ++cur;
                if (cur < P.nsteps) ++cur;
            }
            if (cur >= P.nsteps) --r.remaining;
        }
        if (r.remaining == 0) {
            r.result.resize((size_t)r.shots * (size_t)((P.nrec + 7) / 8));
            if (!r.result.empty())
                SHIP_CHECK(s, hipMemcpy(r.result.data(), s->base + r.rec_off, r.result.size(), hipMemcpyDeviceToHost));
            s->arena.give(r.off, r.bytes);
            s->finished.push_back(r.id);
            const int64_t id = r.id;
            s->done.emplace(id, std::move(r));
            s->resident.erase(s->resident.begin() + (long)i);
            ++s->completed;
            ++*nfin;
        } else {
            ++i;
        }
    }
    return STAB_OK;
}

// Arena and pinned bytes of a request of `shots` shots of program `prog` in its lane.
int srv_request_size(stab_server* s, int prog, int shots, bool* shared, int* bucket, size_t* bytes,
                     size_t* pin_bytes)
{
    SrvProgram& P = s->progs[prog];
    *shared = srv_shared_lane(P);
    *bucket = 0;
    *pin_bytes = 0;
    if (*shared) {
        SrvVariant* V = nullptr;
        const int b = shot_bucket(shots);
        const int rc = srv_variant(s, prog, b, &V);
        if (rc == STAB_OK) {
            *bucket = b;
            *bytes = V->tab_bytes + V->scratch_bytes;
            *pin_bytes = srv_pin_bytes(V->plan, shots);
            return STAB_OK;
        }
        // a stream the shared kernels cannot take (too many shots per copy) goes to the batch
        // lane unless the shared lane was asked for
        if (P.lane == STAB_LANE_SHARED || rc != STAB_ERANGE || s->poisoned) return rc;
        *shared = false;
    }
    *bytes = srv_request_bytes(P.n, P.kfast, shots, P.nrec);
    return STAB_OK;
}

}  // namespace

extern "C" {

int stab_server_request_bytes(const stab_server* s, int32_t prog, int32_t shots, uint64_t* bytes_out)
{
    if (!s || !bytes_out || shots < 1) return fail(STAB_EINVAL, "bad arguments");
    if (prog < 0 || prog >= (int32_t)s->progs.size()) return fail(STAB_EINVAL, "unknown program");
    if (s->poisoned) return fail(STAB_EDEVICE, "server poisoned by an earlier device error");
    bool shared = false;
    int bucket = 0;
    size_t bytes = 0, pin = 0;
    // (the server is logically unchanged: the shared-mode compile is a cache)
    const int rc = srv_request_size(const_cast<stab_server*>(s), prog, shots, &shared, &bucket, &bytes, &pin);
    if (rc) return rc;
    *bytes_out = bytes;
    return STAB_OK;
}

int stab_server_create(void* dev_buf, uint64_t buf_bytes, void* hip_stream, stab_server** out)
{
    if (!out) return fail(STAB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!dev_buf || buf_bytes < 256) return fail(STAB_EINVAL, "need a device arena");
    if (((uintptr_t)dev_buf & 255u) != 0) return fail(STAB_EINVAL, "dev_buf must be 256-byte aligned");
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return fail(STAB_EDEVICE, "no HIP device");
    stab_server* s = new stab_server();
    s->stream = (hipStream_t)hip_stream;
    s->base = (char*)dev_buf;
    s->bytes = (size_t)buf_bytes & ~(size_t)255;
    s->max_lds = lds;
    s->arena.reset(s->bytes);
    (void)hipFuncSetAttribute((const void*)k_batch<1, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_batch<2, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipGetLastError();
    bool ok = hipMalloc((void**)&s->d_err, sizeof(int)) == hipSuccess &&
              hipMalloc((void**)&s->d_counters, kNumCounters * kCounterStripes * sizeof(unsigned long long)) == hipSuccess &&
              hipMemset(s->d_err, 0, sizeof(int)) == hipSuccess &&
              hipMemset(s->d_counters, 0, kNumCounters * kCounterStripes * sizeof(unsigned long long)) == hipSuccess;
    // the shared lane's streams (default priority; they do not wait for the null stream)
    for (int k = 0; k < kSrvStreams && ok; ++k)
        ok = hipStreamCreateWithFlags(&s->lanes[k], hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        stab_server_destroy(s);
        return fail(STAB_ENOMEM, "device allocation failed");
    }
    *out = s;
    return STAB_OK;
}

void stab_server_destroy(stab_server* s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    else (void)hipDeviceSynchronize();
    for (hipStream_t st : s->lanes)
        if (st) (void)hipStreamSynchronize(st);
    for (SrvRequest& r : s->resident) {
        if (!r.shared || !r.ctx) continue;
        delete r.ctx;
        if (r.ev) (void)hipEventDestroy(r.ev);
    }
    for (hipEvent_t e : s->evfree) (void)hipEventDestroy(e);
    for (hipStream_t st : s->lanes)
        if (st) (void)hipStreamDestroy(st);
    for (SrvProgram& P : s->progs)
        for (auto& v : P.variants)
            if (v.second->plan.dev) (void)hipFree(v.second->plan.dev);
    if (s->pinned) (void)hipHostFree(s->pinned);
    for (void* p : {(void*)s->steps.dev, (void*)s->gates.dev, (void*)s->noise.dev, (void*)s->noise_tg.dev,
                    (void*)s->meas.dev, (void*)s->meas_tg.dev, s->d_circ.p, s->d_order.p, s->d_keys.p,
                    s->d_ibase.p, s->d_init.p, (void*)s->d_err, (void*)s->d_counters})
        if (p) (void)hipFree(p);
    delete s;
}

int stab_server_program(stab_server* s, const stab_instr* instrs, int32_t ninstr, const int32_t* targets,
                        int64_t ntargets, int32_t n, int32_t* prog_out)
{
    if (!s || !prog_out) return fail(STAB_EINVAL, "NULL argument");
    if (s->poisoned) return fail(STAB_EDEVICE, "server poisoned by an earlier device error");
    if (n < 1 || ninstr < 0 || ntargets < 0) return fail(STAB_EINVAL, "bad sizes");
    if ((n + 63) / 64 > kBatchMaxWc) return fail(STAB_ERANGE, "more qubits than a batch supports");
    if (batch_lds_words((n + 63) / 64) * 8 > s->max_lds) return fail(STAB_ERANGE, "circuit too large for LDS");
    if ((ninstr > 0 && !instrs) || (ntargets > 0 && !targets)) return fail(STAB_EINVAL, "null stream");
    SrvProgram P;
    P.n = n;
    P.ninstr = ninstr;
    P.step_base = (int)s->steps.host.size();
    const size_t g0 = s->gates.host.size(), n0 = s->noise.host.size(), nt0 = s->noise_tg.host.size(),
                 m0 = s->meas.host.size(), mt0 = s->meas_tg.host.size();
    long long nrec = 0;
    int kfast = 0;
    const int rc = batch_compile_one(0, n, instrs, ninstr, targets, ntargets, s->steps.host, s->gates.host,
                                     s->noise.host, s->noise_tg.host, s->meas.host, s->meas_tg.host, nrec, kfast);
    if (rc) {
        s->steps.host.resize(P.step_base);
        s->gates.host.resize(g0);
        s->noise.host.resize(n0);
        s->noise_tg.host.resize(nt0);
        s->meas.host.resize(m0);
        s->meas_tg.host.resize(mt0);
        return rc;
    }
    P.nsteps = (int)s->steps.host.size() - P.step_base;
    P.nrec = nrec;
    P.kfast = kfast;
    // the shared lane compiles its own plan from the stream
    P.instrs.assign(instrs, instrs + ninstr);
    P.targets.assign(targets, targets + ntargets);
    for (int32_t k = 0; k < ninstr; ++k)
        if (instrs[k].kind == STAB_T1T2) P.pauli_only = false;
    int rc2;
    if ((rc2 = devvec_sync(s->steps, s->stream)) || (rc2 = devvec_sync(s->gates, s->stream)) ||
        (rc2 = devvec_sync(s->noise, s->stream)) || (rc2 = devvec_sync(s->noise_tg, s->stream)) ||
        (rc2 = devvec_sync(s->meas, s->stream)) || (rc2 = devvec_sync(s->meas_tg, s->stream))) {
        s->poisoned = true;
        return rc2;
    }
    s->progs.push_back(std::move(P));
    *prog_out = (int32_t)s->progs.size() - 1;
    return STAB_OK;
}

int stab_server_set_lane(stab_server* s, int32_t prog, int32_t lane)
{
    if (!s) return fail(STAB_EINVAL, "server is NULL");
    if (prog < 0 || prog >= (int32_t)s->progs.size()) return fail(STAB_EINVAL, "unknown program");
    if (lane != STAB_LANE_AUTO && lane != STAB_LANE_BATCH && lane != STAB_LANE_SHARED)
        return fail(STAB_EINVAL, "lane must be STAB_LANE_AUTO, STAB_LANE_BATCH or STAB_LANE_SHARED");
    if (lane == STAB_LANE_SHARED && !s->progs[prog].pauli_only)
        return fail(STAB_EINVAL, "a stream with T1T2 noise changes x|z shot by shot: it runs in the batch lane");
    s->progs[prog].lane = lane;
    return STAB_OK;
}

int64_t stab_server_program_records(const stab_server* s, int32_t prog)
{
    if (!s || prog < 0 || prog >= (int32_t)s->progs.size()) return -1;
    return s->progs[prog].nrec;
}

int stab_server_submit(stab_server* s, int32_t prog, int32_t shots, uint64_t seed, int64_t* id_out)
{
    if (!s || !id_out) return fail(STAB_EINVAL, "NULL argument");
    if (s->poisoned) return fail(STAB_EDEVICE, "server poisoned by an earlier device error");
    if (prog < 0 || prog >= (int32_t)s->progs.size()) return fail(STAB_EINVAL, "unknown program");
    if (shots < 1) return fail(STAB_EINVAL, "shots < 1");
    SrvRequest r;
    int rc = srv_request_size(s, prog, shots, &r.shared, &r.bucket, &r.bytes, &r.pin_bytes);
    if (rc) return rc;
    if (r.bytes > s->bytes) return fail(STAB_ERANGE, "request larger than the whole arena");
    if (r.shared) {
        if (r.pin_bytes > kSrvPinnedBytes) return fail(STAB_ERANGE, "request records larger than the pinned staging");
        if (!s->pinned) {
            if (hipHostMalloc((void**)&s->pinned, kSrvPinnedBytes, hipHostMallocDefault) != hipSuccess) {
                s->pinned = nullptr;
                (void)hipGetLastError();
                return fail(STAB_ENOMEM, "pinned host allocation failed");
            }
            s->pin.reset(kSrvPinnedBytes);
        }
    }
    const SrvProgram& P = s->progs[prog];
    r.id = s->next_id++;
    r.prog = prog;
    r.shots = shots;
    r.seed = seed;
    if (!r.shared) {
        r.cursor.assign(shots, 0);
        r.remaining = P.nsteps == 0 ? 0 : shots;
    }
    s->queue.push_back(std::move(r));
    *id_out = s->queue.back().id;
    return STAB_OK;
}

int stab_server_step(stab_server* s, int32_t* finished_out)
{
    if (!s) return fail(STAB_EINVAL, "server is NULL");
    if (s->poisoned) return fail(STAB_EDEVICE, "server poisoned by an earlier device error");
    if (finished_out) *finished_out = 0;
    int nfin = 0;
    int rc;
    if ((rc = srv_retire_shared(s, &nfin)) || (rc = srv_admit(s)) || (rc = srv_batch_step(s, &nfin))) return rc;
    if (finished_out) *finished_out = nfin;
    return STAB_OK;
}

int stab_server_cancel(stab_server* s, int64_t id)
{
    if (!s) return fail(STAB_EINVAL, "server is NULL");
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
        if (it->id != id) continue;
        s->queue.erase(it);
        ++s->cancelled;
        return STAB_OK;
    }
    for (size_t i = 0; i < s->resident.size(); ++i) {
        SrvRequest& r = s->resident[i];
        if (r.id != id) continue;
        if (r.cancelled) break;
        if (r.shared) {
            // its launches are in flight: its blocks are freed when its event fires
            r.cancelled = true;
        } else {
            // (no batch launch is in flight between calls)
            s->arena.give(r.off, r.bytes);
            s->resident.erase(s->resident.begin() + (long)i);
        }
        ++s->cancelled;
        return STAB_OK;
    }
    const auto d = s->done.find(id);
    if (d != s->done.end()) {
        s->done.erase(d);
        for (auto f = s->finished.begin(); f != s->finished.end(); ++f)
            if (*f == id) {
                s->finished.erase(f);
                break;
            }
        ++s->cancelled;
        return STAB_OK;
    }
    return fail(STAB_EINVAL, "unknown request (or already cancelled or taken)");
}

int stab_server_poll(stab_server* s, int64_t* ids, int32_t max_ids)
{
    if (!s || (!ids && max_ids > 0) || max_ids < 0) return fail(STAB_EINVAL, "bad arguments");
    int k = 0;
    while (k < max_ids && !s->finished.empty()) {
        ids[k++] = s->finished.front();
        s->finished.pop_front();
    }
    return k;
}

int64_t stab_server_records(const stab_server* s, int64_t id)
{
    if (!s) return -1;
    const auto it = s->done.find(id);
    if (it == s->done.end()) return -1;
    return s->progs[it->second.prog].nrec;
}

int stab_server_result(stab_server* s, int64_t id, uint8_t* out_bits)
{
    if (!s) return fail(STAB_EINVAL, "server is NULL");
    auto it = s->done.find(id);
    if (it == s->done.end()) return fail(STAB_EINVAL, "request not finished (or already taken)");
    if (!it->second.result.empty()) {
        if (!out_bits) return fail(STAB_EINVAL, "out_bits is NULL");
        std::memcpy(out_bits, it->second.result.data(), it->second.result.size());
    }
    s->done.erase(it);
    return STAB_OK;
}

int stab_server_stats(const stab_server* s, int64_t* out, int32_t nout)
{
    if (!s || !out || nout < 0 || nout > 9) return fail(STAB_EINVAL, "bad arguments");
    long long shots = 0;
    for (const auto& r : s->resident) shots += r.shared ? r.shots : r.remaining;
    const int64_t v[9] = {(int64_t)s->queue.size(), (int64_t)s->resident.size(), (int64_t)shots,
                          (int64_t)s->arena.in_use, (int64_t)s->bytes, (int64_t)s->iterations, (int64_t)s->completed,
                          (int64_t)s->in_flight, (int64_t)s->cancelled};
    for (int i = 0; i < nout; ++i) out[i] = v[i];
    return STAB_OK;
}

}  // extern "C"
