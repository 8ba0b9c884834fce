// stab_server_api.hip -- continuous batching of sampling requests (include/stab.h,
// stab_server_*).  Included at the end of stab_api.hip, after the batch code it runs on.
//
// A request is an op stream with a shot count and a seed.  Each of its shots is one circuit of
// the batch kernel (its own tableau, RNG key (seed, shot)), so a request's records are exactly
// those of a full-mode context and do not depend on what else is resident.  Requests are
// admitted in arrival order while their bytes (tableaux, signs, records) fit in the caller's
// arena; every step() runs one launch that advances every resident shot by one measurement
// step (a round of a memory experiment), so rounds of all resident requests share each
// launch, new requests join at the next step and finished ones leave.  Streams are compiled
// and uploaded once (stab_server_program) and submitted by program id.

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

struct SrvProgram {
    int n = 0;
    long long nrec = 0;
    int ninstr = 0;
    int step_base = 0, nsteps = 0;
    int kfast = 0;                // column scratch targets per band
};

struct SrvRequest {
    int64_t id = 0;
    int prog = 0;
    int shots = 0;
    uint64_t seed = 0;
    size_t off = 0, bytes = 0;    // arena block
    size_t rec_off = 0;           // byte offset of the records inside the arena
    std::vector<int> cursor;      // per shot: next program step
    int remaining = 0;            // shots not finished
    std::vector<uint8_t> result;
};

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
    std::map<size_t, size_t> free_blocks;            // offset -> size
    size_t in_use = 0;
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
    long long iterations = 0, completed = 0;
    // per-step device tables
    DevBuf d_circ, d_order, d_keys, d_ibase, d_init;
    int* d_err = nullptr;
    unsigned long long* d_counters = nullptr;
};

namespace {

bool srv_alloc(stab_server* s, size_t bytes, size_t* off)
{
    for (auto it = s->free_blocks.begin(); it != s->free_blocks.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            s->free_blocks.erase(it);
            if (rest) s->free_blocks[at] = rest;
            s->in_use += bytes;
            return true;
        }
    }
    return false;
}

void srv_free(stab_server* s, size_t off, size_t bytes)
{
    s->in_use -= bytes;
    auto it = s->free_blocks.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != s->free_blocks.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        s->free_blocks.erase(nx);
    }
    if (it != s->free_blocks.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            s->free_blocks.erase(it);
        }
    }
}

// Circuit table entry of shot `shot` of request r starting at program step `cursor`.
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

#define SHIP_CHECK(s, call)                                                                    \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            (s)->poisoned = true;                                                              \
            return fail(STAB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
        }                                                                                      \
    } while (0)

// Admit queued requests in order while they fit: place them, set their tableaux to |0...0>
// and clear their records.
int srv_admit(stab_server* s)
{
    std::vector<BatchCirc> init;
    std::vector<std::pair<size_t, size_t>> clear;   // record byte ranges
    while (!s->queue.empty()) {
        SrvRequest& r = s->queue.front();
        size_t off = 0;
        if (!srv_alloc(s, r.bytes, &off)) break;
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

}  // namespace

extern "C" {

int stab_server_request_bytes(const stab_server* s, int32_t prog, int32_t shots, uint64_t* bytes_out)
{
    if (!s || !bytes_out || shots < 1) return fail(STAB_EINVAL, "bad arguments");
    if (prog < 0 || prog >= (int32_t)s->progs.size()) return fail(STAB_EINVAL, "unknown program");
    const SrvProgram& P = s->progs[prog];
    *bytes_out = srv_request_bytes(P.n, P.kfast, shots, P.nrec);
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
    s->free_blocks[0] = s->bytes;
    (void)hipFuncSetAttribute((const void*)k_batch<1, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_batch<2, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipGetLastError();
    if (hipMalloc((void**)&s->d_err, sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&s->d_counters, kNumCounters * kCounterStripes * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(s->d_err, 0, sizeof(int)) != hipSuccess ||
        hipMemset(s->d_counters, 0, kNumCounters * kCounterStripes * sizeof(unsigned long long)) != hipSuccess) {
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
    int rc2;
    if ((rc2 = devvec_sync(s->steps, s->stream)) || (rc2 = devvec_sync(s->gates, s->stream)) ||
        (rc2 = devvec_sync(s->noise, s->stream)) || (rc2 = devvec_sync(s->noise_tg, s->stream)) ||
        (rc2 = devvec_sync(s->meas, s->stream)) || (rc2 = devvec_sync(s->meas_tg, s->stream))) {
        s->poisoned = true;
        return rc2;
    }
    s->progs.push_back(P);
    *prog_out = (int32_t)s->progs.size() - 1;
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
    const SrvProgram& P = s->progs[prog];
    const size_t bytes = srv_request_bytes(P.n, P.kfast, shots, P.nrec);
    if (bytes > s->bytes) return fail(STAB_ERANGE, "request larger than the whole arena");
    SrvRequest r;
    r.id = s->next_id++;
    r.prog = prog;
    r.shots = shots;
    r.seed = seed;
    r.bytes = bytes;
    r.cursor.assign(shots, 0);
    r.remaining = shots;
    if (P.nsteps == 0) r.remaining = 0;
    s->queue.push_back(std::move(r));
    *id_out = s->queue.back().id;
    return STAB_OK;
}

int stab_server_step(stab_server* s, int32_t* finished_out)
{
    if (!s) return fail(STAB_EINVAL, "server is NULL");
    if (s->poisoned) return fail(STAB_EDEVICE, "server poisoned by an earlier device error");
    if (finished_out) *finished_out = 0;
    int rc = srv_admit(s);
    if (rc) return rc;
    // one launch: every unfinished resident shot advances by one measurement step
    std::vector<BatchCirc> circ;
    std::vector<ulonglong2> keys;
    int maxwc = 1;
    for (auto& r : s->resident) {
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
        A.meas_quota = 1;
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
    // the kernel ran each shot to just after its next measurement step (or to the end)
    int nfin = 0;
    for (size_t i = 0; i < s->resident.size();) {
        SrvRequest& r = s->resident[i];
        const SrvProgram& P = s->progs[r.prog];
        for (int sh = 0; sh < r.shots && nc > 0; ++sh) {
            int& cur = r.cursor[sh];
            if (cur >= P.nsteps) continue;
            while (cur < P.nsteps && s->steps.host[P.step_base + cur].x != 2) ++cur;
            if (cur < P.nsteps) ++cur;
            if (cur >= P.nsteps) --r.remaining;
        }
        if (r.remaining == 0) {
            r.result.resize((size_t)r.shots * (size_t)((P.nrec + 7) / 8));
            if (!r.result.empty())
                SHIP_CHECK(s, hipMemcpy(r.result.data(), s->base + r.rec_off, r.result.size(), hipMemcpyDeviceToHost));
            srv_free(s, r.off, r.bytes);
            s->finished.push_back(r.id);
            const int64_t id = r.id;
            s->done.emplace(id, std::move(r));
            s->resident.erase(s->resident.begin() + (long)i);
            ++s->completed;
            ++nfin;
        } else {
            ++i;
        }
    }
    if (finished_out) *finished_out = nfin;
    return STAB_OK;
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
    if (!s || !out || nout < 0 || nout > 7) return fail(STAB_EINVAL, "bad arguments");
    long long circs = 0;
    for (const auto& r : s->resident) circs += r.remaining;
    const int64_t v[7] = {(int64_t)s->queue.size(), (int64_t)s->resident.size(), (int64_t)circs,
                          (int64_t)s->in_use, (int64_t)s->bytes, (int64_t)s->iterations, (int64_t)s->completed};
    for (int i = 0; i < nout; ++i) out[i] = v[i];
    return STAB_OK;
}

}  // extern "C"
