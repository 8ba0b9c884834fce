// stab_batch_api.hip -- host side of the multi-circuit batch (include/stab.h, stab_batch_*).
// Included at the end of stab_api.hip: it uses that file's error, buffer and stream helpers.

struct stab_batch {
    int ncirc = 0;
    std::vector<BatchCirc> circ;     // geometry and storage offsets (no program fields)
    uint64_t seed = 0;
    hipStream_t stream = nullptr;
    uint64_t* tab = nullptr;
    uint64_t* rs = nullptr;
    BatchCirc* d_circ = nullptr;
    int* d_err = nullptr;
    unsigned long long* d_counters = nullptr;
    int max_lds = 0;
    bool poisoned = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    DevBuf rec;
    uint64_t* d_ibase = nullptr;      // per-circuit instruction counters (device copy)
    std::vector<uint64_t> icount;     // instructions each circuit has executed
    double kernel_ms = 0.0;           // batch kernel time of the last execution
    size_t bytes = 0;                 // tableaux and signs in dev_buf
};

struct stab_batch_program {
    int ncirc = 0;
    std::vector<int> n;               // circuit sizes it was compiled for
    std::vector<long long> nrec;      // records per circuit
    std::vector<long long> ninstr;    // instructions per circuit
    std::vector<long long> rec_byte;  // first output byte per circuit (ncirc + 1 entries)
    int lds_bytes = 0;
    int nw = 1;                       // x words per lane (kernel variant)
    int tile = 0;                     // launch configuration (BatchArgs::tile)
    uint64_t shape = 0;               // fingerprint of the program's shape (autotuner cache key)
    void* dev = nullptr;
    uint64_t* cols = nullptr;         // column scratch of every circuit
    BatchCirc* d_circ = nullptr;
    int* d_order = nullptr;
    int4* d_steps = nullptr;
    uint2* d_gates = nullptr;
    NoiseDesc* d_noise = nullptr;
    int* d_noise_tg = nullptr;
    BatchMeas* d_meas = nullptr;
    int* d_meas_tg = nullptr;
};

namespace {

struct BatchLayout {
    std::vector<long long> tab_off, rs_off;
    size_t bytes = 0;
};

int batch_layout(int32_t ncirc, const int32_t* n, BatchLayout& L)
{
    if (ncirc < 1 || !n) return fail(STAB_EINVAL, "need at least one circuit and its sizes");
    L.tab_off.resize(ncirc);
    L.rs_off.resize(ncirc);
    size_t words = 0;
    for (int c = 0; c < ncirc; ++c) {
        if (n[c] < 1) return fail(STAB_EINVAL, "circuit " + std::to_string(c) + ": n < 1");
        const int Wc = (n[c] + 63) / 64;
        if (Wc > kBatchMaxWc) return fail(STAB_ERANGE, "circuit " + std::to_string(c) + ": more qubits than a batch supports");
        L.tab_off[c] = (long long)words;
        words += align256((size_t)2 * 64 * Wc * 2 * Wc * 8) / 8;
    }
    for (int c = 0; c < ncirc; ++c) {
        L.rs_off[c] = (long long)words;
        words += align256((size_t)2 * ((n[c] + 63) / 64) * 8) / 8;
    }
    L.bytes = words * 8;
    return STAB_OK;
}

#define BHIP_CHECK(b, call)                                                                    \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            (b)->poisoned = true;                                                              \
            return fail(STAB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
        }                                                                                      \
    } while (0)

int batch_init(stab_batch* b)
{
    std::fill(b->icount.begin(), b->icount.end(), 0ull);
    k_batch_init<<<b->ncirc, 256, 0, b->stream>>>(b->d_circ, b->tab, b->rs);
    BHIP_CHECK(b, hipGetLastError());
    BHIP_CHECK(b, hipMemsetAsync(b->d_err, 0, sizeof(int), b->stream));
    return STAB_OK;
}

// Compile circuit c's stream into program steps (gate layers on disjoint qubits, noise
// layers, measurement instructions); validation as for a single context.
int batch_compile_one(int c, int n, const stab_instr* ins, int64_t ninstr, const int32_t* tg, int64_t ntg,
                      std::vector<int4>& steps, std::vector<uint2>& gates, std::vector<NoiseDesc>& noise,
                      std::vector<int>& noise_tg, std::vector<BatchMeas>& meas, std::vector<int>& meas_tg,
                      long long& nrec, int& kfast)
{
    const std::string where = "circuit " + std::to_string(c) + ", instruction ";
    std::vector<int> stamp(n, -1), mstamp(n, -1);
    kfast = 0;
    int layer_id = 0, open_begin = -1, open_mod = 0;
    auto close_layer = [&]() {
        if (open_begin >= 0) {
            const int cnt = (int)gates.size() - open_begin;
            if (cnt > 0) steps.push_back(make_int4(0, open_begin, cnt, open_mod));
            open_begin = -1;
            open_mod = 0;
        }
        ++layer_id;
    };
    nrec = 0;
    int64_t off = 0;
    for (int64_t k = 0; k < ninstr; ++k) {
        const uint32_t kind = ins[k].kind, nt = ins[k].ntargets;
        if (!valid_kind(kind)) return fail(STAB_EINVAL, where + std::to_string(k) + ": unknown kind");
        if (off + (int64_t)nt > ntg) return fail(STAB_EINVAL, where + std::to_string(k) + ": targets run past the target array");
        if ((kind == STAB_CX || kind == STAB_DEP2) && (nt & 1u))
            return fail(STAB_EINVAL, where + std::to_string(k) + ": odd target count for a two-qubit kind");
        const int32_t* t = tg + off;
        for (uint32_t q = 0; q < nt; ++q)
            if (t[q] < 0 || t[q] >= n)
                return fail(STAB_EINVAL, where + std::to_string(k) + ": target " + std::to_string(t[q]) + " out of range");
        switch (kind) {
        case STAB_TICK:
            break;
        case STAB_H: case STAB_S: case STAB_X: case STAB_Y: case STAB_Z:
            for (uint32_t q = 0; q < nt; ++q) {
                if (stamp[t[q]] == layer_id) close_layer();
                if (open_begin < 0) open_begin = (int)gates.size();
                stamp[t[q]] = layer_id;
                gates.push_back(make_uint2(kind | ((uint32_t)t[q] << 4), 0u));
                if (kind == STAB_H || kind == STAB_S) open_mod = 1;
            }
            break;
        case STAB_CX:
            for (uint32_t q = 0; q < nt; q += 2) {
                const int a = t[q], d = t[q + 1];
                if (a == d) return fail(STAB_EINVAL, where + std::to_string(k) + ": CX with equal qubits");
                if (stamp[a] == layer_id || stamp[d] == layer_id) close_layer();
                if (open_begin < 0) open_begin = (int)gates.size();
                stamp[a] = stamp[d] = layer_id;
                gates.push_back(make_uint2(kind | ((uint32_t)a << 4), (uint32_t)d));
                open_mod = 1;
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
            d.bucket = (int)noise.size();
            noise_tg.insert(noise_tg.end(), t, t + nt);
            steps.push_back(make_int4(1, (int)noise.size(), 0, 0));
            noise.push_back(d);
        } break;
        case STAB_M: case STAB_MR: case STAB_R: case STAB_T1T2: {
            close_layer();
            if (nt == 0) break;
            if (kind == STAB_T1T2 && ins[k].t1 < ins[k].t0)
                return fail(STAB_EINVAL, where + std::to_string(k) + ": T1T2 thresholds must not decrease");
            BatchMeas m{};
            m.instr = (uint64_t)k;
            m.t0 = ins[k].t0;
            m.t1 = ins[k].t1;
            m.kind = (int)kind;
            m.tq = (int)meas_tg.size();
            m.K = (int)nt;
            const bool recorded = kind == STAB_M || kind == STAB_MR;
            m.rec = recorded ? (int)nrec : -1;
            if (recorded) nrec += nt;
            // distinct qubits: its columns can come out of the band pass before it
            m.fast = kind != STAB_T1T2 ? 1 : 0;
            for (uint32_t q = 0; q < nt && m.fast; ++q) {
                if (mstamp[t[q]] == (int)k) m.fast = 0;
                mstamp[t[q]] = (int)k;
            }
            if (m.fast) kfast = std::max(kfast, (int)nt);
            meas_tg.insert(meas_tg.end(), t, t + nt);
            steps.push_back(make_int4(2, (int)meas.size(), 0, 0));
            meas.push_back(m);
        } break;
        default:
            return fail(STAB_EINVAL, "unknown kind");
        }
        off += nt;
    }
    if (off != ntg) return fail(STAB_EINVAL, where + "*: target array longer than the instructions consume");
    close_layer();
    if (gates.size() > (size_t)INT32_MAX || meas_tg.size() > (size_t)INT32_MAX || noise_tg.size() > (size_t)INT32_MAX ||
        nrec > INT32_MAX)
        return fail(STAB_ERANGE, "batch program too large");
    return STAB_OK;
}

}  // namespace

extern "C" {

int stab_batch_bytes(int32_t ncirc, const int32_t* n, uint64_t* bytes_out)
{
    if (!bytes_out) return fail(STAB_EINVAL, "bytes_out is NULL");
    BatchLayout L;
    const int rc = batch_layout(ncirc, n, L);
    if (rc) return rc;
    *bytes_out = L.bytes;
    return STAB_OK;
}

int stab_batch_create(int32_t ncirc, const int32_t* n, uint64_t seed, void* dev_buf, uint64_t buf_bytes,
                      void* hip_stream, stab_batch** out)
{
    if (!out) return fail(STAB_EINVAL, "out is NULL");
    *out = nullptr;
    BatchLayout L;
    int rc = batch_layout(ncirc, n, L);
    if (rc) return rc;
    if (!dev_buf) return fail(STAB_EINVAL, "dev_buf is NULL");
    if (((uintptr_t)dev_buf & 255u) != 0) return fail(STAB_EINVAL, "dev_buf must be 256-byte aligned");
    if (buf_bytes < L.bytes) return fail(STAB_ENOMEM, "dev_buf smaller than stab_batch_bytes()");
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return fail(STAB_EDEVICE, "no HIP device");
    for (int c = 0; c < ncirc; ++c)
        if (batch_lds_words((n[c] + 63) / 64) * 8 > lds)
            return fail(STAB_ERANGE, "circuit " + std::to_string(c) + ": a 64-row band does not fit in LDS");
    stab_batch* b = new stab_batch();
    b->ncirc = ncirc;
    b->seed = seed;
    b->stream = (hipStream_t)hip_stream;
    b->tab = (uint64_t*)dev_buf;
    b->rs = (uint64_t*)dev_buf;
    b->max_lds = lds;
    b->bytes = L.bytes;
    b->circ.resize(ncirc);
    b->icount.assign(ncirc, 0ull);
    for (int c = 0; c < ncirc; ++c) {
        BatchCirc& C = b->circ[c];
        C = BatchCirc{};
        C.n = n[c];
        C.Wc = (n[c] + 63) / 64;
        C.RS = 2 * C.Wc;
        C.NR = 64 * C.Wc;
        C.tab_off = L.tab_off[c];
        C.rs_off = L.rs_off[c];
    }
    (void)hipFuncSetAttribute((const void*)k_batch<1, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_batch<2, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_batch<1, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipFuncSetAttribute((const void*)k_batch<2, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    (void)hipGetLastError();
    const bool ok = hipMalloc((void**)&b->d_circ, sizeof(BatchCirc) * ncirc) == hipSuccess &&
                    hipMalloc((void**)&b->d_err, sizeof(int)) == hipSuccess &&
                    hipMalloc((void**)&b->d_ibase, sizeof(uint64_t) * ncirc) == hipSuccess &&
                    hipMalloc((void**)&b->d_counters, kNumCounters * kCounterStripes * sizeof(unsigned long long)) == hipSuccess &&
                    hipEventCreate(&b->ev0) == hipSuccess && hipEventCreate(&b->ev1) == hipSuccess;
    if (!ok) {
        stab_batch_destroy(b);
        return fail(STAB_ENOMEM, "device allocation failed");
    }
    if (hipMemcpy(b->d_circ, b->circ.data(), sizeof(BatchCirc) * ncirc, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(b->d_counters, 0, kNumCounters * kCounterStripes * sizeof(unsigned long long)) != hipSuccess) {
        stab_batch_destroy(b);
        return fail(STAB_EDEVICE, "device copy failed");
    }
    rc = batch_init(b);
    if (rc == STAB_OK && hipStreamSynchronize(b->stream) != hipSuccess) rc = fail(STAB_EDEVICE, "init failed");
    if (rc) {
        stab_batch_destroy(b);
        return rc;
    }
    *out = b;
    return STAB_OK;
}

void stab_batch_destroy(stab_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    else (void)hipDeviceSynchronize();
    if (b->d_circ) (void)hipFree(b->d_circ);
    if (b->d_err) (void)hipFree(b->d_err);
    if (b->d_ibase) (void)hipFree(b->d_ibase);
    if (b->d_counters) (void)hipFree(b->d_counters);
    if (b->rec.p) (void)hipFree(b->rec.p);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    delete b;
}

int stab_batch_reset(stab_batch* b, uint64_t seed)
{
    if (!b) return fail(STAB_EINVAL, "batch is NULL");
    if (b->poisoned) return fail(STAB_EDEVICE, "batch poisoned by an earlier device error");
    b->seed = seed;
    return batch_init(b);
}

int stab_batch_compile(stab_batch* b, const stab_instr* instrs, const int64_t* instr_off, const int32_t* targets,
                       const int64_t* target_off, stab_batch_program** out)
{
    if (!b || !out || !instr_off || !target_off) return fail(STAB_EINVAL, "NULL argument");
    *out = nullptr;
    const int C = b->ncirc;
    if (instr_off[0] != 0 || target_off[0] != 0) return fail(STAB_EINVAL, "offsets must start at 0");
    for (int c = 0; c < C; ++c)
        if (instr_off[c + 1] < instr_off[c] || target_off[c + 1] < target_off[c])
            return fail(STAB_EINVAL, "offsets must be non-decreasing");
    if ((instr_off[C] > 0 && !instrs) || (target_off[C] > 0 && !targets)) return fail(STAB_EINVAL, "null stream");
    std::vector<int4> steps;
    std::vector<uint2> gates;
    std::vector<NoiseDesc> noise;
    std::vector<int> noise_tg, meas_tg;
    std::vector<BatchMeas> meas;
    std::vector<BatchCirc> circ = b->circ;
    stab_batch_program* P = new stab_batch_program();
    P->ncirc = C;
    P->n.resize(C);
    P->nrec.resize(C);
    P->ninstr.resize(C);
    P->rec_byte.assign(C + 1, 0);
    std::vector<double> cost(C, 0.0);
    int maxwc = 1;
    size_t cols_words = 0;
    for (int c = 0; c < C; ++c) {
        const int s0 = (int)steps.size();
        long long nrec = 0;
        int kfast = 0;
        const int rc = batch_compile_one(c, circ[c].n, instrs + instr_off[c], instr_off[c + 1] - instr_off[c],
                                         targets + target_off[c], target_off[c + 1] - target_off[c], steps, gates,
                                         noise, noise_tg, meas, meas_tg, nrec, kfast);
        if (rc) {
            delete P;
            return rc;
        }
        circ[c].step_begin = s0;
        circ[c].step_count = (int)steps.size() - s0;
        circ[c].rec_bit_off = 8 * P->rec_byte[c];
        circ[c].col_k = kfast;
        circ[c].col_off = (long long)cols_words;
        cols_words += align256((size_t)2 * 2 * circ[c].Wc * kfast * 8) / 8;
        P->n[c] = circ[c].n;
        P->nrec[c] = nrec;
        P->ninstr[c] = instr_off[c + 1] - instr_off[c];
        P->rec_byte[c + 1] = P->rec_byte[c] + (nrec + 7) / 8;
        // work estimate: every measured target and every band pass touches ~the whole tableau
        const double tabw = 2.0 * circ[c].NR * circ[c].RS;
        long long mt = 0, runs = 0;
        for (int s = s0; s < (int)steps.size(); ++s) {
            if (steps[s].x == 2) mt += meas[steps[s].y].K;
            else if (s == s0 || steps[s - 1].x == 2) ++runs;
        }
        cost[c] = tabw * (double)(mt + runs);
        maxwc = std::max(maxwc, circ[c].Wc);
    }
    std::vector<int> order(C);
    for (int c = 0; c < C; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    if (reverse_blocks()) std::reverse(order.begin(), order.end());
    P->lds_bytes = batch_lds_words(maxwc) * 8;
    P->nw = maxwc <= 64 ? 1 : 2;
    // shape fingerprint: sizes and per-circuit step, gate and measured-target counts
    {
        uint64_t h = 0x9E3779B97F4A7C15ull ^ (uint64_t)C;
        auto mix = [&](uint64_t v) {
            h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
            h *= 0xff51afd7ed558ccdull;
        };
        for (int c = 0; c < C; ++c) {
            long long ng = 0, mt = 0;
            for (int st = circ[c].step_begin; st < circ[c].step_begin + circ[c].step_count; ++st) {
                if (steps[st].x == 0) ng += steps[st].z;
                else if (steps[st].x == 2) mt += meas[steps[st].y].K;
            }
            mix((uint64_t)circ[c].n);
            mix((uint64_t)circ[c].step_count);
            mix((uint64_t)ng);
            mix((uint64_t)mt);
        }
        P->shape = h;
    }

    std::vector<char> blob;
    const size_t o_circ = put(blob, circ), o_order = put(blob, order), o_steps = put(blob, steps),
                 o_gates = put(blob, gates), o_noise = put(blob, noise), o_ntg = put(blob, noise_tg),
                 o_meas = put(blob, meas), o_mtg = put(blob, meas_tg);
    if (hipMalloc(&P->dev, blob.size()) != hipSuccess) {
        P->dev = nullptr;
        delete P;
        return fail(STAB_ENOMEM, "device allocation failed");
    }
    if (cols_words > 0 && hipMalloc((void**)&P->cols, cols_words * 8) != hipSuccess) {
        P->cols = nullptr;
        stab_batch_program_destroy(P);
        return fail(STAB_ENOMEM, "device allocation failed");
    }
    if (hipMemcpy(P->dev, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
        stab_batch_program_destroy(P);
        b->poisoned = true;
        return fail(STAB_EDEVICE, "program upload failed");
    }
    char* base = (char*)P->dev;
    P->d_circ = (BatchCirc*)(base + o_circ);
    P->d_order = (int*)(base + o_order);
    P->d_steps = (int4*)(base + o_steps);
    P->d_gates = (uint2*)(base + o_gates);
    P->d_noise = (NoiseDesc*)(base + o_noise);
    P->d_noise_tg = (int*)(base + o_ntg);
    P->d_meas = (BatchMeas*)(base + o_meas);
    P->d_meas_tg = (int*)(base + o_mtg);
    *out = P;
    return STAB_OK;
}

int64_t stab_batch_program_records(const stab_batch_program* P, int32_t circuit)
{
    if (!P || circuit < 0 || circuit >= P->ncirc) return -1;
    return P->nrec[circuit];
}

void stab_batch_program_destroy(stab_batch_program* P)
{
    if (!P) return;
    if (P->dev || P->cols) (void)hipDeviceSynchronize();
    if (P->dev) (void)hipFree(P->dev);
    if (P->cols) (void)hipFree(P->cols);
    delete P;
}

namespace {

// Zero the record, upload the instruction counters and launch the batch kernel between the
// batch's two events, with launch configuration tile and measurement quota (0: whole program).
int batch_launch(stab_batch* b, const stab_batch_program* P, int tile, int quota)
{
    const long long bytes = P->rec_byte[b->ncirc];
    const long long words = (bytes + 3) / 4;
    if (ensure(b->rec, (size_t)std::max<long long>(words, 1) * 4)) return STAB_ENOMEM;
    BHIP_CHECK(b, hipMemcpyAsync(b->d_ibase, b->icount.data(), sizeof(uint64_t) * b->ncirc, hipMemcpyHostToDevice,
                                  b->stream));
    BHIP_CHECK(b, hipEventRecord(b->ev0, b->stream));
    if (words > 0) {
        const int blocks = (int)std::min<long long>((words + 255) / 256, 4096);
        k_zero32<<<blocks, 256, 0, b->stream>>>((uint32_t*)b->rec.p, words);
        BHIP_CHECK(b, hipGetLastError());
    }
    BatchArgs A{};
    A.circ = P->d_circ;
    A.order = P->d_order;
    A.steps = P->d_steps;
    A.gates = P->d_gates;
    A.noise = P->d_noise;
    A.noise_tg = P->d_noise_tg;
    A.meas = P->d_meas;
    A.meas_tg = P->d_meas_tg;
    A.tab = b->tab;
    A.rs = b->rs;
    A.rec = (uint32_t*)b->rec.p;
    A.ibase = b->d_ibase;
    A.keys = nullptr;
    A.meas_quota = quota;
    A.tile = tile;
    A.cols = P->cols;
    A.seed = b->seed;
    A.err = b->d_err;
    A.counters = b->d_counters;
    const bool one = (tile & kTileOneBlock) != 0;
    if (P->nw == 1) {
        if (one) k_batch<1, 2><<<b->ncirc, kBatchThreads, P->lds_bytes, b->stream>>>(A);
        else k_batch<1, 4><<<b->ncirc, kBatchThreads, P->lds_bytes, b->stream>>>(A);
    } else {
        if (one) k_batch<2, 2><<<b->ncirc, kBatchThreads, P->lds_bytes, b->stream>>>(A);
        else k_batch<2, 4><<<b->ncirc, kBatchThreads, P->lds_bytes, b->stream>>>(A);
    }
    BHIP_CHECK(b, hipGetLastError());
    BHIP_CHECK(b, hipEventRecord(b->ev1, b->stream));
    return STAB_OK;
}

}  // namespace

int stab_batch_execute(stab_batch* b, const stab_batch_program* P, uint8_t* out_bits, float* elapsed_ms)
{
    if (!b || !P) return fail(STAB_EINVAL, "NULL argument");
    if (b->poisoned) return fail(STAB_EDEVICE, "batch poisoned by an earlier device error");
    if (P->ncirc != b->ncirc) return fail(STAB_EINVAL, "program compiled for another batch");
    for (int c = 0; c < b->ncirc; ++c)
        if (P->n[c] != b->circ[c].n) return fail(STAB_EINVAL, "program compiled for other circuit sizes");
    if (P->lds_bytes > b->max_lds) return fail(STAB_ERANGE, "program needs more LDS than the device has");
    const long long bytes = P->rec_byte[b->ncirc];
    const int lrc = batch_launch(b, P, P->tile, 0);
    if (lrc) return lrc;
    if (out_bits && bytes > 0)
        BHIP_CHECK(b, hipMemcpyAsync(out_bits, b->rec.p, (size_t)bytes, hipMemcpyDeviceToHost, b->stream));
    int err = 0;
    BHIP_CHECK(b, hipMemcpyAsync(&err, b->d_err, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    BHIP_CHECK(b, hipStreamSynchronize(b->stream));
    float ms = 0.f;
    BHIP_CHECK(b, hipEventElapsedTime(&ms, b->ev0, b->ev1));
    b->kernel_ms = ms;
    for (int c = 0; c < b->ncirc; ++c) b->icount[c] += (uint64_t)P->ninstr[c];
    if (elapsed_ms) *elapsed_ms = ms;
    if (err) {
        b->poisoned = true;
        return fail(STAB_EINTERNAL, "device consistency check failed (odd rowsum phase or a deterministic "
                                    "product that is not +-Z)");
    }
    return STAB_OK;
}

static_assert(kTileWholeWave == STAB_TILE_WHOLE_WAVE, "tile flag of include/stab.h");
static_assert(kTileOneBlock == STAB_TILE_ONE_BLOCK, "tile flag of include/stab.h");

namespace {

std::mutex g_tune_mu;
std::map<uint64_t, int> g_tune;   // (program shape, device) -> launch configuration

bool tile_valid(int tile)
{
    const int R = tile & 0xff;
    return (tile & ~(0xff | kTileWholeWave | kTileOneBlock)) == 0 && (R == 2 || R == 4 || R == 8);
}

bool tune_file_lookup(uint64_t key, int* tile)
{
    const char* path = std::getenv("STAB_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    unsigned long long k = 0;
    int t = 0;
    bool found = false;
    while (std::fscanf(f, "%llx %d", &k, &t) == 2)
        if (k == key && tile_valid(t)) {
            *tile = t;   // the last entry for a key wins
            found = true;
        }
    std::fclose(f);
    return found;
}

void tune_file_store(uint64_t key, int tile)
{
    const char* path = std::getenv("STAB_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%016llx %d\n", (unsigned long long)key, tile);
    std::fclose(f);
}

}  // namespace

int stab_batch_autotune(stab_batch* b, stab_batch_program* P, int32_t meas_quota, int32_t flags, int32_t* tile_out)
{
    if (!b || !P) return fail(STAB_EINVAL, "NULL argument");
    if (b->poisoned) return fail(STAB_EDEVICE, "batch poisoned by an earlier device error");
    if (meas_quota < 0) return fail(STAB_EINVAL, "meas_quota < 0");
    if (flags & ~STAB_TUNE_FORCE) return fail(STAB_EINVAL, "unknown flags");
    if (P->ncirc != b->ncirc) return fail(STAB_EINVAL, "program compiled for another batch");
    for (int c = 0; c < b->ncirc; ++c)
        if (P->n[c] != b->circ[c].n) return fail(STAB_EINVAL, "program compiled for other circuit sizes");
    if (P->lds_bytes > b->max_lds) return fail(STAB_ERANGE, "program needs more LDS than the device has");
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(STAB_EDEVICE, "no HIP device");
    const uint64_t key = P->shape ^ ((uint64_t)(P->nw * 4096 + cus) << 40);
    if (!(flags & STAB_TUNE_FORCE)) {
        int t = 0;
        bool hit = false;
        {
            std::lock_guard<std::mutex> g(g_tune_mu);
            auto it = g_tune.find(key);
            if (it != g_tune.end()) {
                t = it->second;
                hit = true;
            }
        }
        if (!hit && tune_file_lookup(key, &t)) {
            hit = true;
            std::lock_guard<std::mutex> g(g_tune_mu);
            g_tune[key] = t;
        }
        if (hit) {
            P->tile = t;
            if (tile_out) *tile_out = t;
            return STAB_OK;
        }
    }
    // candidates: lanes per row sized to the circuit or the whole wave, 2, 4 or 8 rows in
    // flight, registers capped for two blocks per compute unit or not (one block)
    std::vector<int> cand;
    for (int one = 0; one < 2; ++one)
        for (int wide = 0; wide < 2; ++wide)
            for (int R : {2, 4, 8}) cand.push_back(R | (wide ? kTileWholeWave : 0) | (one ? kTileOneBlock : 0));
    const long long bytes = P->rec_byte[b->ncirc];
    void* save = nullptr;
    if (hipMalloc(&save, b->bytes) != hipSuccess) return fail(STAB_ENOMEM, "device allocation failed");
    std::vector<unsigned long long> ctr(kNumCounters * kCounterStripes);
    std::vector<uint8_t> ref((size_t)bytes), got((size_t)bytes);
    auto done = [&](int rc) {
        // the batch's state as it was before tuning
        if (hipMemcpyAsync(b->tab, save, b->bytes, hipMemcpyDeviceToDevice, b->stream) != hipSuccess ||
            hipMemcpyAsync(b->d_counters, ctr.data(), ctr.size() * 8, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
            hipStreamSynchronize(b->stream) != hipSuccess) {
            b->poisoned = true;
            if (rc == STAB_OK) rc = fail(STAB_EDEVICE, "restoring the batch after tuning failed");
        }
        (void)hipFree(save);
        return rc;
    };
    if (hipMemcpyAsync(save, b->tab, b->bytes, hipMemcpyDeviceToDevice, b->stream) != hipSuccess ||
        hipMemcpyAsync(ctr.data(), b->d_counters, ctr.size() * 8, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        (void)hipFree(save);
        b->poisoned = true;
        return fail(STAB_EDEVICE, "saving the batch before tuning failed");
    }
    int best = -1;
    float best_ms = 0.f;
    // the first launch warms up and is not timed
    for (int i = -1; i < (int)cand.size(); ++i) {
        const int tile = cand[i < 0 ? 0 : i];
        if (i >= 0 && hipMemcpyAsync(b->tab, save, b->bytes, hipMemcpyDeviceToDevice, b->stream) != hipSuccess)
            return done(fail(STAB_EDEVICE, "restoring the batch between candidates failed"));
        int rc = batch_launch(b, P, tile, meas_quota);
        if (rc) return done(rc);
        int err = 0;
        if ((bytes > 0 && hipMemcpyAsync(got.data(), b->rec.p, (size_t)bytes, hipMemcpyDeviceToHost, b->stream) !=
                              hipSuccess) ||
            hipMemcpyAsync(&err, b->d_err, sizeof(int), hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
            hipStreamSynchronize(b->stream) != hipSuccess)
            return done(fail(STAB_EDEVICE, "candidate launch failed"));
        if (err) {
            b->poisoned = true;
            return done(fail(STAB_EINTERNAL, "device consistency check failed while tuning"));
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, b->ev0, b->ev1) != hipSuccess) return done(fail(STAB_EDEVICE, "event timing failed"));
        if (i < 0) {
            ref = got;
            continue;
        }
        if (got != ref) return done(fail(STAB_EINTERNAL, "launch configurations gave different records"));
        if (std::getenv("STAB_TUNE_LOG")) std::fprintf(stderr, "[stab tune] tile 0x%x: %.3f ms\n", tile, ms);
        if (best < 0 || ms < best_ms) {
            best = tile;
            best_ms = ms;
        }
    }
    const int rc = done(STAB_OK);
    if (rc) return rc;
    P->tile = best;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[key] = best;
    }
    tune_file_store(key, best);
    if (tile_out) *tile_out = best;
    return STAB_OK;
}

int stab_batch_program_set_tile(stab_batch_program* P, int32_t tile)
{
    if (!P) return fail(STAB_EINVAL, "program is NULL");
    if (tile != 0 && !tile_valid(tile)) return fail(STAB_EINVAL, "unknown launch configuration");
    P->tile = tile;
    return STAB_OK;
}

int32_t stab_batch_program_tile(const stab_batch_program* P)
{
    return P ? P->tile : -1;
}

int stab_batch_get_tableau(stab_batch* b, int32_t circuit, uint8_t* x, uint8_t* z, uint8_t* r)
{
    if (!b) return fail(STAB_EINVAL, "batch is NULL");
    if (b->poisoned) return fail(STAB_EDEVICE, "batch poisoned by an earlier device error");
    if (circuit < 0 || circuit >= b->ncirc) return fail(STAB_EINVAL, "circuit out of range");
    const BatchCirc& C = b->circ[circuit];
    std::vector<uint64_t> tab((size_t)2 * C.NR * C.RS), rs(2 * C.Wc);
    BHIP_CHECK(b, hipStreamSynchronize(b->stream));
    BHIP_CHECK(b, hipMemcpy(tab.data(), b->tab + C.tab_off, tab.size() * 8, hipMemcpyDeviceToHost));
    BHIP_CHECK(b, hipMemcpy(rs.data(), b->rs + C.rs_off, rs.size() * 8, hipMemcpyDeviceToHost));
    const int n = C.n;
    for (int half = 0; half < 2; ++half) {
        for (int i = 0; i < n; ++i) {
            const int row = half * C.NR + i;
            const int o = half * n + i;
            const uint64_t* w = &tab[(size_t)row * C.RS];
            for (int j = 0; j < n; ++j) {
                if (x) x[(size_t)o * n + j] = (uint8_t)((w[j >> 6] >> (j & 63)) & 1ull);
                if (z) z[(size_t)o * n + j] = (uint8_t)((w[C.Wc + (j >> 6)] >> (j & 63)) & 1ull);
            }
            if (r) r[o] = (uint8_t)((rs[row >> 6] >> (row & 63)) & 1ull);
        }
    }
    return STAB_OK;
}

int stab_batch_get_counters(stab_batch* b, uint64_t* counters, int32_t ncounters)
{
    if (!b || !counters || ncounters < 0 || ncounters > kNumCounters) return fail(STAB_EINVAL, "bad arguments");
    unsigned long long c[kNumCounters * kCounterStripes];
    BHIP_CHECK(b, hipStreamSynchronize(b->stream));
    BHIP_CHECK(b, hipMemcpy(c, b->d_counters, sizeof(c), hipMemcpyDeviceToHost));
    for (int i = 0; i < ncounters; ++i) {
        uint64_t v = 0;
        for (int j = 0; j < kCounterStripes; ++j) v += c[i * kCounterStripes + j];
        counters[i] = v;
    }
    return STAB_OK;
}

}  // extern "C"
