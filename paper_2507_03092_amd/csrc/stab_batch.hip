// stab_batch.hip -- uneven multi-circuit batching: many independent circuits of different
// sizes, each with its own tableau and its own op stream, run by ONE persistent launch.
//
// One block per circuit executes that circuit's whole program: runs of gate and noise layers
// as band passes (64 rows staged in LDS and turned into qubit-major words, every layer of
// the run applied there, written back once), and measurement instructions target by target
// (Sec. 2.4: pivot = first stabilizer row with x at the qubit, rowsum from it (Appendix A.2)
// for a random outcome, the product of the selected stabilizer rows for a deterministic
// one).  Blocks are dispatched largest circuit first so the long ones start early.
//
// Randomness: Philox4x64-10 with key (seed, circuit index), counter (instruction index in the
// circuit's stream, target position), the index counting every instruction the circuit has
// executed since the batch was created or reset: circuit c draws exactly what a one-shot
// context with first_shot = c draws for the same sequence of streams.
//
// Included by stab_api.hip (same translation unit: it shares the device helpers above).

namespace stabdev {

// Largest circuit of a batch: a lane owns at most two x words and two z words of a row.
constexpr int kBatchMaxWc = 128;
constexpr int kBatchThreads = 512;
constexpr int kBatchWaves = kBatchThreads / 64;

struct BatchCirc {
    int n, Wc, RS, NR;          // NR = 64 * Wc rows per half; RS = 2 * Wc words per row
    long long tab_off;          // first word of the tableau [2*NR][RS]
    long long rs_off;           // first word of the sign vector [2*Wc]
    int step_begin, step_count; // program steps
    long long rec_bit_off;      // bit offset of the circuit's first record in the output
    long long col_off;          // first word of the column scratch [2][NB][col_k] (if col_k > 0)
    int col_k;                  // targets the scratch holds per band (0: no scratch)
};

struct BatchMeas {
    uint64_t instr;  // instruction index in the circuit's stream
    uint64_t t0, t1; // T1T2 thresholds: reset iff u0 < t0, else Z iff u0 < t1
    int kind;        // M, MR, R or T1T2
    int tq;          // first target in the measurement target array
    int K;           // targets
    int rec;         // record index (within the circuit) of the first target; -1 if none
    int fast;        // M/MR/R on distinct qubits: its columns can be extracted in the band pass
};

// Program step: (0, first gate, gates, modifies x|z) gate layer on disjoint qubits;
// (1, noise descriptor, 0, 0) noise layer; (2, measurement descriptor, 0, 0).
struct BatchArgs {
    const BatchCirc* circ;
    const int* order;           // block -> circuit
    const int4* steps;
    const uint2* gates;
    const NoiseDesc* noise;
    const int* noise_tg;
    const BatchMeas* meas;
    const int* meas_tg;
    uint64_t* tab;
    uint64_t* rs;
    uint32_t* rec;              // packed record bits, zeroed before the launch
    uint64_t* cols;             // base of the circuits' column scratch
    const uint64_t* ibase;      // per circuit: instructions it executed before this launch
    const ulonglong2* keys;     // per circuit RNG key, or NULL for (seed, circuit index)
    int meas_quota;             // stop a circuit after this many measurement steps (0: run all)
    int tile;                   // launch configuration (kTileWholeWave and rows in flight)
    uint64_t seed;
    int* err;
    unsigned long long* counters;
};

// LDS words (uint64) the batch kernel needs for a circuit with Wc column words.
__host__ __device__ inline int batch_lds_words(int Wc)
{
    const int RS = 2 * Wc, NB = 2 * Wc;
    const int seg = 64 * (RS + 1) + 16;
    // signs, x-column bits, pivot row, per-wave (X, Z) partial products, 32 ints, row list
    // (uint16, one entry per row), outcome and random-at-start bits of up to 64*Wc targets and
    // the list of the random-at-start ones (uint16)
    const int meas = 2 * NB + RS + 2 * kBatchWaves * RS + 16 + (NB * 64 * 2 + 7) / 8 + 2 * Wc + 16 * Wc;
    return seg > meas ? seg : meas;
}

constexpr int kMK = 7, kMRK = 8, kRK = 9, kT1T2K = 13;   // kinds (include/stab.h enum)
// A measurement instruction with at least this many targets gets an extraction-only band
// pass when no gate pass precedes it.
constexpr int kBatchExtractMin = 8;

__device__ __forceinline__ ulonglong2 batch_key(const BatchArgs& A, int ci)
{
    if (A.keys) return A.keys[ci];
    ulonglong2 k;
    k.x = A.seed;
    k.y = (uint64_t)ci;
    return k;
}

// -------------------------------------------------------------------------------- gates ---
__device__ __forceinline__ void batch_gate(uint64_t* T, int RSP, int Wc, uint2 gt, uint64_t& racc)
{
    const int kind = (int)(gt.x & 15u);
    const int q0 = (int)(gt.x >> 4);
    const int i0 = (q0 & 63) * RSP + (q0 >> 6);
    const uint64_t x0 = T[i0], z0 = T[i0 + Wc];
    switch (kind) {
    case STAB_KIND_H:
        racc ^= x0 & z0;
        T[i0] = z0;
        T[i0 + Wc] = x0;
        break;
    case STAB_KIND_S:
        racc ^= x0 & z0;
        T[i0 + Wc] = z0 ^ x0;
        break;
    case STAB_KIND_X: racc ^= z0; break;
    case STAB_KIND_Y: racc ^= x0 ^ z0; break;
    case STAB_KIND_Z: racc ^= x0; break;
    case STAB_KIND_CX: {
        const int q1 = (int)gt.y;
        const int i1 = (q1 & 63) * RSP + (q1 >> 6);
        const uint64_t x1 = T[i1], z1 = T[i1 + Wc];
        racc ^= x0 & z1 & ~(x1 ^ z0);
        T[i1] = x1 ^ x0;
        T[i0 + Wc] = z0 ^ z1;
    } break;
    default: break;
    }
}

// Noise unit u of descriptor d for circuit ci: XOR into racc the sign flips of the staged
// band's rows (the rows the drawn Pauli anticommutes with).
__device__ __forceinline__ void batch_noise(const uint64_t* T, int RSP, int Wc, const NoiseDesc& d,
                                            const int* __restrict__ ntg, int u, ulonglong2 key,
                                            uint64_t ibase, uint64_t& racc)
{
    uint64_t u0, u1;
    philox(ibase + d.instr, (uint64_t)u, key.x, key.y, u0, u1);
    int q[2], P[2], ne = 0;
    if (d.kind == STAB_KIND_DEP1) {
        if (u0 < d.t0) { q[ne] = ntg[d.toff + u]; P[ne++] = 1 + (int)__umul64hi(u1, 3ull); }
    } else if (d.kind == STAB_KIND_DEP2) {
        if (u0 < d.t0) {
            const int k = 1 + (int)__umul64hi(u1, 15ull);
            if (k >> 2) { q[ne] = ntg[d.toff + 2 * u]; P[ne++] = k >> 2; }
            if (k & 3) { q[ne] = ntg[d.toff + 2 * u + 1]; P[ne++] = k & 3; }
        }
    } else {
        const int p = (u0 < d.t0) ? 1 : (u0 < d.t1) ? 2 : (u0 < d.t2) ? 3 : 0;
        if (p) { q[ne] = ntg[d.toff + u]; P[ne++] = p; }
    }
    for (int e = 0; e < ne; ++e) {
        const int iq = (q[e] & 63) * RSP + (q[e] >> 6);
        const uint64_t xq = T[iq], zq = T[iq + Wc];
        racc ^= (P[e] == 1) ? zq : (P[e] == 3) ? xq : (xq ^ zq);
    }
}

// One run of gate/noise steps [st, en) over every band of the circuit.
// With `ext` set, the band pass also writes the x and z columns of that measurement's targets
// (64 rows per word) to the circuit's column scratch, [band][target].
__device__ void batch_segment(const BatchArgs& A, const BatchCirc& C, int ci, int st, int en,
                              uint64_t* lds, const BatchMeas* ext)
{
    const int tid = threadIdx.x, nt = kBatchThreads;
    const int lane = tid & 63, wave = tid >> 6;
    const int RS = C.RS, RSP = C.RS + 1, Wc = C.Wc, NB = 2 * C.Wc;
    uint64_t* T = lds;
    uint64_t* red = lds + 64 * RSP;
    uint64_t* tab = A.tab + C.tab_off;
    uint64_t* rs = A.rs + C.rs_off;
    const ulonglong2 key = batch_key(A, ci);
    int wb = 0;
    for (int k = st; k < en; ++k) wb |= (A.steps[k].x == 0) ? A.steps[k].w : 0;
    const int npairs = 32 * RS;
    for (int band = 0; band < NB; ++band) {
        uint64_t* gb = tab + (size_t)band * 64 * RS;
        const ulonglong2* gb2 = (const ulonglong2*)gb;
        for (int p0 = 0; p0 < npairs; p0 += 4 * nt) {
            ulonglong2 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int p = p0 + u * nt + tid;
                if (p < npairs) v[u] = gb2[p];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int p = p0 + u * nt + tid;
                if (p < npairs) {
                    const int i = 2 * p;
                    const int r = i / RS;
                    const int c = i - r * RS;
                    T[r * RSP + c] = v[u].x;
                    T[r * RSP + c + 1] = v[u].y;
                }
            }
        }
        __syncthreads();
        for (int c = wave; c < RS; c += kBatchWaves) {
            const uint64_t v = transpose64(T[lane * RSP + c], lane);
            T[lane * RSP + c] = v;
        }
        __syncthreads();
        uint64_t racc = 0;
        for (int k = st; k < en; ++k) {
            const int4 s = A.steps[k];
            if (s.x == 0) {
                for (int gi = tid; gi < s.z; gi += nt) batch_gate(T, RSP, Wc, A.gates[s.y + gi], racc);
            } else {
                const NoiseDesc d = A.noise[s.y];
                for (int u = tid; u < d.units; u += nt)
                    batch_noise(T, RSP, Wc, d, A.noise_tg, u, key, A.ibase[ci], racc);
            }
            __syncthreads();
        }
        if (ext) {
            uint64_t* Xs = A.cols + C.col_off + (size_t)band * C.col_k;
            uint64_t* Zs = Xs + (size_t)NB * C.col_k;
            for (int k = tid; k < ext->K; k += nt) {
                const int q = A.meas_tg[ext->tq + k];
                const int iq = (q & 63) * RSP + (q >> 6);
                Xs[k] = T[iq];
                Zs[k] = T[iq + Wc];
            }
            __syncthreads();    // the transpose back rewrites T
        }
        if (wb) {
            for (int c = wave; c < RS; c += kBatchWaves) {
                const uint64_t v = transpose64(T[lane * RSP + c], lane);
                T[lane * RSP + c] = v;
            }
            __syncthreads();
            ulonglong2* gw2 = (ulonglong2*)gb;
            for (int p = tid; p < npairs; p += nt) {
                const int i = 2 * p;
                const int r = i / RS;
                const int c = i - r * RS;
                ulonglong2 v;
                v.x = T[r * RSP + c];
                v.y = T[r * RSP + c + 1];
                gw2[p] = v;
            }
        }
        racc = wave_xor(racc);
        if (lane == 0) red[wave] = racc;
        __syncthreads();
        if (tid == 0) {
            uint64_t t = 0;
            for (int w = 0; w < kBatchWaves; ++w) t ^= red[w];
            if (t) rs[band] ^= t;
        }
        __syncthreads();    // the next band reuses the LDS tile
    }
    if (tid == 0) count_add(A.counters, 7, (unsigned long long)NB * 64 * RS * 8 * (wb ? 2 : 1));
}

// -------------------------------------------------------------------------- measurement ---
// Bit `bit` of word `word` of every row, as 64-row words (one per band), into out[0..NB).
// With xor_into set the words are XORed into out (used to flip signs) instead of stored.
__device__ __forceinline__ void batch_column(const uint64_t* __restrict__ tab, int RS, int NB,
                                             int word, int bit, uint64_t* out, bool xor_into)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c0 = wave; c0 < NB; c0 += 4 * kBatchWaves) {
        uint64_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + u * kBatchWaves;
            v[u] = (c < NB) ? tab[(size_t)(64 * c + lane) * RS + word] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + u * kBatchWaves;
            const uint64_t m = __ballot((v[u] >> bit) & 1ull);
            if (c < NB && lane == 0) {
                if (xor_into) out[c] ^= m;
                else out[c] = m;
            }
        }
    }
}

// Rows whose bit is set in words [w0, w1) of bits, minus `skip` rows, listed in row order into
// list (uint16) -- block-wide; returns the count (valid in every thread after the call).
__device__ int batch_list(const uint64_t* bits, int w0, int w1, int skip0, int skip1,
                          uint16_t* list, int* s_tot)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int* wtot = s_tot + 1;
    int total = 0;
    for (int base = w0; base < w1; base += kBatchThreads) {
        const int w = base + tid;
        uint64_t m = 0;
        if (w < w1) {
            m = bits[w];
            if ((skip0 >> 6) == w) m &= ~(1ull << (skip0 & 63));
            if ((skip1 >> 6) == w) m &= ~(1ull << (skip1 & 63));
        }
        const int c = __popcll(m);
        const int ex = wave_excl_scan(c, lane);
        if (lane == 63) wtot[wave] = ex + c;
        __syncthreads();
        int off = total;
        for (int v = 0; v < wave; ++v) off += wtot[v];
        int t = 0;
        for (int v = 0; v < kBatchWaves; ++v) t += wtot[v];
        off += ex;
        while (m) {
            list[off++] = (uint16_t)(64 * w + ctz64(m));
            m &= m - 1;
        }
        total += t;
        __syncthreads();
    }
    return total;
}

// Launch configuration of the batch kernel (BatchArgs::tile): bits 0-7 rows each lane group
// keeps in flight in a rowsum (2, 4 or 8, at most 4 with two x words per lane; 0 = 8 for one
// x word per lane, 2 for two); bit 8
// set: every row takes the whole wave (64 lanes per row), clear: a row takes the smallest
// power of two of lanes that covers its x words, so a wave updates 64 / lanes rows per load.
constexpr int kTileWholeWave = 1 << 8;
// bit 9 set: the kernel variant with registers for one block per compute unit (no spills);
// clear: capped for two blocks per compute unit.
constexpr int kTileOneBlock = 1 << 9;

// rowsum(row, p) for every listed row: x|z ^= pivot, sign from the g-sum (Appendix A.2).
// A row is owned by a group of lpr lanes (lane sub of the group holds x words sub,
// sub + lpr, ..., NW of them, and the matching z words); a wave holds 64 / lpr groups and
// each group keeps R rows in flight so their loads overlap.  The g-sums are reduced within
// the group, eight bits per row, four rows per int.
template <int NW, int R>
__device__ void batch_rowsum_tile(const BatchCirc& C, uint64_t* __restrict__ tab, const uint64_t* prow,
                                  int rp, const uint16_t* list, int nlist, uint64_t* sg, int* err, int lpr)
{
    static_assert(R <= 8, "two packed ints hold eight rows");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int Wc = C.Wc, RS = C.RS;
    const int sub = lane & (lpr - 1), grp = lane / lpr, groups = 64 / lpr;
    uint64_t px[NW], pz[NW];
#pragma unroll
    for (int t = 0; t < NW; ++t) {
        const int j = sub + lpr * t;
        px[t] = (j < Wc) ? prow[j] : 0;
        pz[t] = (j < Wc) ? prow[Wc + j] : 0;
    }
    const int step = R * groups;
    for (int base = wave * step; base < nlist; base += kBatchWaves * step) {
        uint64_t x[R][NW], z[R][NW];
        int row[R];
        bool ok[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int li = base + r * groups + grp;
            ok[r] = li < nlist;
            row[r] = ok[r] ? (int)list[li] : 0;
#pragma unroll
            for (int t = 0; t < NW; ++t) {
                const int j = sub + lpr * t;
                x[r][t] = z[r][t] = 0;
                if (ok[r] && j < Wc) {
                    x[r][t] = tab[(size_t)row[r] * RS + j];
                    z[r][t] = tab[(size_t)row[r] * RS + Wc + j];
                }
            }
        }
        int pk[2] = {0, 0};
#pragma unroll
        for (int r = 0; r < R; ++r) {
            int G = 0;
#pragma unroll
            for (int t = 0; t < NW; ++t) G += gsum(px[t], pz[t], x[r][t], z[r][t]);
            pk[r >> 2] += (G & 3) << (8 * (r & 3));
        }
        // at most 64 lanes add at most 3 each: the 8-bit fields do not carry
        for (int m = lpr >> 1; m >= 1; m >>= 1) {
            pk[0] += __shfl_xor(pk[0], m, 64);
            if (R > 4) pk[1] += __shfl_xor(pk[1], m, 64);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (ok[r]) {
#pragma unroll
                for (int t = 0; t < NW; ++t) {
                    const int j = sub + lpr * t;
                    if (j < Wc) {
                        tab[(size_t)row[r] * RS + j] = x[r][t] ^ px[t];
                        tab[(size_t)row[r] * RS + Wc + j] = z[r][t] ^ pz[t];
                    }
                }
                if (sub == 0) {
                    const int G = (pk[r >> 2] >> (8 * (r & 3))) & 3;
                    const int ri = (int)((sg[row[r] >> 6] >> (row[r] & 63)) & 1ull);
                    const int e = (2 * ri + 2 * rp + G) & 3;
                    if (e & 1) atomicOr(err, 1);
                    if ((e >> 1) != ri) atomicXor((unsigned long long*)&sg[row[r] >> 6], 1ull << (row[r] & 63));
                }
            }
        }
    }
}

template <int NW>
__device__ void batch_rowsum(const BatchCirc& C, uint64_t* __restrict__ tab, const uint64_t* prow, int rp,
                             const uint16_t* list, int nlist, uint64_t* sg, int* err, int tile)
{
    int lpr = 64;
    if (!(tile & kTileWholeWave))
        while (lpr > 1 && (lpr >> 1) >= C.Wc) lpr >>= 1;
    const int R = tile & 0xff;
    // two x words per lane: at most 4 rows in flight (register budget)
    if ((R == 8 || R == 0) && NW == 1) batch_rowsum_tile<NW, 8>(C, tab, prow, rp, list, nlist, sg, err, lpr);
    else if (R == 2 || (R == 0 && NW == 2)) batch_rowsum_tile<NW, 2>(C, tab, prow, rp, list, nlist, sg, err, lpr);
    else batch_rowsum_tile<NW, 4>(C, tab, prow, rp, list, nlist, sg, err, lpr);
}

// Sign of the product of the listed stabilizer rows (destabilizer indices i -> row NR + i):
// for Paulis P_k = (-1)^r_k i^|x_k & z_k| X^x_k Z^z_k the product carries
// i^(sum_k (2 r_k + |x_k & z_k|) + 2 sum_{i<k} z_i . x_k); the rows commute, so waves reduce
// contiguous chunks and the cross terms between chunks are added from their (X, Z) parities.
// The result must be +-Z (X = 0 and an even exponent), else *err is set.  Block-wide.
template <int NW>
__device__ int batch_det(const BatchCirc& C, const uint64_t* __restrict__ tab, const uint16_t* list,
                         int nlist, const uint64_t* sg, uint64_t* part, int* s_res, int* err)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int Wc = C.Wc, RS = C.RS, NR = C.NR;
    const int per = (nlist + kBatchWaves - 1) / kBatchWaves;
    const int b0 = min(nlist, wave * per), b1 = min(nlist, b0 + per);
    uint64_t X[NW], Z[NW];
#pragma unroll
    for (int t = 0; t < NW; ++t) X[t] = Z[t] = 0;
    int e = 0, cross = 0;
    for (int c0 = b0; c0 < b1; c0 += 4) {
        uint64_t x[4][NW], z[4][NW];
        int ii[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            ii[r] = (c0 + r < b1) ? (int)list[c0 + r] : -1;
#pragma unroll
            for (int t = 0; t < NW; ++t) {
                const int j = lane + 64 * t;
                x[r][t] = z[r][t] = 0;
                if (ii[r] >= 0 && j < Wc) {
                    x[r][t] = tab[(size_t)(NR + ii[r]) * RS + j];
                    z[r][t] = tab[(size_t)(NR + ii[r]) * RS + Wc + j];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int t = 0; t < NW; ++t) {
                e += __popcll(x[r][t] & z[r][t]);
                cross += __popcll(Z[t] & x[r][t]);
                X[t] ^= x[r][t];
                Z[t] ^= z[r][t];
            }
            if (ii[r] >= 0 && lane == 0) e += 2 * (int)((sg[(NR + ii[r]) >> 6] >> ((NR + ii[r]) & 63)) & 1ull);
        }
    }
    // chunk parities for the cross terms between waves
#pragma unroll
    for (int t = 0; t < NW; ++t) {
        const int j = lane + 64 * t;
        if (j < Wc) {
            part[(2 * wave) * Wc + j] = X[t];
            part[(2 * wave + 1) * Wc + j] = Z[t];
        }
    }
    int v = wave_sum((e & 3) + 2 * (cross & 1));
    if (lane == 0) s_res[1 + wave] = v;
    __syncthreads();
    if (wave == 0) {
        int cr = 0;
        uint64_t xall = 0;
#pragma unroll
        for (int t = 0; t < NW; ++t) {
            const int j = lane + 64 * t;
            if (j < Wc) {
                uint64_t zp = 0, xa = 0;
                for (int w = 0; w < kBatchWaves; ++w) {
                    const uint64_t xw = part[(2 * w) * Wc + j];
                    cr += __popcll(zp & xw);
                    zp ^= part[(2 * w + 1) * Wc + j];
                    xa ^= xw;
                }
                xall |= xa;
            }
        }
        cr = wave_sum(cr & 1);
        xall = wave_or(xall);
        if (lane == 0) {
            int tot = 2 * cr;
            for (int w = 0; w < kBatchWaves; ++w) tot += s_res[1 + w];
            tot &= 3;
            if ((tot & 1) || xall) atomicOr(err, 1);
            s_res[0] = tot >> 1;
        }
    }
    __syncthreads();
    return s_res[0];
}

// LDS of a measurement instruction (see batch_lds_words).
struct MeasLds {
    uint64_t* sg;      // NB sign words
    uint64_t* colx;    // NB words: x bit of the target, per row
    uint64_t* prow;    // RS words: pivot row
    uint64_t* part;    // 2 * kBatchWaves * RS words
    int* s_int;        // 32 ints: pivot, list and det scratch, T1T2 event masks
    uint16_t* list;    // 2 * NR row indices
    uint64_t* outb;    // outcome bits of the instruction's targets
    uint64_t* rndb;    // random-at-start bits
    uint16_t* rlist;   // the random-at-start targets in op order
};

__device__ __forceinline__ MeasLds meas_lds(const BatchCirc& C, uint64_t* lds)
{
    const int NB = 2 * C.Wc, RS = C.RS;
    MeasLds L;
    L.sg = lds;
    L.colx = L.sg + NB;
    L.prow = L.colx + NB;
    L.part = L.prow + RS;
    L.s_int = (int*)(L.part + 2 * kBatchWaves * RS);
    L.list = (uint16_t*)(L.s_int + 32);
    L.outb = (uint64_t*)(L.s_int + 32) + 16 * NB;
    L.rndb = L.outb + C.Wc;
    L.rlist = (uint16_t*)(L.rndb + C.Wc);
    return L;
}

struct MeasWork {
    int nrand = 0, ndet = 0;
    long long nrows = 0, bytes = 0;
};

// Z measurement of qubit a on the live tableau (block-wide): pivot search from the x column,
// then rowsum and row moves (random, outcome rand_bit) or the deterministic product.
//
// The x column is gathered from the tableau (a word per row), or, with Xs, read from column k
// of the column scratch, which the fast form keeps current for the instruction's remaining
// random-at-start targets (the rest targets listed in later[], qubits tq[]): after a random
// outcome every row with x at a (the rowsum rows) flips its x at a later target's qubit by the
// old pivot row's x there, the pivot row's becomes 0 (it is now Z_a) and its partner
// destabilizer's becomes the old pivot row's.
template <int NW>
__device__ int batch_measure_one(const BatchArgs& A, const BatchCirc& C, int a, int rand_bit, const MeasLds& L,
                                 MeasWork& W, uint64_t* Xs = nullptr, int k = 0, const uint16_t* later = nullptr,
                                 int rest = 0, const int* tq = nullptr)
{
    const int tid = threadIdx.x;
    const int Wc = C.Wc, RS = C.RS, NR = C.NR, NB = 2 * C.Wc, CK = C.col_k;
    uint64_t* tab = A.tab + C.tab_off;
    const long long row_b = (long long)RS * 8;
    const long long col_b = Xs ? (long long)NB * 8 : (long long)2 * NR * 8;
    if (Xs) {
        for (int w = tid; w < NB; w += kBatchThreads) L.colx[w] = Xs[(size_t)w * CK + k];
    } else {
        batch_column(tab, RS, NB, a >> 6, a & 63, L.colx, false);
    }
    __syncthreads();
    // pivot: first stabilizer row with x at a (rows NR + n .. 2NR - 1 are zero padding)
    if (tid < 64) {
        int first = 0x7fffffff;
        for (int w = Wc + tid; w < NB; w += 64)
            if (L.colx[w]) first = min(first, 64 * w + ctz64(L.colx[w]));
        first = wave_min(first);
        if (tid == 0) L.s_int[0] = first;
    }
    __syncthreads();
    const int p = L.s_int[0];
    int outcome;
    if (p != 0x7fffffff) {
        outcome = rand_bit;
        for (int j = tid; j < RS; j += kBatchThreads) L.prow[j] = tab[(size_t)p * RS + j];
        const int rp = (int)((L.sg[p >> 6] >> (p & 63)) & 1ull);
        const int nl = batch_list(L.colx, 0, NB, p, p - NR, L.list, L.s_int + 1);
        __syncthreads();    // prow staged
        batch_rowsum<NW>(C, tab, L.prow, rp, L.list, nl, L.sg, A.err, A.tile);
        __syncthreads();
        // destabilizer p - NR <- old stabilizer p; stabilizer p <- (-1)^outcome Z_a
        const int d = p - NR;
        for (int j = tid; j < RS; j += kBatchThreads) {
            tab[(size_t)d * RS + j] = L.prow[j];
            tab[(size_t)p * RS + j] = (j == Wc + (a >> 6)) ? (1ull << (a & 63)) : 0ull;
        }
        if (tid == 0) {
            uint64_t wd = L.sg[d >> 6];
            wd = (wd & ~(1ull << (d & 63))) | ((uint64_t)rp << (d & 63));
            L.sg[d >> 6] = wd;
            uint64_t wp = L.sg[p >> 6];
            wp = (wp & ~(1ull << (p & 63))) | ((uint64_t)outcome << (p & 63));
            L.sg[p >> 6] = wp;
        }
        ++W.nrand;
        W.nrows += nl;
        // column, pivot row, rowsum read+write, two row writes
        W.bytes += col_b + row_b + 2 * nl * row_b + 2 * row_b;
        if (Xs && rest > 0) {
            // the later targets' columns.  A target whose qubit the old pivot row has x at flips
            // at every row of the measured column (row p's bit, set in both, clears with them)
            // and its row-d bit becomes 1; any other target keeps its column except row d's bit,
            // which becomes 0.  The flipping targets are listed (in any order) in L.list, free
            // since the rowsum, and their words are then updated four to a thread at a time.
            __shared__ int s_nf;
            if (tid == 0) s_nf = 0;
            __syncthreads();
            const uint64_t bd = 1ull << (d & 63);
            const int wdw = d >> 6;
            for (int j = tid; j < rest; j += kBatchThreads) {
                const int k2 = later[j], a2 = tq[k2];
                if ((L.prow[a2 >> 6] >> (a2 & 63)) & 1ull) {
                    L.list[atomicAdd(&s_nf, 1)] = (uint16_t)k2;
                } else {
                    uint64_t* xw = Xs + (size_t)wdw * CK + k2;
                    const uint64_t v = *xw;
                    if (v & bd) *xw = v & ~bd;
                }
            }
            __syncthreads();
            const int nf = s_nf;
            for (int id0 = tid; id0 < nf * NB; id0 += 4 * kBatchThreads) {
                uint64_t v[4];
                uint64_t* xw[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int id = id0 + u * kBatchThreads;
                    xw[u] = nullptr;
                    v[u] = 0;
                    if (id < nf * NB) {
                        const int w = id / nf, j = id - w * nf;
                        xw[u] = Xs + (size_t)w * CK + L.list[j];
                        v[u] = *xw[u] ^ L.colx[w];
                        if (w == wdw) v[u] |= bd;
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (xw[u]) *xw[u] = v[u];
            }
            __syncthreads();
            // read and write of every word of the flipping columns, one word of the others
            W.bytes += (long long)nf * NB * 16 + (long long)(rest - nf) * 16;
        }
    } else {
        const int nl = batch_list(L.colx, 0, Wc, -1, -1, L.list, L.s_int + 1);
        outcome = batch_det<NW>(C, tab, L.list, nl, L.sg, L.part, L.s_int + 10, A.err);
        ++W.ndet;
        W.nrows += nl;
        W.bytes += col_b + nl * row_b;
    }
    __syncthreads();
    return outcome;
}

// One wave: the outcome of target k of an instruction whose columns are in the scratch, if it
// is deterministic (no stabilizer has x at the qubit); -1 if it is random.  The product of
// the stabilizers selected by the destabilizers with x at the qubit, as in batch_det.
template <int NW>
__device__ int batch_det_from_cols(const BatchArgs& A, const BatchCirc& C, const uint64_t* Xs, int k,
                                   const uint64_t* sg, int& nrows)
{
    const int lane = threadIdx.x & 63;
    const int Wc = C.Wc, RS = C.RS, NR = C.NR, CK = C.col_k;
    const uint64_t* tab = A.tab + C.tab_off;
    bool st = false;
    for (int w = Wc + lane; w < 2 * Wc; w += 64) st |= Xs[(size_t)w * CK + k] != 0ull;
    if (__ballot(st)) return -1;
    uint64_t X[NW], Z[NW];
#pragma unroll
    for (int t = 0; t < NW; ++t) X[t] = Z[t] = 0;
    int e = 0, cross = 0, rows = 0;
    for (int w = 0; w < Wc; ++w) {
        uint64_t m = Xs[(size_t)w * CK + k];
        while (m) {
            const int i = 64 * w + ctz64(m);
            m &= m - 1;
            const uint64_t* row = tab + (size_t)(NR + i) * RS;
#pragma unroll
            for (int t = 0; t < NW; ++t) {
                const int j = lane + 64 * t;
                const uint64_t x = (j < Wc) ? row[j] : 0ull, z = (j < Wc) ? row[Wc + j] : 0ull;
                e += __popcll(x & z);
                cross += __popcll(Z[t] & x);
                X[t] ^= x;
                Z[t] ^= z;
            }
            if (lane == 0) e += 2 * (int)((sg[(NR + i) >> 6] >> ((NR + i) & 63)) & 1ull);
            ++rows;
        }
    }
    uint64_t xr = 0;
#pragma unroll
    for (int t = 0; t < NW; ++t) xr |= X[t];
    const int tot = wave_sum((e & 3) + 2 * (cross & 1)) & 3;
    xr = wave_or(xr);
    if (lane == 0 && ((tot & 1) || xr)) atomicOr(A.err, 1);
    nrows += rows;
    return tot >> 1;
}

// One M / MR / R / T1T2 instruction of circuit ci.
//
// Slow form (any instruction): target by target on the live tableau.  A T1T2 instruction runs
// here too: per target a Philox draw picks reset (u0 < t0: a measurement whose random outcome
// is u1 >> 63, then X if it is 1), Z (u0 < t1: sign flip of every row with x at the qubit) or
// nothing; one wave draws 64 targets at a time (draws do not depend on the tableau).
//
// Fast form (M/MR/R on distinct qubits whose columns the band pass extracted): every target
// deterministic at the start of the instruction is reduced at once, one wave per target (a
// deterministic outcome does not change when other qubits are measured or reset); the
// random-at-start ones then run in op order on the live tableau; resets come last (an X on a
// measured qubit flips signs only, which commutes with the other measurements).
template <int NW>
__device__ void batch_measure(const BatchArgs& A, const BatchCirc& C, int ci, const BatchMeas& md,
                              uint64_t* lds, bool fast)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int Wc = C.Wc, RS = C.RS, NR = C.NR, NB = 2 * C.Wc;
    uint64_t* tab = A.tab + C.tab_off;
    uint64_t* rs = A.rs + C.rs_off;
    const MeasLds L = meas_lds(C, lds);
    const ulonglong2 key = batch_key(A, ci);
    const long long row_b = (long long)RS * 8, col_b = (long long)2 * NR * 8;
    MeasWork W;
    for (int w = tid; w < NB; w += kBatchThreads) L.sg[w] = rs[w];
    __syncthreads();

    if (fast) {
        const uint64_t* Xs = A.cols + C.col_off;
        const uint64_t* Zs = Xs + (size_t)NB * C.col_k;
        const int KW = (md.K + 63) >> 6;
        for (int w = tid; w < KW; w += kBatchThreads) L.outb[w] = L.rndb[w] = 0;
        __syncthreads();
        int nrows = 0, ndet = 0;
        for (int k = wave; k < md.K; k += kBatchWaves) {
            const int o = batch_det_from_cols<NW>(A, C, Xs, k, L.sg, nrows);
            if (lane == 0) {
                if (o < 0) atomicOr((unsigned long long*)&L.rndb[k >> 6], 1ull << (k & 63));
                else if (o) atomicOr((unsigned long long*)&L.outb[k >> 6], 1ull << (k & 63));
            }
            if (o >= 0) ++ndet;
        }
        // (per-wave work, counted by each wave; the block-wide work in W by thread 0 below)
        if (lane == 0 && ndet) {
            count_add(A.counters, 2, (unsigned long long)ndet);
            count_add(A.counters, 5, (unsigned long long)nrows);
            count_add(A.counters, 6, (unsigned long long)((long long)ndet * NB * 8 + (long long)nrows * row_b));
        }
        __syncthreads();
        // random at the start of the instruction: in op order, on the live tableau, their x
        // columns read from the scratch and kept current there
        uint16_t* rl = L.rlist;
        const int nr = batch_list(L.rndb, 0, KW, -1, -1, rl, L.s_int + 1);
        const bool ran = nr > 0;
        uint64_t* Xw = A.cols + C.col_off;
        for (int i = 0; i < nr; ++i) {
            const int k = rl[i];
            uint64_t u0, u1;
            philox(A.ibase[ci] + md.instr, (uint64_t)k, key.x, key.y, u0, u1);
            const int o = batch_measure_one<NW>(A, C, A.meas_tg[md.tq + k], (int)(u0 >> 63), L, W, Xw, k, rl + i + 1,
                                                nr - i - 1, A.meas_tg + md.tq);
            if (tid == 0 && o) L.outb[k >> 6] |= 1ull << (k & 63);
            __syncthreads();
        }
        if (md.rec >= 0)
            for (int k = tid; k < md.K; k += kBatchThreads)
                if ((L.outb[k >> 6] >> (k & 63)) & 1ull) {
                    const long long rb = C.rec_bit_off + md.rec + k;
                    atomicOr(&A.rec[rb >> 5], 1u << (rb & 31));
                }
        if (md.kind != kMK) {
            if (!ran) {
                // the extracted z columns are still those of the live tableau
                for (int w = tid; w < NB; w += kBatchThreads) {
                    uint64_t x = 0;
                    for (int kw = 0; kw < KW; ++kw) {
                        uint64_t m = L.outb[kw];
                        while (m) {
                            const int k = 64 * kw + ctz64(m);
                            m &= m - 1;
                            x ^= Zs[(size_t)w * C.col_k + k];
                        }
                    }
                    L.sg[w] ^= x;
                }
                __syncthreads();
            } else {
                for (int kw = 0; kw < KW; ++kw) {
                    uint64_t m = L.outb[kw];
                    while (m) {
                        const int k = 64 * kw + ctz64(m);
                        m &= m - 1;
                        const int a = A.meas_tg[md.tq + k];
                        batch_column(tab, RS, NB, Wc + (a >> 6), a & 63, L.sg, true);
                        __syncthreads();
                        W.bytes += col_b;
                    }
                }
            }
        }
    } else {
        const bool stoch = md.kind == kT1T2K;
        uint64_t* s_ev = (uint64_t*)(L.s_int + 24);        // a T1T2 chunk: reset, Z, outcome masks
        for (int c0 = 0; c0 < md.K; c0 += 64) {
            const int cn = min(64, md.K - c0);
            const uint64_t live = cn == 64 ? ~0ull : ((1ull << cn) - 1ull);
            uint64_t ev_meas = live, ev_z = 0, ev_bits = 0;  // M / MR / R: every target, in order
            if (stoch) {
                if (tid < 64) {
                    int act = 0, rb = 0;
                    if (tid < cn) {
                        uint64_t u0, u1;
                        philox(A.ibase[ci] + md.instr, (uint64_t)(c0 + tid), key.x, key.y, u0, u1);
                        act = u0 < md.t0 ? 1 : (u0 < md.t1 ? 2 : 0);
                        rb = (int)(u1 >> 63);
                    }
                    const uint64_t m1 = __ballot(act == 1), m2 = __ballot(act == 2), mb = __ballot(rb);
                    if (tid == 0) {
                        s_ev[0] = m1;
                        s_ev[1] = m2;
                        s_ev[2] = mb;
                    }
                }
                __syncthreads();
                ev_meas = s_ev[0];
                ev_z = s_ev[1];
                ev_bits = s_ev[2];
                __syncthreads();
            }
            uint64_t evm = (ev_meas | ev_z) & live;
            while (evm) {
                const int bit = ctz64(evm);
                evm &= evm - 1;
                const int t = c0 + bit;
                const int a = A.meas_tg[md.tq + t];
                if ((ev_z >> bit) & 1ull) {
                    // Z on the qubit: flip the sign of every row with x at it
                    batch_column(tab, RS, NB, a >> 6, a & 63, L.sg, true);
                    __syncthreads();
                    W.bytes += col_b;
                    continue;
                }
                int rand_bit;
                if (stoch) {
                    rand_bit = (int)((ev_bits >> bit) & 1ull);
                } else {
                    uint64_t u0, u1;
                    philox(A.ibase[ci] + md.instr, (uint64_t)t, key.x, key.y, u0, u1);
                    rand_bit = (int)(u0 >> 63);
                }
                const int outcome = batch_measure_one<NW>(A, C, a, rand_bit, L, W);
                if (md.rec >= 0 && tid == 0 && outcome) {
                    const long long rb = C.rec_bit_off + md.rec + t;
                    atomicOr(&A.rec[rb >> 5], 1u << (rb & 31));
                }
                if (md.kind != kMK && outcome) {
                    // reset: apply X_a, i.e. flip the sign of every row with z at a
                    batch_column(tab, RS, NB, Wc + (a >> 6), a & 63, L.sg, true);
                    __syncthreads();
                    W.bytes += col_b;
                }
            }
        }
    }
    __syncthreads();
    for (int w = tid; w < NB; w += kBatchThreads) rs[w] = L.sg[w];
    if (tid == 0 && (W.ndet || W.nrand || W.nrows)) {
        count_add(A.counters, 4, (unsigned long long)W.nrand);
        count_add(A.counters, 2, (unsigned long long)W.ndet);
        count_add(A.counters, 5, (unsigned long long)W.nrows);
        count_add(A.counters, 6, (unsigned long long)W.bytes);
    }
    __syncthreads();
}

// NW = x words per lane of a row: 1 when every circuit has at most 4096 qubits, else 2.
// OCC = waves per SIMD the registers are sized for: 4 caps them at 128 so two blocks share a
// compute unit (the compiler spills some values to scratch), 2 lets one block per compute unit
// use up to 256 with no spills.  Which is faster depends on the batch; the autotuner times both.
template <int NW, int OCC>
__global__ void __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(OCC))) k_batch(BatchArgs A)
{
    extern __shared__ uint64_t lds[];
    const int ci = A.order[blockIdx.x];
    const BatchCirc C = A.circ[ci];
    const int end = C.step_begin + C.step_count;
    int done = 0, ext_step = -1;
    for (int st = C.step_begin; st < end && (A.meas_quota == 0 || done < A.meas_quota);) {
        const int4 s0 = A.steps[st];
        if (s0.x == 2) {
            const BatchMeas md = A.meas[s0.y];
            if (ext_step != st && A.cols && md.fast && md.K <= C.col_k && md.K >= kBatchExtractMin) {
                // no band pass ran since the last measurement: one that only reads the rows
                // and extracts the columns is far cheaper than measuring target by target
                batch_segment(A, C, ci, st, st, lds, &A.meas[s0.y]);
                ext_step = st;
            }
            batch_measure<NW>(A, C, ci, md, lds, ext_step == st);
            ext_step = -1;
            ++st;
            ++done;
            continue;
        }
        int en = st + 1;
        while (en < end && A.steps[en].x != 2) ++en;
        // the next measurement's columns come out of this band pass when it allows that
        const BatchMeas* nx = nullptr;
        if (en < end && A.cols) {
            const BatchMeas* m = &A.meas[A.steps[en].y];
            if (m->fast && m->K <= C.col_k) nx = m;
        }
        batch_segment(A, C, ci, st, en, lds, nx);
        if (nx) ext_step = en;
        st = en;
    }
}

// |0...0> for every circuit: block per circuit.
__global__ void k_batch_init(const BatchCirc* __restrict__ circ, uint64_t* __restrict__ tab,
                             uint64_t* __restrict__ rs)
{
    const BatchCirc C = circ[blockIdx.x];
    uint64_t* t = tab + C.tab_off;
    const long long words = (long long)2 * C.NR * C.RS;
    for (long long idx = threadIdx.x; idx < words; idx += blockDim.x) {
        const int row = (int)(idx / C.RS);
        const int c = (int)(idx - (long long)row * C.RS);
        uint64_t v = 0;
        if (row < C.NR) {
            if (row < C.n && c == (row >> 6)) v = 1ull << (row & 63);
        } else {
            const int i = row - C.NR;
            if (i < C.n && c == C.Wc + (i >> 6)) v = 1ull << (i & 63);
        }
        t[idx] = v;
    }
    for (int w = threadIdx.x; w < 2 * C.Wc; w += blockDim.x) rs[C.rs_off + w] = 0;
}

__global__ void k_zero32(uint32_t* __restrict__ p, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace stabdev
