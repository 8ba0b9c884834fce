// stab_device.h -- structures shared by the kernels and the host side of libstab.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace stabdev {

// Most 64-bit column words a lane of the deterministic-measurement wave keeps in registers.
constexpr int kMaxWordsPerLane = 4;
// Most sign/band words (2 * ceil(n/64)) a lane of the chain's analysis wave reads.
constexpr int kMaxBandsPerLane = 5;
constexpr int kMaxStabBandsPerLane = (32 * kMaxBandsPerLane + 63) / 64;   // the stabilizer half

struct Geom {
    int n;    // qubits
    int Wc;   // column words per row and component: ceil(n / 64)
    int Wr;   // 64-row bands per half: ceil(n / 64)
    int NR;   // rows per half, padded: 64 * Wr
    int RS;   // row stride in words: 2 * Wc (x words, then z words)
    int NB;   // bands (and sign words) per tableau: 2 * Wr
    int S;    // tableau copies
    int B;    // shots
    int bpc;  // shots per copy (B / S)
    int rev;  // 1: kernels take their blocks in reverse order (a determinism check)
};

// Block index along x (y) in the order the kernels take blocks: reversed when g.rev is set, so a
// run with the flag changes which work each dispatched workgroup does and the order in which the
// work reaches the device; the results must not change.
__device__ __forceinline__ int blk_x(const Geom& g) { return g.rev ? (int)gridDim.x - 1 - (int)blockIdx.x : (int)blockIdx.x; }
__device__ __forceinline__ int blk_y(const Geom& g) { return g.rev ? (int)gridDim.y - 1 - (int)blockIdx.y : (int)blockIdx.y; }

// One noise instruction of a segment.
struct NoiseDesc {
    uint64_t instr;        // instruction index (Philox counter word 0)
    uint64_t t0, t1, t2;   // thresholds
    int kind;              // DEP1, DEP2 or PAULI1
    int toff;              // first target in the segment's noise target array
    int units;             // targets (DEP1, PAULI1) or pairs (DEP2)
    int bucket;            // event bucket (= item.w of the noise item; consecutive noise layers share one)
};

// Work counters are striped over this many addresses (by block) to keep atomics uncontended.
constexpr int kCounterStripes = 32;
constexpr int kNumCounters = 12;

__device__ __forceinline__ void count_add(unsigned long long* counters, int idx, unsigned long long v)
{
    if (counters) atomicAdd(&counters[idx * kCounterStripes + (blockIdx.x & (kCounterStripes - 1))], v);
}

// Random-measurement chain: window of pending targets, rows a batched target may touch, and
// the largest batch whose pivot rows are staged in LDS so all waves share its rowsums.
constexpr int kWin = 64;
constexpr int kRCap = 128;
constexpr int kWide = 4;
constexpr int kAnalyze = 48;     // window entries (re)analysed per round, at most
constexpr int kAffCap = 1024;    // column-upkeep work list of a wide batch
constexpr int kPListCap = 16;    // pending targets listed per run target (more: replay walks rows)

// Dynamic LDS layout of the chain kernel (byte offsets), shared by host and device.
struct ChainLds {
    int solo;    // block-solo buffers: 2 rows, 2 band masks, per-shot pivot signs, word list
    int owner;   // NR ints: first window target owning each row pair
    int wide;    // kWide pivot rows of the batch
    int words;   // kWide x kRCap (word, mask) lists of the batch's rowsum rows
    int aff;     // kAffCap column-upkeep entries {code, flags, batch index}
    int win;     // window arrays: 9 x kWin ints + kWin x kRCap row indices
    int tm;      // n int16: qubit -> pending target whose x column is kept, or -1
    int pbit;    // NR bits: row pairs that are pivots of the round's executed targets
    int total;
};

__host__ __device__ inline int align16i(int v) { return (v + 15) & ~15; }

__host__ __device__ inline ChainLds chain_lds_layout(const Geom& g)
{
    ChainLds L;
    const int nrdw = (g.bpc + 63) / 64;
    L.solo = 0;
    L.owner = align16i((2 * g.RS + 2 * g.NB + nrdw) * 8 + g.NB * 4);
    L.wide = L.owner + align16i(g.NR * 4);
    L.words = L.wide + kWide * g.RS * 8;
    L.aff = L.words + kWide * kRCap * 12;
    L.win = L.aff + kAffCap * 12;
    L.tm = L.win + (9 * kWin + kWin * kRCap) * 4;
    L.pbit = L.tm + align16i(g.n * 2);
    L.total = L.pbit + align16i((g.NR + 31) / 32 * 4);
    return L;
}

struct SegArgs {
    const int4* items;     // {0, first gate, gate count, -1} or {1, first event slot, event capacity, bucket}
    int nitems;
    const uint2* gates;    // {kind | i0 << 4, i1}, i = the qubit's word index in the staged tile
    const uint2* events;   // noise events {tile word index of the qubit | pauli << 28, shot}
    const int* ev_count;   // per bucket
    const int* ev_base;    // per bucket: first slot in events
    int write_back;        // 1 if some gate changes x|z (H, S, CX)
    int lds_rd;            // 1: accumulate per-shot signs in LDS (bpc fits)
    const int* ext_q;      // qubits whose columns the next measurement layer needs
    int K;
    uint64_t* Xcol;        // [S][NB][K]
    uint64_t* Zcol;
    const int* gate;       // if set and *gate == 0 the launch does nothing
};

}  // namespace stabdev
