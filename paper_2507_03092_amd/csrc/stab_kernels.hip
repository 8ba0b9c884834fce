// stab_kernels.hip -- device code of the MI355X tableau simulator (gfx950, wave64).
//
// Storage (per tableau copy s):
//   tab  [2*NR][RS] uint64, row-major.  Row i < NR is destabilizer i, row NR+i stabilizer i
//        (NR = 64*ceil(n/64); rows >= n of each half are zero padding).  A row holds Wc x-words
//        (bit j%64 of word j/64 = x at qubit j) then Wc z-words; RS = 2*Wc.
//   rs   [NB] uint64 sign words of the copy (NB = 2*NR/64; word w holds rows 64w..64w+63).
//   rd   [B][NB] per-shot sign words.  The sign of row i in shot b is rs ^ rd[b].  In the
//        shared mode one x|z tableau serves every shot: gates only ever XOR shot-independent
//        masks into signs, so those go to rs, while noise, random outcomes and resets (the
//        only shot-dependent parts) go to rd.
//
// A "band" is 64 consecutive rows.  The segment kernel stages half a band (32 rows) in LDS,
// turns its 32x32 bit tiles into qubit-major 32-bit words (one bit per row of one qubit
// column), applies a whole run of gate and noise layers there, extracts the columns the next
// measurement layer needs and writes the rows back.  Measurements then work on rows (rowsum,
// Appendix A.2).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "stab_device.h"

#define STAB_KIND_H 1
#define STAB_KIND_S 2
#define STAB_KIND_X 3
#define STAB_KIND_Y 4
#define STAB_KIND_Z 5
#define STAB_KIND_CX 6
#define STAB_KIND_DEP1 10
#define STAB_KIND_DEP2 11
#define STAB_KIND_PAULI1 12

namespace stabdev {

// ------------------------------------------------------------------------------------------
// Philox4x64-10, from Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
// 1, 2, 3" (SC'11): ten rounds, each multiplying words 0 and 2 by the two published
// multipliers (full 128-bit products) and mixing the halves with the other words and the
// key; the key advances by the two published Weyl constants between rounds.
// Counter = (c0, c1, 0, 0), key = (k0, k1).
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void philox(uint64_t c0, uint64_t c1, uint64_t k0, uint64_t k1,
                                       uint64_t& u0, uint64_t& u1)
{
    uint64_t a = c0, b = c1, c = 0, d = 0;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t pa_lo = 0xD2E7470EE14C6C93ull * a;
        const uint64_t pa_hi = __umul64hi(0xD2E7470EE14C6C93ull, a);
        const uint64_t pc_lo = 0xCA5A826395121157ull * c;
        const uint64_t pc_hi = __umul64hi(0xCA5A826395121157ull, c);
        a = pc_hi ^ b ^ k0;
        b = pc_lo;
        c = pa_hi ^ d ^ k1;
        d = pa_lo;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    u0 = a;
    u1 = b;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m)
{
    const int lo = __shfl_xor((int)(uint32_t)v, m, 64);
    const int hi = __shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    const int lo = __shfl((int)(uint32_t)v, src, 64);
    const int hi = __shfl((int)(uint32_t)(v >> 32), src, 64);
    return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ uint64_t wave_xor(uint64_t v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v ^= shfl_xor_u64(v, m);
    return v;
}

__device__ __forceinline__ uint64_t wave_or(uint64_t v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v |= shfl_xor_u64(v, m);
    return v;
}

// In-register transpose of a 64x64 bit matrix held one row per lane (bit c of lane r's word =
// element (r, c)).  Six butterfly stages swap the off-diagonal blocks of size 32, 16, ..., 1.
// Every lane of the wave must take part.
__device__ __forceinline__ uint64_t transpose64(uint64_t v, int lane)
{
    const uint64_t masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                               0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const int j = 32 >> st;
        const uint64_t m = masks[st];
        const uint64_t o = shfl_xor_u64(v, j);
        if (lane & j) {
            v ^= ((o >> j) ^ v) & m;
        } else {
            v ^= (((v >> j) ^ o) & m) << j;
        }
    }
    return v;
}

// Sum over the 64 bit positions of g(x1,z1,x2,z2) from the rowsum algorithm (Appendix A.2):
// the power of i from multiplying the Pauli (x1,z1) into (x2,z2), per bit in {-1, 0, +1}.
__device__ __forceinline__ int gsum(uint64_t x1, uint64_t z1, uint64_t x2, uint64_t z2)
{
    const uint64_t y1 = x1 & z1, xo = x1 & ~z1, zo = ~x1 & z1;
    const uint64_t plus = (y1 & ~x2 & z2) | (xo & x2 & z2) | (zo & x2 & ~z2);
    const uint64_t minus = (y1 & x2 & ~z2) | (xo & ~x2 & z2) | (zo & x2 & z2);
    return __popcll(plus) - __popcll(minus);
}

__device__ __forceinline__ int ctz64(uint64_t v) { return __builtin_ctzll(v); }

// Lane l's 64-bit value, l uniform (scalar result).
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// v from lane (lane ^ j), j in {1, 2, 4, 8, 16}, without the LDS crossbar: DPP quad permutes
// and row mirrors for j <= 8 (xor 4 = half-mirror then quad xor 3; xor 8 = mirror then
// half-mirror) and the gfx950 permlane16 swap for j = 16.  Every lane must be active.
__device__ __forceinline__ uint32_t lane_xor32(uint32_t v, int j, int lane)
{
    switch (j) {
    case 1: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, true);
    case 2: return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, true);
    case 4: {
        const int t = __builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, true);
        return (uint32_t)__builtin_amdgcn_update_dpp(0, t, 0x1B, 0xF, 0xF, true);
    }
    case 8: {
        const int t = __builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, true);
        return (uint32_t)__builtin_amdgcn_update_dpp(0, t, 0x141, 0xF, 0xF, true);
    }
    default: {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? r[0] : r[1];
    }
    }
}

// Sum over the wave, every lane active: DPP and permlane steps within each 32-lane half, then the
// two halves' totals read out, so the result is uniform.
__device__ __forceinline__ int wave_sum_uniform(int v, int lane)
{
#pragma unroll
    for (int j = 1; j <= 16; j <<= 1) v += (int)lane_xor32((uint32_t)v, j, lane);
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 32);
}

// Sorted rows as (64-row word, bit mask) runs.  rows[64 h + lane] belongs to lane `lane` of half
// h (nrows <= 128); a lane heads a run when its row starts a new word or the half, so one word
// may head a run in both halves, with disjoint masks.  hm[h]: the head lanes; the head's wv[h]
// and mv[h] are its run's word and mask (a segmented OR over the run's lanes).  Whole wave.
__device__ __forceinline__ void row_runs(const int* rows, int nrows, int lane, uint64_t* hm, int* wv, uint64_t* mv)
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        hm[h] = 0ull;
        wv[h] = 0;
        mv[h] = 0ull;
        const int nv = min(nrows - 64 * h, 64);
        if (nv <= 0) continue;
        const int r = 64 * h + lane;
        const bool valid = lane < nv;
        const int row = valid ? rows[r] : 0;
        const int w = row >> 6;
        const bool head = valid && (lane == 0 || (rows[r - 1] >> 6) != w);
        const uint64_t H = __ballot(head);
        const uint64_t after = lane < 63 ? H >> (lane + 1) : 0ull;
        const int end = after ? lane + 1 + ctz64(after) : nv;
        uint64_t acc = valid ? 1ull << (row & 63) : 0ull;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t v = shfl_u64(acc, lane + off < 64 ? lane + off : lane);
            if (lane + off < end) acc |= v;
        }
        hm[h] = H;
        wv[h] = w;
        mv[h] = acc;
    }
}

// f(word, mask) for every run of row_runs, in a scalar loop over the head lanes (the words and
// masks are read out of their lanes whatever the exec mask, so f may run under a lane mask).
template <class F>
__device__ __forceinline__ void for_runs(const uint64_t* hm, const int* wv, const uint64_t* mv, F f)
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        uint64_t H = hm[h];
        while (H) {
            const int l = ctz64(H);
            H &= H - 1;
            f(__builtin_amdgcn_readlane(wv[h], l), readlane_u64(mv[h], l));
        }
    }
}

// ------------------------------------------------------------------------------------------
// init: |0...0> -- destabilizer i = +X_i, stabilizer i = +Z_i, all signs 0.
// ------------------------------------------------------------------------------------------
__global__ void k_init(Geom g, uint64_t* __restrict__ tab, uint64_t* __restrict__ rs,
                       uint64_t* __restrict__ rd)
{
    const size_t rows = (size_t)g.S * 2 * g.NR;
    const size_t total = rows * g.RS;
    for (size_t idx = blk_x(g) * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t row = idx / g.RS;
        const int c = (int)(idx - row * g.RS);
        const int rr = (int)(row % (2 * (size_t)g.NR));
        uint64_t v = 0;
        if (rr < g.NR) {
            if (rr < g.n && c == (rr >> 6)) v = 1ull << (rr & 63);
        } else {
            const int i = rr - g.NR;
            if (i < g.n && c == g.Wc + (i >> 6)) v = 1ull << (i & 63);
        }
        tab[idx] = v;
    }
    const size_t nrs = (size_t)g.S * g.NB, nrd = (size_t)g.B * g.NB;
    for (size_t idx = blk_x(g) * (size_t)blockDim.x + threadIdx.x; idx < nrs + nrd;
         idx += (size_t)gridDim.x * blockDim.x) {
        if (idx < nrs) rs[idx] = 0;
        else rd[idx - nrs] = 0;
    }
}

// ------------------------------------------------------------------------------------------
// Noise draws: block (x, y) handles kNoiseUnitsPerBlock consecutive (shot, unit) pairs of noise
// instruction y.  Draws never depend on the tableau, so they are made up front (the whole
// program's in one launch when its event slots fit, else a segment's before it) and the
// segment kernel applies them at their layer.  Event = (tile word index of the qubit
// | pauli << 28, shot).  A block gathers its events in LDS and reserves space with one atomic.
// ------------------------------------------------------------------------------------------
constexpr int kNoiseThreads = 1024;
constexpr int kNoiseUnitsPerBlock = 4 * kNoiseThreads;
constexpr int kNoiseLdsEvents = 2048;
// event slots (8 bytes each) up to which a program's noise is drawn in one launch
constexpr long long kDrawAllEvents = 1ll << 28;

// Instruction y of nd[] (y = blockIdx.y, or reversed with rev).  seg_base (may be NULL): per
// instruction, the first event slot of its segment, when every segment's events are drawn by
// one launch.  The order of a bucket's events depends on block timing; applying them commutes.
__global__ void __launch_bounds__(1024)
k_noise_draw(const NoiseDesc* __restrict__ nd, const int* __restrict__ ntg, int B, uint64_t seed,
             uint64_t first_shot, uint64_t instr_base, uint2* __restrict__ events,
             const long long* __restrict__ seg_base, const int* __restrict__ ev_base, int* __restrict__ ev_count,
             unsigned long long* __restrict__ counters, int rev)
{
    __shared__ uint2 sev[kNoiseLdsEvents];
    __shared__ int s_n, s_base;
    const int bx = rev ? (int)gridDim.x - 1 - (int)blockIdx.x : (int)blockIdx.x;
    const int by = rev ? (int)gridDim.y - 1 - (int)blockIdx.y : (int)blockIdx.y;
    const NoiseDesc d = nd[by];
    const long long total = (long long)d.units * B;
    const long long start = (long long)bx * kNoiseUnitsPerBlock;
    if (start >= total) return;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    uint2* gdst = events + (seg_base ? seg_base[by] : 0ll) + ev_base[d.bucket];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const long long idx = start + threadIdx.x + (long long)j * kNoiseThreads;
        if (idx >= total) break;
        const int b = (int)(idx / d.units);
        const int pos = (int)(idx - (long long)b * d.units);
        uint64_t u0, u1;
        philox(instr_base + d.instr, (uint64_t)pos, seed, first_shot + (uint64_t)b, u0, u1);
        uint32_t e[2];
        int ne = 0;
        if (d.kind == STAB_KIND_DEP1) {
            if (u0 < d.t0) e[ne++] = (uint32_t)ntg[d.toff + pos] | ((uint32_t)(1 + (int)__umul64hi(u1, 3ull)) << 28);
        } else if (d.kind == STAB_KIND_DEP2) {
            if (u0 < d.t0) {
                const int k = 1 + (int)__umul64hi(u1, 15ull);
                if (k >> 2) e[ne++] = (uint32_t)ntg[d.toff + 2 * pos] | ((uint32_t)(k >> 2) << 28);
                if (k & 3) e[ne++] = (uint32_t)ntg[d.toff + 2 * pos + 1] | ((uint32_t)(k & 3) << 28);
            }
        } else {  // PAULI1 with cumulative thresholds
            const int P = (u0 < d.t0) ? 1 : (u0 < d.t1) ? 2 : (u0 < d.t2) ? 3 : 0;
            if (P) e[ne++] = (uint32_t)ntg[d.toff + pos] | ((uint32_t)P << 28);
        }
        for (int i = 0; i < ne; ++i) {
            const int slot = atomicAdd(&s_n, 1);
            const uint2 ev = make_uint2(e[i], (uint32_t)b);
            if (slot < kNoiseLdsEvents) sev[slot] = ev;
            else gdst[atomicAdd(&ev_count[d.bucket], 1)] = ev;   // LDS full: direct
        }
    }
    __syncthreads();
    const int n = min(s_n, kNoiseLdsEvents);
    if (threadIdx.x == 0 && s_n) count_add(counters, 7, (unsigned long long)s_n);
    if (n == 0) return;
    if (threadIdx.x == 0) s_base = atomicAdd(&ev_count[d.bucket], n);
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) gdst[s_base + i] = sev[i];
}

// ------------------------------------------------------------------------------------------
// Segment kernel helpers.  Column j of a staged half-band: x word at
// T[(j & 63) * RSP + (j >> 6)], z word at + Wc (32-bit words, one bit per staged row).
// ------------------------------------------------------------------------------------------
constexpr int kSegPrefetch = 5;   // gates / events per thread prefetched into registers

// Registers holding one item's gate or noise-event list (first kSegPrefetch * blockDim.x).
struct ItemBuf {
    uint2 v[kSegPrefetch];
    int count;     // units in the item
    int type;      // 0 gates, 1 noise, -1 none
    const uint2* src;
};

__device__ __forceinline__ void fetch_item(const SegArgs& a, int it, int tid, int nt, ItemBuf& b)
{
    if (it >= a.nitems) {
        b.type = -1;
        b.count = 0;
        return;
    }
    const int4 item = a.items[it];
    b.type = item.x;
    // gates: count known; events: the bucket's slots are read up to its capacity while its
    // count is loaded (both in flight at once), and the count bounds their use
    b.src = item.x == 0 ? a.gates + item.y : a.events + item.y;
    b.count = item.x == 0 ? item.z : a.ev_count[item.w];
#pragma unroll
    for (int u = 0; u < kSegPrefetch; ++u) {
        const int i = tid + u * nt;
        if (i < item.z) b.v[u] = b.src[i];
    }
}

// A gate on the 32 staged rows: x word of qubit q at T[(q & 63) * RSP + (q >> 6)], z at + Wc;
// the gate list holds these word indices (resolved on the host).
__device__ __forceinline__ void apply_gate(uint32_t* T, int Wc, uint2 gt, uint32_t& racc)
{
    const int kind = (int)(gt.x & 15u);
    const int i0 = (int)(gt.x >> 4);
    const uint32_t x0 = T[i0], z0 = T[i0 + Wc];
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
        const int i1 = (int)gt.y;
        const uint32_t x1 = T[i1], z1 = T[i1 + Wc];
        racc ^= x0 & z1 & ~(x1 ^ z0);
        T[i1] = x1 ^ x0;
        T[i0 + Wc] = z0 ^ z1;
    } break;
    default: break;
    }
}

// Noise event {tile word index of the qubit | pauli << 28, shot}: flip the signs of the rows the
// Pauli anticommutes with.
__device__ __forceinline__ void apply_event(const uint32_t* T, int Wc, uint2 v, int s, int hb,
                                            const Geom& g, const SegArgs& a, uint32_t* rdacc,
                                            uint32_t* rd32)
{
    const int sb = (int)v.y - s * g.bpc;
    if (sb < 0 || sb >= g.bpc) return;
    const int iq = (int)(v.x & 0x0FFFFFFFu), P = (int)(v.x >> 28);
    const uint32_t xq = T[iq], zq = T[iq + Wc];
    const uint32_t m = (P == 1) ? zq : (P == 3) ? xq : (xq ^ zq);
    if (m) {
        if (a.lds_rd) atomicXor(&rdacc[sb], m);
        else atomicXor(&rd32[(size_t)(s * g.bpc + sb) * 2 * g.NB + hb], m);
    }
}

// In-register transpose of the 32x32 bit matrix held by each half-wave, one row per lane
// (bit c of lane r's word = element (r, c)); lanes 32..63 transpose their own matrix.
__device__ __forceinline__ uint32_t transpose32(uint32_t v, int lane)
{
    const uint32_t masks[5] = {0x0000FFFFu, 0x00FF00FFu, 0x0F0F0F0Fu, 0x33333333u, 0x55555555u};
#pragma unroll
    for (int st = 0; st < 5; ++st) {
        const int j = 16 >> st;
        const uint32_t m = masks[st];
        const uint32_t o = lane_xor32(v, j, lane);
        if (lane & j) {
            v ^= ((o >> j) ^ v) & m;
        } else {
            v ^= (((v >> j) ^ o) & m) << j;
        }
    }
    return v;
}

// Transpose every 32x32 tile (column c of the 64 staged lanes) in place, four tiles per wave in
// flight so that their LDS reads overlap.  A wave's pair of tiles that is all zero (most of a
// sparse tableau, such as a surface code's) is its own transpose and is left as it is.
__device__ __forceinline__ void transpose_tiles(uint32_t* T, int RSP, int RS, int lane, int wave, int nwaves)
{
    int c = wave;
    for (; c + 3 * nwaves < RS; c += 4 * nwaves) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = T[lane * RSP + c + u * nwaves];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (__ballot(v[u] != 0u)) {
                v[u] = transpose32(v[u], lane);
                T[lane * RSP + c + u * nwaves] = v[u];
            }
        }
    }
    for (; c < RS; c += nwaves) {
        const uint32_t v = T[lane * RSP + c];
        if (__ballot(v != 0u)) T[lane * RSP + c] = transpose32(v, lane);
    }
}

// ------------------------------------------------------------------------------------------
// Segment kernel: grid (2 * NB half-bands, S copies), 1024 threads.  A block stages 32 rows
// (half of a 64-row band) as 32-bit qubit-major words: row r's 64-bit word c is split into
// its low half (columns 64c..64c+31, staged at lane r) and high half (lane 32 + r); each
// half-wave then transposes its 32x32 tile, so afterwards lane L of tile c holds column
// 64c + L for the 32 rows.  Two such blocks fit the LDS of one compute unit.  The block owns
// the 32-bit half of every sign word and column-extract word of its band.
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8)))
k_segment(Geom g, uint64_t* __restrict__ tab, uint64_t* __restrict__ rs,
          uint64_t* __restrict__ rd, SegArgs a)
{
    if (a.gate && *a.gate == 0) return;   // an extraction pass with nothing to refresh
    extern __shared__ uint32_t lds32[];
    const int hb = blk_x(g);                     // half-band: band = hb >> 1, half = hb & 1
    const int band = hb >> 1, half = hb & 1;
    const int s = blk_y(g);
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
    const int RS = g.RS, RSP = g.RS + 1, Wc = g.Wc;
    uint32_t* T = lds32;                         // 64 x RSP
    uint32_t* red = lds32 + 64 * RSP;            // nwaves words
    uint32_t* rdacc = red + 16;                  // bpc words when a.lds_rd
    uint64_t* gb = tab + ((size_t)s * 2 * g.NR + (size_t)band * 64 + (size_t)half * 32) * RS;
    uint32_t* rs32 = (uint32_t*)rs;
    uint32_t* rd32 = (uint32_t*)rd;

    ItemBuf cur, nxt;
    fetch_item(a, 0, tid, nt, cur);

    // 32 rows -> LDS with 16-byte loads (RS is even, so a pair never crosses a row), 4 in
    // flight; word (r, c) splits into T[r][c] (low half) and T[32 + r][c] (high half)
    const int npairs = 16 * RS;
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
                uint32_t* lo = T + r * RSP + c;
                uint32_t* hi = lo + 32 * RSP;
                lo[0] = (uint32_t)v[u].x;
                lo[1] = (uint32_t)v[u].y;
                hi[0] = (uint32_t)(v[u].x >> 32);
                hi[1] = (uint32_t)(v[u].y >> 32);
            }
        }
    }
    if (a.lds_rd)
        for (int b = tid; b < g.bpc; b += nt) rdacc[b] = 0;
    __syncthreads();
    transpose_tiles(T, RSP, RS, lane, wave, nwaves);
    __syncthreads();

    uint32_t racc = 0;
    for (int it = 0; it < a.nitems; ++it) {
        fetch_item(a, it + 1, tid, nt, nxt);       // next item's list, in flight meanwhile
        if (cur.type == 0) {
#pragma unroll
            for (int u = 0; u < kSegPrefetch; ++u)
                if (tid + u * nt < cur.count) apply_gate(T, Wc, cur.v[u], racc);
            for (int gi = tid + kSegPrefetch * nt; gi < cur.count; gi += nt)
                apply_gate(T, Wc, cur.src[gi], racc);
        } else {
#pragma unroll
            for (int u = 0; u < kSegPrefetch; ++u)
                if (tid + u * nt < cur.count) apply_event(T, Wc, cur.v[u], s, 2 * band + half, g, a, rdacc, rd32);
            for (int e = tid + kSegPrefetch * nt; e < cur.count; e += nt)
                apply_event(T, Wc, cur.src[e], s, 2 * band + half, g, a, rdacc, rd32);
        }
        __syncthreads();
        cur = nxt;
    }

    if (a.K > 0) {
        uint32_t* Xc = (uint32_t*)(a.Xcol + ((size_t)s * g.NB + band) * a.K);
        uint32_t* Zc = (uint32_t*)(a.Zcol + ((size_t)s * g.NB + band) * a.K);
        for (int k = tid; k < a.K; k += nt) {
            const int q = a.ext_q[k];
            const int iq = (q & 63) * RSP + (q >> 6);
            Xc[2 * k + half] = T[iq];
            Zc[2 * k + half] = T[iq + Wc];
        }
    }
    if (a.write_back) {
        __syncthreads();
        transpose_tiles(T, RSP, RS, lane, wave, nwaves);
        __syncthreads();
        ulonglong2* gw2 = (ulonglong2*)gb;
        for (int p = tid; p < npairs; p += nt) {
            const int i = 2 * p;
            const int r = i / RS;
            const int c = i - r * RS;
            const uint32_t* lo = T + r * RSP + c;
            const uint32_t* hi = lo + 32 * RSP;
            ulonglong2 v;
            v.x = (uint64_t)lo[0] | ((uint64_t)hi[0] << 32);
            v.y = (uint64_t)lo[1] | ((uint64_t)hi[1] << 32);
            gw2[p] = v;
        }
    }
    // sign contributions: XOR-reduce 32-bit masks
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) racc ^= (uint32_t)__shfl_xor((int)racc, m, 64);
    if (lane == 0) red[wave] = racc;
    __syncthreads();
    if (tid == 0) {
        uint32_t t = 0;
        for (int w = 0; w < nwaves; ++w) t ^= red[w];
        if (t) rs32[((size_t)s * g.NB + band) * 2 + half] ^= t;
    }
    if (a.lds_rd) {
        for (int b = tid; b < g.bpc; b += nt) {
            const uint32_t v = rdacc[b];
            if (v) rd32[((size_t)(s * g.bpc + b) * g.NB + band) * 2 + half] ^= v;
        }
    }
}

// ------------------------------------------------------------------------------------------
// Classification and deterministic outcomes of a measurement layer (Sec. 2.4), one wave per
// (copy, target).
//
// pass 0, at layer start: the block's eight consecutive targets have their x columns staged in
// LDS first (a band's eight words are contiguous in Xcol, so the loads are coalesced), then a
// wave takes each target's column one word per 64-row band and lane.  The first stabilizer with x at the qubit is the pivot: the target is
// random, its class is that stabilizer index (the random chain takes it).  Without one the
// outcome is deterministic: +-Z_a is the product of the stabilizers NR + i over the
// destabilizers i with x at the qubit (class -1).  pass 1, after the chain on the final
// tableau (only when a random target ran): the targets the chain marked deterministic (-2)
// are reduced and marked -3.  A deterministic outcome is unchanged by Z measurements and
// resets on other qubits, so every one of a layer is reduced in parallel (the paper
// serialises every row behind two grid barriers, Alg. 2).
//
// The product.  The destabilizer bits are enumerated in row order (ballot, then scalar loops
// over the few nonzero words), 64 rows at a time with lane c holding the c-th; rows are loaded
// kDetRowBatch at a time (no load conditional, so a batch is in flight at once).  Its phase is
// telescoped: with |u| the number of qubits where u has both x and z, multiplying rows into
// the scratch row S raises i to sum|row| - |S| + 2 sum z_row.x_S (mod 4), and only the parity
// of the last sum matters, so it is XOR-accumulated and popcounted once.  The per-shot part of
// the sign is the parity of each shot's sign bits over the same rows; the bits of a shot group
// of 64 gather in LDS (nrdw words per wave).
// ------------------------------------------------------------------------------------------
// targets (waves) per block: four with one-word rows (small tableaux: more blocks in flight),
// eight otherwise (a band's eight column words are one coalesced 64-byte read)
constexpr int det_targets(int wpl) { return wpl == 1 ? 4 : 8; }
constexpr int kDetRowBatch = 3;                // rows a wave loads at once

// WPL = ceil(Wc / 64): column words (and stabilizer bands) a lane holds of a row.
template <int WPL>
__global__ void __launch_bounds__(64 * det_targets(WPL)) __attribute__((amdgpu_waves_per_eu(4)))
k_det(Geom g, const uint64_t* __restrict__ tab, const uint64_t* __restrict__ rs,
      const uint64_t* __restrict__ rd, const uint64_t* __restrict__ Xcol, int K, int* __restrict__ cls,
      uint8_t* __restrict__ obuf, int* __restrict__ ran, int* __restrict__ err,
      unsigned long long* __restrict__ counters, int pass, int* __restrict__ ran_log)
{
    extern __shared__ uint64_t dsm[];
    constexpr int kDetTargets = det_targets(WPL);
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int k0 = blk_x(g) * kDetTargets, k = k0 + wave;
    const int s = blk_y(g);
    const int NB = g.NB, nrdw = (g.bpc + 63) >> 6;
    uint64_t* colw = dsm;                                          // [kDetTargets][NB] columns
    uint64_t* parw = dsm + (size_t)kDetTargets * NB + (size_t)wave * nrdw;   // shot parity bits
    // the block's work counters, flushed with one atomic each at the end
    __shared__ unsigned int s_det, s_rows;
    if (threadIdx.x == 0) {
        s_det = 0;
        s_rows = 0;
    }
    if (pass == 0) {
        // the next launch (the random chain) sets this when a random target runs
        if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *ran = 0;
    } else {
        // (ran_log, when given: whether a target of this layer ran, for the host)
        const int r = *ran;
        if (ran_log && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *ran_log = r;
        if (r == 0) return;
    }
    const uint64_t* X = Xcol + (size_t)s * NB * K;
    // eight words per thread at a time: all loads in flight before the LDS stores
    const int tot = NB * kDetTargets;
    for (int i0 = threadIdx.x; i0 < tot; i0 += 8 * (int)blockDim.x) {
        uint64_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            const int w = i / kDetTargets, j = i - w * kDetTargets;
            v[u] = (i < tot && k0 + j < K) ? X[(size_t)w * K + k0 + j] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            const int w = i / kDetTargets, j = i - w * kDetTargets;
            if (i < tot) colw[j * NB + w] = v[u];
        }
    }
    __syncthreads();
    // one wave per target; a wave that is done returns from here
    [&]() {
        if (k >= K) return;
        if (pass == 1 && cls[s * K + k] != -2) return;
        const uint64_t* tb = tab + (size_t)s * 2 * g.NR * g.RS;
        const uint64_t* rsc = rs + (size_t)s * NB;
        // the column: destabilizer words cd, stabilizer words cs (band lane + 64 u of each half)
        uint64_t cd[WPL], cs[WPL];
#pragma unroll
        for (int u = 0; u < WPL; ++u) {
            const int w = lane + 64 * u;
            cd[u] = w < g.Wr ? colw[wave * NB + w] : 0ull;
            cs[u] = w < g.Wr && pass == 0 ? colw[wave * NB + g.Wr + w] : 0ull;
        }
        if (pass == 0) {
#pragma unroll
            for (int u = 0; u < WPL; ++u) {
                const uint64_t m = __ballot(cs[u] != 0ull);
                if (m) {
                    const int l = ctz64(m);
                    if (lane == 0) cls[s * K + k] = (l + 64 * u) * 64 + ctz64(readlane_u64(cs[u], l));
                    return;                              // random at layer start
                }
            }
        }
        if (lane == 0) cls[s * K + k] = pass == 0 ? -1 : -3;
        for (int u = lane; u < nrdw; u += 64) parw[u] = 0;
        const uint64_t* base = tb + (size_t)g.NR * g.RS;
        int jc[WPL];
        uint64_t msk[WPL], sx[WPL], sz[WPL], cr[WPL];
#pragma unroll
        for (int t = 0; t < WPL; ++t) {
            const int j = lane + 64 * t;
            jc[t] = j < g.Wc ? j : 0;
            msk[t] = j < g.Wc ? ~0ull : 0ull;
            sx[t] = sz[t] = cr[t] = 0;
        }
        int G = 0, rsum = 0, cnt = 0, nc = 0, myrow = 0;
        // multiply the nc listed rows (lane c holds the c-th) into S, and their shot sign bits
        auto flush = [&]() {
            // nothing below depends on a row's contents except the product itself, so with
            // one-word rows the first batch of rows, the listed rows' shared sign words and the
            // shots' sign words are requested together: one round trip instead of three.  With
            // wider rows the registers that holds cost more occupancy than the round trips save
            // (d=71: 71 -> 90 VGPRs and the pass 18 % slower), so they go one after another.
            uint64_t rx[kDetRowBatch][WPL], rz[kDetRowBatch][WPL];
            auto load = [&](int u0) {
#pragma unroll
                for (int u = 0; u < kDetRowBatch; ++u) {
                    const int i = __shfl(myrow, min(u0 + u, nc - 1), 64);
                    const uint64_t* row = base + (size_t)i * g.RS;
#pragma unroll
                    for (int t = 0; t < WPL; ++t) {
                        rx[u][t] = row[jc[t]];
                        rz[u][t] = row[g.Wc + jc[t]];
                    }
                }
            };
            auto parity = [&]() {
                for (int b0 = 0; b0 < g.bpc; b0 += 64) {
                    const uint64_t* rdb = rd + (size_t)(s * g.bpc + min(b0 + lane, g.bpc - 1)) * g.NB + g.Wr;
                    int par = 0;
                    for (int c = 0; c < nc; c += 8) {
                        int iu[8];
                        uint64_t wv[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) iu[u] = __shfl(myrow, min(c + u, nc - 1), 64);
#pragma unroll
                        for (int u = 0; u < 8; ++u) wv[u] = rdb[iu[u] >> 6];
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            if (c + u < nc) par ^= (int)((wv[u] >> (iu[u] & 63)) & 1ull);
                    }
                    const uint64_t pb = __ballot(par & 1);
                    if (lane == 0) parw[b0 >> 6] ^= pb;
                }
            };
            uint64_t rsw;
            if (WPL == 1) {
                load(0);
                rsw = rsc[g.Wr + ((lane < nc ? myrow : 0) >> 6)];
                parity();
            } else {
                rsw = rsc[g.Wr + ((lane < nc ? myrow : 0) >> 6)];
            }
            rsum += __popcll(__ballot(lane < nc && ((rsw >> (myrow & 63)) & 1ull)));
            for (int u0 = 0; u0 < nc; u0 += kDetRowBatch) {
                if (u0 > 0 || WPL != 1) load(u0);
#pragma unroll
                for (int u = 0; u < kDetRowBatch; ++u) {
                    if (u0 + u >= nc) break;
#pragma unroll
                    for (int t = 0; t < WPL; ++t) {
                        const uint64_t a = rx[u][t] & msk[t], b = rz[u][t] & msk[t];
                        cr[t] ^= b & sx[t];
                        G += __popcll(a & b);
                        sx[t] ^= a;
                        sz[t] ^= b;
                    }
                }
            }
            if (WPL != 1) parity();
            cnt += nc;
            nc = 0;
        };
#pragma unroll
        for (int u = 0; u < WPL; ++u) {
            uint64_t lanes = __ballot(cd[u] != 0ull);
            while (lanes) {
                const int l = ctz64(lanes);
                lanes &= lanes - 1;
                uint64_t v = readlane_u64(cd[u], l);
                const int wb = l + 64 * u;
                while (v) {
                    const int bit = ctz64(v);
                    v &= v - 1;
                    if (lane == nc) myrow = wb * 64 + bit;
                    if (++nc == 64) flush();
                }
            }
        }
        if (nc) flush();
        uint64_t xres = 0;
#pragma unroll
        for (int t = 0; t < WPL; ++t) {
            G += 2 * __popcll(cr[t]) - __popcll(sx[t] & sz[t]);
            xres |= sx[t];
        }
        G = wave_sum(G);
        xres = wave_or(xres);
        const int e = (2 * rsum + G) & 3;
        if (lane == 0 && ((e & 1) || xres)) atomicOr(err, 1);
        const int shared = e >> 1;
        for (int b = lane; b < g.bpc; b += 64)
            obuf[(size_t)(s * g.bpc + b) * K + k] = (uint8_t)(shared ^ (int)((parw[b >> 6] >> (b & 63)) & 1ull));
        if (lane == 0) {
            atomicAdd(&s_det, 1u);
            atomicAdd(&s_rows, (unsigned int)cnt);
        }
    }();
    __syncthreads();
    if (threadIdx.x == 0 && s_det) {
        count_add(counters, pass == 0 ? 2 : 6, (unsigned long long)s_det);
        count_add(counters, 3, (unsigned long long)s_rows);
    }
}

// ------------------------------------------------------------------------------------------
// Random-at-start targets of a measurement layer, one block per tableau copy.
//
// Sequential semantics (Sec. 2.4): targets are measured in op order; each may have turned
// deterministic because of an earlier one in the same layer.  A random one: pivot p = first
// stabilizer with x at the qubit; rowsum(i, p) for every other row i with x at the qubit; the
// pivot's destabilizer q <- old row p (its own rowsum is overwritten); p <- Z_a with the
// outcome as sign.  A deterministic one reads the stabilizers selected by the destabilizers
// with x at the qubit.
//
// Split of the work.  Nothing a later target of the layer decides on (its pivot, its row
// list, its outcome) depends on destabilizer rows, so this kernel runs the stabilizer half
// only and logs each executed target's old pivot row with its signs; k_replay then applies
// the destabilizer updates (rowsums and the q <- p moves) in op order, one wave per touched
// destabilizer, all rows in parallel.  Targets that turn deterministic are marked and
// reduced after the layer on the final tableau.
//
// Batching: the block looks at a window of the next pending targets.  A target's stabilizer
// rows are its pivot and the other stabilizers with x at its qubit.  Target t of the window
// runs now iff none of its stabilizer rows belongs to an earlier window target (run or
// deferred).  Such targets touch disjoint rows, and every later target whose inputs an
// earlier one could change shares a row with it (the earlier pivot would have x at the later
// qubit), so running them at once gives exactly the sequential result; shared words (signs,
// target columns) are updated with XOR, AND and OR atomics on distinct bits.  A target
// touching more than kRCap rows runs alone, with the whole block.  The stabilizer half of
// Xcol is kept equal to the current tableau's x columns of the pending targets; the whole of
// Xcol/Zcol is extracted again after the replay.
// ------------------------------------------------------------------------------------------
enum { T_RANDOM = 0, T_DET = 1, T_BIG_RANDOM = 2, T_BIG_DET = 3, T_UNKNOWN = 4, T_DEAD = 5 };

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m, 64));
    return v;
}

__device__ __forceinline__ int wave_excl_scan(int v, int lane)
{
    int incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    return incl - v;
}

struct ChainCtx {
    Geom g;
    uint64_t* tb;        // this copy's tableau
    uint64_t* rs;        // this copy's sign words
    uint64_t* rd;        // all shots' sign words
    uint64_t* X;         // this copy's Xcol
    uint64_t* Z;
    int K, s;
    const int* tq;
    int16_t* tm;             // (LDS) qubit -> pending target whose x column is kept, or -1
    int* cl;                 // this copy's target classes (-2 marks "deterministic now")
    int* lp;                 // pivot log: stabilizer index of target k's pivot (-1: not run)
    uint64_t* lrow;          // old pivot row of target k (RS words)
    int* lrs;                // its shared sign
    uint64_t* lrd;           // its per-shot signs (nrdw words, bit b = shot b of the copy)
    int nrdw;
    int* ran;                // set to 1 when any random target of the layer runs
    uint16_t* plist;         // per run target k: pending targets whose qubit has x in its pivot
    int* pcnt;               // their count (kPListCap at most; *povf = 1 beyond)
    int* povf;
    uint64_t seed, first_shot, instr;
    int pos_base;
    uint8_t* obuf;
    int* err;
    unsigned long long* counters;
    unsigned int* lcnt;      // (LDS) random measurements and stabilizer rows updated, flushed at the end
};

// Pending target k2 has x in the pivot row of target k: the replay must flip that bit of a
// destabilizer it multiplies by the pivot.
__device__ __forceinline__ void plist_add(const ChainCtx& c, int k, int k2)
{
    const int slot = atomicAdd(&c.pcnt[k], 1);
    if (slot < kPListCap) c.plist[(size_t)k * kPListCap + slot] = (uint16_t)k2;
    else *c.povf = 1;
}

// Outcome draw of target k for global shot index b.
__device__ __forceinline__ int outcome_bit(const ChainCtx& c, int k, int b)
{
    uint64_t u0, u1;
    philox(c.instr, (uint64_t)(c.pos_base + k), c.seed, c.first_shot + (uint64_t)b, u0, u1);
    return (int)(u0 >> 63);
}

// v is the same in every lane (the compiler cannot see that for values read from LDS): keeping
// it in a scalar register makes loops over it scalar loops.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// An empty asm that takes v in a VGPR and may change it: the compiler waits for v's load here
// (not at a later first use that some paths skip) and keeps work that uses v below this point.
__device__ __forceinline__ void settle(uint64_t& v) { asm volatile("" : "+v"(v)); }

// rowsum(i, p) for rows[r], r = r0, r0 + stride, ... < nrows, pivot row words in registers
// (lane owns column words lane + 64 t, WPL = ceil(Wc / 64)).  Sign r_i <- r_i ^ r_p ^
// (i-power / 2).  Every batch loads RB rows (the last row again past nrows, a stabilizer row
// when there is none) and settles every loaded word, so the number of loads in flight never
// depends on the path taken and no load is left pending for a later loop to wait on: the
// first batch's loads are issued before anything waits for the pivot row, whose loads (and the
// caller's pend[] words, loaded before it) are settled right after.  r_p = bit rbit of pend[0].
template <int WPL, int NP>
__device__ __forceinline__ void rowsum_rows(const ChainCtx& c, uint64_t* xp, uint64_t* zp, uint64_t (&pend)[NP],
                                            int rbit, const int* rows, int nrows, int r0, int stride, int lane)
{
    const Geom& g = c.g;
    const int Wc = g.Wc, RS = g.RS;
    nrows = uni(nrows);
    r0 = uni(r0);
    stride = uni(stride);
    rbit = uni(rbit);
    // rows in flight: four, three when a lane holds three or more words of a row
    constexpr int RB = WPL <= 2 ? 4 : 3;
    uint64_t rx[RB][WPL], rz[RB][WPL];
    auto row_of = [&](int r) { return nrows > 0 ? rows[min(r, nrows - 1)] : g.NR; };
    auto load = [&](int rb) {
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const uint64_t* row = c.tb + (size_t)row_of(rb + u * stride) * RS;
#pragma unroll
            for (int t = 0; t < WPL; ++t) {
                // (lanes past Wc read the last word and hold a zero pivot word)
                const int cw = min(lane + 64 * t, Wc - 1);
                rx[u][t] = row[cw];
                rz[u][t] = row[Wc + cw];
            }
        }
    };
    load(r0);
#pragma unroll
    for (int t = 0; t < WPL; ++t) {
        settle(xp[t]);
        settle(zp[t]);
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) settle(pend[i]);
    const int rsp = (int)((pend[0] >> rbit) & 1ull);
    for (int rb = r0;;) {
        // the batch's words are taken here, whether or not a row is past nrows
#pragma unroll
        for (int u = 0; u < RB; ++u)
#pragma unroll
            for (int t = 0; t < WPL; ++t) {
                settle(rx[u][t]);
                settle(rz[u][t]);
            }
        // only the i-power mod 4 matters: byte u of P sums row u's per-lane residues (at most
        // 64 x 3), so one wave sum serves the batch
        int P = 0;
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int r = rb + u * stride;
            int G = 0;
#pragma unroll
            for (int t = 0; t < WPL; ++t) G += gsum(xp[t], zp[t], rx[u][t], rz[u][t]);
            if (r < nrows) {
                uint64_t* row = c.tb + (size_t)rows[r] * RS;
#pragma unroll
                for (int t = 0; t < WPL; ++t) {
                    const int cw = lane + 64 * t;
                    if (cw < Wc && (xp[t] | zp[t])) {
                        row[cw] = rx[u][t] ^ xp[t];
                        row[Wc + cw] = rz[u][t] ^ zp[t];
                    }
                }
                P |= (G & 3) << (8 * u);
            }
        }
        P = wave_sum_uniform(P, lane);
        if (lane == 0) {
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const int r = rb + u * stride;
                if (r < nrows) {
                    const int G = (P >> (8 * u)) & 3;
                    const int i = rows[r];
                    if (G & 1) atomicOr(c.err, 4);
                    const uint64_t flip = (uint64_t)((rsp ^ (G >> 1)) & 1) << (i & 63);
                    if (flip) atomicXor((unsigned long long*)&c.rs[i >> 6], (unsigned long long)flip);
                }
            }
        }
        rb += RB * stride;
        if (rb >= nrows) break;
        load(rb);
    }
}

// The rest of a random measurement, one wave: per-shot signs of the rowsum rows and the
// outcomes, the pending targets' x columns at the rowsum rows and at p, the pivot log entry
// (old row p with its signs, for the destabilizer replay) and p <- Z_a.  xp, zp: the old row p
// (lane owns column words lane + 64 t).  rows[] (stabilizer rows) is sorted, so runs in one
// 64-row word are applied as one word mask.  Column upkeep follows tmap (k >= 0: the pending
// target whose x column is kept).  When `aff` is given (wide batches), the per-target column
// work is appended there as {target, 0, batch index j} for the whole block to apply; it is
// done in-wave otherwise or when the list is full.
template <int WPL>
__device__ void random_epilogue(const ChainCtx& c, int k, int a, int ip, int rsp, const uint64_t* xp,
                                const uint64_t* zp, const int* rows, int nrows, int lane,
                                int* aff = nullptr, int* aff_n = nullptr, int j = 0,
                                bool have_rd0 = false, uint64_t rd0 = 0, uint64_t rd1 = 0,
                                int out0 = 0, int out1 = 0)
{
    const Geom& g = c.g;
    const int Wc = g.Wc, Wr = g.Wr, NB = g.NB, RS = g.RS, K = c.K;
    k = uni(k);
    a = uni(a);
    ip = uni(ip);
    rsp = uni(rsp);
    nrows = uni(nrows);
    j = uni(j);
    uint64_t* gp = c.tb + (size_t)(g.NR + ip) * RS;
    const int wq = ip >> 6;
    const uint64_t bq = 1ull << (ip & 63);
    uint64_t* lrow = c.lrow + (size_t)k * RS;
#pragma unroll
    for (int t = 0; t < WPL; ++t) {
        const int cw = lane + 64 * t;
        if (cw < Wc) {
            lrow[cw] = xp[t];
            lrow[Wc + cw] = zp[t];
        }
    }
    if (lane == 0) {
        c.lrs[k] = rsp;
        c.lp[k] = ip;
        *c.ran = 1;
        atomicAnd((unsigned long long*)&c.rs[Wr + wq], ~(unsigned long long)bq);
    }
    // the rowsum rows as word runs, read out as scalars by every loop below
    uint64_t hm[2], mv[2];
    int wv[2];
    row_runs(rows, nrows, lane, hm, wv, mv);
    // 64 shots: rw = each shot's pivot sign word, out = its outcome draw
    auto shots = [&](int b0, uint64_t rw, int out) {
        const int b = b0 + lane;
        const bool in = b < g.bpc;
        const int gb = c.s * g.bpc + min(b, g.bpc - 1);
        uint64_t* rdb = c.rd + (size_t)gb * NB;
        const bool rdp = in && ((rw >> (ip & 63)) & 1ull) != 0;
        if (in) {
            // the pivot's sign becomes the outcome (no rowsum row is the pivot)
            if ((int)rdp != out) atomicXor((unsigned long long*)&rdb[Wr + wq], (unsigned long long)bq);
            c.obuf[(size_t)gb * K + k] = (uint8_t)out;
        }
        for_runs(hm, wv, mv, [&](int w, uint64_t m) {
            if (rdp) atomicXor((unsigned long long*)&rdb[w], (unsigned long long)m);
        });
        const uint64_t m = __ballot(rdp);
        if (lane == 0) c.lrd[(size_t)k * c.nrdw + (b0 >> 6)] = m;
    };
    int b0 = 0;
    if (have_rd0) {
        // the first 128 shots' sign words and draws came with the pivot row: no load waits here
        shots(0, rd0, out0);
        if (g.bpc > 64) shots(64, rd1, out1);
        b0 = 128;
    }
    for (; b0 < g.bpc; b0 += 64) {
        const int gb = c.s * g.bpc + min(b0 + lane, g.bpc - 1);
        shots(b0, c.rd[(size_t)gb * NB + Wr + wq], outcome_bit(c, k, gb));
    }
    // x columns of pending targets: rows with x at the pivot's qubits flip there; p's x clears
    auto upkeep = [&](int k2) {
        unsigned long long* X2 = (unsigned long long*)(c.X + k2);
        for_runs(hm, wv, mv, [&](int w, uint64_t m) { atomicXor(&X2[(size_t)w * K], (unsigned long long)m); });
        atomicAnd(&X2[(size_t)(Wr + wq) * K], ~(unsigned long long)bq);
    };
    if (aff) {
#pragma unroll
        for (int t = 0; t < WPL; ++t) {
            const int cw = lane + 64 * t;
            if (cw >= Wc) continue;
            uint64_t bits = xp[t];
            while (bits) {
                const int bit = ctz64(bits);
                bits &= bits - 1;
                const int k2 = c.tm[cw * 64 + bit];
                if (k2 < 0 || k2 == k) continue;
                const int slot = atomicAdd(aff_n, 1);
                if (slot < kAffCap) {
                    aff[3 * slot] = k2;
                    aff[3 * slot + 1] = 0;
                    aff[3 * slot + 2] = j;
                    continue;
                }
                plist_add(c, k, k2);
                upkeep(k2);
            }
        }
    } else {
        // this wave is the only writer of target k's list: slots by ballot rank, no atomics
        int np = 0;
#pragma unroll
        for (int t = 0; t < WPL; ++t) {
            const int cw = lane + 64 * t;
            uint64_t bits = cw < Wc ? xp[t] : 0ull;
            while (__ballot(bits != 0ull)) {
                int k2 = -1;
                if (bits) {
                    const int bit = ctz64(bits);
                    bits &= bits - 1;
                    k2 = c.tm[cw * 64 + bit];
                }
                const bool hit = k2 >= 0 && k2 != k;
                const uint64_t hm = __ballot(hit);
                if (hit) {
                    const int slot = np + __popcll(hm & ((1ull << lane) - 1ull));
                    if (slot < kPListCap) c.plist[(size_t)k * kPListCap + slot] = (uint16_t)k2;
                    upkeep(k2);
                }
                np += __popcll(hm);
            }
        }
        if (lane == 0 && np) {
            c.pcnt[k] = np;
            if (np > kPListCap) *c.povf = 1;
        }
    }
#pragma unroll
    for (int t = 0; t < WPL; ++t) {
        const int cw = lane + 64 * t;
        if (cw < Wc) {
            gp[cw] = 0ull;
            gp[Wc + cw] = (cw == (a >> 6)) ? (1ull << (a & 63)) : 0ull;
        }
    }
    // this target's x column is never read again
    if (lane == 0) c.tm[a] = -1;
    if (lane == 0) {
        atomicAdd(&c.lcnt[0], 1u);
        atomicAdd(&c.lcnt[1], (unsigned int)nrows);
    }
}

// Load one row's words for this lane (from global or LDS).
template <int WPL>
__device__ __forceinline__ void load_row_lane(const uint64_t* row, int Wc, int lane, uint64_t* x, uint64_t* z)
{
#pragma unroll
    for (int t = 0; t < WPL; ++t) {
        const int cw = lane + 64 * t;
        const bool in = cw < Wc;
        x[t] = in ? row[cw] : 0ull;
        z[t] = in ? row[Wc + cw] : 0ull;
    }
}

// One wave: the whole random measurement of target k (pivot stabilizer index ip).
template <int WPL>
__device__ void wave_random(const ChainCtx& c, int k, int ip, const int* rows, int nrows, int lane)
{
    const Geom& g = c.g;
    k = uni(k);
    ip = uni(ip);
    nrows = uni(nrows);
    // the pivot's sign words (first 128 shots), its rs bit and the target's qubit are read
    // first, then the pivot row: waiting for the row also covers them
    const uint64_t rd0 = lane < g.bpc ? c.rd[(size_t)(c.s * g.bpc + lane) * g.NB + g.Wr + (ip >> 6)] : 0ull;
    const uint64_t rd1 =
        lane + 64 < g.bpc ? c.rd[(size_t)(c.s * g.bpc + 64 + lane) * g.NB + g.Wr + (ip >> 6)] : 0ull;
    const uint64_t rsw = c.rs[g.Wr + (ip >> 6)];
    const int a = c.tq[k];
    uint64_t xp[WPL], zp[WPL];
    const uint64_t* prow = c.tb + (size_t)(g.NR + ip) * g.RS;
    // (lanes past Wc load nothing and hold zeros, so nothing waits for the row before the
    // rowsum rows' loads are issued)
#pragma unroll
    for (int t = 0; t < WPL; ++t) {
        xp[t] = zp[t] = 0ull;
        if (lane + 64 * t < g.Wc) {
            xp[t] = prow[lane + 64 * t];
            zp[t] = prow[g.Wc + lane + 64 * t];
        }
    }
    // the outcome draws depend on the key and the target only: made while the loads are in flight
    const int gb0 = c.s * g.bpc + lane;
    const int out0 = lane < g.bpc ? outcome_bit(c, k, gb0) : 0;
    const int out1 = lane + 64 < g.bpc ? outcome_bit(c, k, gb0 + 64) : 0;
    uint64_t pend[4] = {rsw, rd0, rd1, (uint64_t)(uint32_t)a};
    rowsum_rows<WPL>(c, xp, zp, pend, ip & 63, rows, nrows, 0, 1, lane);
    const int rsp = (int)((pend[0] >> (ip & 63)) & 1ull);
    random_epilogue<WPL>(c, k, (int)(uint32_t)pend[3], ip, rsp, xp, zp, rows, nrows, lane, nullptr, nullptr, 0, true,
                         pend[1], pend[2], out0, out1);
}

// Whole block: one target with many stabilizer rows (dense tableaux).  Called by every thread.
__device__ void block_solo(const ChainCtx& c, int k, uint64_t* sm, int tid, int nt)
{
    const Geom& g = c.g;
    const int lane = tid & 63, wave = uni(tid >> 6), nwaves = nt >> 6;
    const int Wc = g.Wc, Wr = g.Wr, NB = g.NB, RS = g.RS, K = c.K;
    const int nrdw = c.nrdw;
    uint64_t* rowp = sm;
    uint64_t* sM = rowp + RS;      // stabilizer words w = 0..Wr-1 (rows NR + 64 w ...)
    uint64_t* sC = sM + Wr;
    uint64_t* sRdp = sC + Wr;
    int* nz = (int*)(sRdp + nrdw);
    __shared__ int s_piv, s_nnz, s_rsp;
    const int a = c.tq[k];
    uint64_t* X = c.X;
    uint64_t* tb = c.tb;

    if (tid == 0) {
        s_piv = INT_MAX;
        s_nnz = 0;
    }
    __syncthreads();
    for (int w = tid; w < Wr; w += nt) {
        const uint64_t v = X[(size_t)(Wr + w) * K + k];
        if (v) atomicMin(&s_piv, w * 64 + ctz64(v));
    }
    __syncthreads();
    const int ip = uni(s_piv);
    if (ip == INT_MAX) {
        // deterministic now: reduced after the layer on the final tableau
        if (tid == 0) c.cl[k] = -2;
        __syncthreads();
        return;
    }
    // gather the pivot row and the stabilizer rows with x at the qubit
    const int wq = ip >> 6;
    const uint64_t bq = 1ull << (ip & 63);
    uint64_t* gp = tb + (size_t)(g.NR + ip) * RS;
    for (int j = tid; j < RS; j += nt) rowp[j] = gp[j];
    for (int w = tid; w < Wr; w += nt) {
        uint64_t v = X[(size_t)(Wr + w) * K + k];
        if (w == wq) v &= ~bq;
        sM[w] = v;
        sC[w] = 0;
        if (v) nz[atomicAdd(&s_nnz, 1)] = w;
    }
    for (int t = tid; t < nrdw; t += nt) sRdp[t] = 0;
    if (tid == 0) s_rsp = (int)((c.rs[Wr + wq] >> (ip & 63)) & 1ull);
    __syncthreads();
    // per-shot pivot signs; rowsum(i, p), one row per wave at a time
    for (int b = tid; b < g.bpc; b += nt) {
        const uint64_t bit = (c.rd[(size_t)(c.s * g.bpc + b) * NB + Wr + wq] >> (ip & 63)) & 1ull;
        if (bit) atomicOr((unsigned long long*)&sRdp[b >> 6], 1ull << (b & 63));
    }
    const int nnz = uni(s_nnz);
    int idx = 0;
    for (int t = 0; t < nnz; ++t) {
        const int w = nz[t];
        uint64_t v = sM[w];
        while (v) {
            const int bit = ctz64(v);
            v &= v - 1;
            if ((idx++ % nwaves) != wave) continue;
            uint64_t* row = tb + (size_t)(g.NR + w * 64 + bit) * RS;
            int G = 0;
            for (int j = lane; j < Wc; j += 64) {
                const uint64_t xp = rowp[j], zp = rowp[Wc + j];
                if ((xp | zp) == 0) continue;
                const uint64_t xi = row[j], zi = row[Wc + j];
                G += gsum(xp, zp, xi, zi);
                row[j] = xi ^ xp;
                row[Wc + j] = zi ^ zp;
            }
            G = wave_sum_uniform(G, lane);
            if (lane == 0) {
                if (G & 1) atomicOr(c.err, 4);
                if (G & 2) atomicOr((unsigned long long*)&sC[w], 1ull << bit);
            }
        }
    }
    if (tid == 0) {
        atomicAdd(&c.lcnt[0], 1u);
        atomicAdd(&c.lcnt[1], (unsigned int)idx);
    }
    __syncthreads();
    // signs of the rowsum rows, pending targets' x columns, the pivot log
    const int rsp = uni(s_rsp);
    for (int t = tid; t < nnz; t += nt) {
        const int w = nz[t];
        c.rs[Wr + w] ^= (rsp ? sM[w] : 0ull) ^ sC[w];
    }
    for (int id = tid; id < nnz * g.bpc; id += nt) {
        const int b = id / nnz, t = id - b * nnz;
        if ((sRdp[b >> 6] >> (b & 63)) & 1ull) {
            const int w = nz[t];
            c.rd[(size_t)(c.s * g.bpc + b) * NB + Wr + w] ^= sM[w];
        }
    }
    for (int j = tid; j < Wc; j += nt) {
        uint64_t bits = rowp[j];
        while (bits) {
            const int bit = ctz64(bits);
            bits &= bits - 1;
            const int k2 = c.tm[j * 64 + bit];
            if (k2 < 0 || k2 == k) continue;
            plist_add(c, k, k2);
            uint64_t* X2 = X + k2;
            for (int t = 0; t < nnz; ++t) X2[(size_t)(Wr + nz[t]) * K] ^= sM[nz[t]];
            X2[(size_t)(Wr + wq) * K] &= ~bq;
        }
    }
    uint64_t* lrow = c.lrow + (size_t)k * RS;
    for (int j = tid; j < RS; j += nt) lrow[j] = rowp[j];
    for (int t = tid; t < nrdw; t += nt) c.lrd[(size_t)k * nrdw + t] = sRdp[t];
    if (tid == 0) {
        c.lrs[k] = rsp;
        c.lp[k] = ip;
        *c.ran = 1;
    }
    __syncthreads();
    // p <- Z_a with the outcome as its sign
    const int za = Wc + (a >> 6);
    for (int j = tid; j < RS; j += nt) gp[j] = (j == za) ? (1ull << (a & 63)) : 0ull;
    if (tid == 0) c.rs[Wr + wq] &= ~bq;
    for (int b = tid; b < g.bpc; b += nt) {
        const int gb = c.s * g.bpc + b;
        const int out = outcome_bit(c, k, gb);
        uint64_t* rdb = c.rd + (size_t)gb * NB;
        rdb[Wr + wq] = (rdb[Wr + wq] & ~bq) | (out ? bq : 0ull);
        c.obuf[(size_t)gb * K + k] = (uint8_t)out;
    }
    if (tid == 0) c.tm[a] = -1;
    __syncthreads();
}

// WPL = column words per lane of a row, ceil(Wc / 64) (= stabilizer bands per lane): the
// one-wave paths keep that many words of the pivot and of a batch of rows in registers, so
// narrow tableaux get a kernel without the registers the widest one needs, and room for twelve
// waves instead of eight (more of a round's targets run at once).
constexpr int chain_threads(int wpl) { return wpl == 1 ? 768 : 512; }
template <int WPL>
__global__ void __launch_bounds__(chain_threads(WPL))
k_chain(Geom g, uint64_t* __restrict__ tab, uint64_t* __restrict__ rs, uint64_t* __restrict__ rd,
        uint64_t* __restrict__ Xcol, uint64_t* __restrict__ Zcol, int K,
        int* __restrict__ cls, const int* __restrict__ tq, int* __restrict__ pend, uint64_t seed, uint64_t first_shot, uint64_t instr, int pos_base,
        int* __restrict__ plog_p, uint64_t* __restrict__ plog_row, int* __restrict__ plog_rs,
        uint64_t* __restrict__ plog_rd, int* __restrict__ ran, uint16_t* __restrict__ plist,
        int* __restrict__ pcnt, int* __restrict__ povf, uint8_t* __restrict__ obuf,
        int* __restrict__ err, unsigned long long* __restrict__ counters)
{
    extern __shared__ uint64_t sm[];
    const int s = blk_x(g);
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = uni(tid >> 6), nwaves = nt >> 6;
    const ChainLds L = chain_lds_layout(g);
    int* owner = (int*)((char*)sm + L.owner);
    // window entries live in fixed slots; wpos[] lists the slots in op order
    int* sk = (int*)((char*)sm + L.win);   // target id per slot
    int* stype = sk + kWin;                 // T_RANDOM, T_BIG_RANDOM, T_UNKNOWN, T_DEAD
    int* spiv = stype + kWin;
    int* scnt = spiv + kWin;
    int* wpos = scnt + kWin;                // window order -> slot
    int* wsel = wpos + kWin;                // per window position: selected this round
    int* wstale = wsel + kWin;              // per window position: must be analysed again
    int* selpos = wstale + kWin;            // positions selected this round
    int* alist = selpos + kWin;             // slots analysed this round
    int* srows = alist + kWin;              // kWin * kRCap
    uint64_t* wideP = (uint64_t*)((char*)sm + L.wide);   // kWide pivot rows
    uint64_t* wlm = (uint64_t*)((char*)sm + L.words);     // kWide x kRCap word masks
    int* wlw = (int*)(wlm + kWide * kRCap);               // and their word indices
    int* aff = (int*)((char*)sm + L.aff);                 // kAffCap x {code, flags, j}
    __shared__ int s_cnt[16], s_nwin, s_tail, s_bar, s_nsel, s_na, s_aff, s_rsp[kWide], s_wln[kWide];
    // bit i: row pair i is the pivot of a target executed this round (set and cleared in selection)
    unsigned int* pbit = (unsigned int*)((char*)sm + L.pbit);

    ChainCtx c;
    c.g = g;
    c.tb = tab + (size_t)s * 2 * g.NR * g.RS;
    c.rs = rs + (size_t)s * g.NB;
    c.rd = rd;
    c.X = Xcol + (size_t)s * g.NB * K;
    c.Z = Zcol + (size_t)s * g.NB * K;
    c.K = K;
    c.s = s;
    c.tq = tq;
    c.tm = (int16_t*)((char*)sm + L.tm);
    c.cl = cls + (size_t)s * K;
    c.nrdw = (g.bpc + 63) >> 6;
    c.lp = plog_p + (size_t)s * K;
    c.lrow = plog_row + (size_t)s * K * g.RS;
    c.lrs = plog_rs + (size_t)s * K;
    c.lrd = plog_rd + (size_t)s * K * c.nrdw;
    c.ran = ran;
    c.plist = plist + (size_t)s * K * kPListCap;
    c.pcnt = pcnt + (size_t)s * K;
    c.povf = povf + s;
    c.seed = seed;
    c.first_shot = first_shot;
    c.instr = instr;
    c.pos_base = pos_base;
    c.obuf = obuf;
    c.err = err;
    c.counters = counters;
    __shared__ unsigned int s_lcnt[2];
    c.lcnt = s_lcnt;
    if (tid == 0) {
        s_lcnt[0] = 0;
        s_lcnt[1] = 0;
    }
    int* pd = pend + (size_t)s * K;
    int* cl = cls + (size_t)s * K;

    // a layer with no random target at its start (most of them) ends here, after one pass of
    // independent loads (nothing runs, so nothing downstream reads the log)
    {
        bool any = false;
        for (int k0 = 0; k0 < K; k0 += 8 * nt) {
            int v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = k0 + u * nt + tid;
                v[u] = k < K ? cl[k] : -1;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) any |= v[u] >= 0;
        }
        if (!__syncthreads_or(any)) return;
    }
    // no target of this layer has run yet (the replay reads the log)
    for (int k = tid; k < K; k += nt) {
        c.lp[k] = -1;
        c.pcnt[k] = 0;
    }
    if (tid == 0) *c.povf = 0;
    // pending list: random-at-start targets in op order (stable compaction)
    int base = 0;
    for (int k0 = 0; k0 < K; k0 += nt) {
        const int k = k0 + tid;
        const bool f = k < K && cl[k] >= 0;
        const uint64_t m = __ballot(f);
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) s_cnt[wave] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < nwaves; ++w) {
            if (w < wave) before += s_cnt[w];
            total += s_cnt[w];
        }
        if (f) pd[base + before + rank] = k;
        base += total;
        __syncthreads();
    }
    const int npend = base;
    if (npend == 0) return;
    // column upkeep: the x columns of pending random targets
    for (int q = tid; q < g.n; q += nt) c.tm[q] = -1;
    __syncthreads();
    for (int k = tid; k < K; k += nt)
        if (cl[k] >= 0) c.tm[tq[k]] = (int16_t)k;
    // owner[i]: (round << 7) | (127 - t) of the first window position t that claimed row pair i
    // in that round; a claim from an earlier round counts as no claim, so nothing is reset
    for (int i = tid; i < g.NR; i += nt) owner[i] = 0;
    for (int i = tid; i < (g.NR + 31) / 32; i += nt) pbit[i] = 0u;
    const int w0 = min(kWin, npend);
    for (int t = tid; t < w0; t += nt) {
        sk[t] = pd[t];
        stype[t] = T_UNKNOWN;
        wpos[t] = t;
    }
    if (tid == 0) {
        s_nwin = w0;
        s_tail = w0;
    }
    __syncthreads();
    int rounds = 0;

    // a round can empty the window; the refill below brings in the next pending targets
    while (s_nwin > 0 || s_tail < npend) {
        ++rounds;
        const int nwin = uni(s_nwin);
        // ---- analysis: the first kAnalyze entries not yet analysed (new, or touched) ----
        if (wave == 0) {
            const bool un = lane < nwin && stype[wpos[lane]] == T_UNKNOWN;
            const uint64_t m = __ballot(un);
            const int rank = __popcll(m & ((1ull << lane) - 1ull));
            if (un && rank < kAnalyze) alist[rank] = wpos[lane];
            if (lane == 0) s_na = min(__popcll(m), kAnalyze);
        }
        __syncthreads();
        // the stabilizer half of an entry's column (band Wr + lane + 64 u), all words at once;
        // a wave's next entry is read while it works on the current one (lanes past Wr read
        // band Wr and are masked)
        const int na = uni(s_na);
        auto load_col = [&](int a_i, uint64_t* cw) {
            const int kk = a_i < na ? sk[alist[a_i]] : 0;
#pragma unroll
            for (int u = 0; u < WPL; ++u) {
                const int w = lane + 64 * u;
                cw[u] = c.X[(size_t)(g.Wr + (w < g.Wr ? w : 0)) * K + kk];
            }
        };
        uint64_t cwn[WPL];
        if (wave < na) load_col(wave, cwn);
        for (int a_i = wave; a_i < na; a_i += nwaves) {
            const int sl = alist[a_i];
            const int k = sk[sl];
            uint64_t cw[WPL];
#pragma unroll
            for (int u = 0; u < WPL; ++u) cw[u] = lane + 64 * u < g.Wr ? cwn[u] : 0ull;
            if (a_i + nwaves < na) load_col(a_i + nwaves, cwn);
            // pivot = first set bit in band order, the other set bits are the rowsum rows
            // (ascending); the few nonzero words are read out one by one with scalar loops
            int pv = INT_MAX, cnt = 0;
#pragma unroll
            for (int u = 0; u < WPL; ++u) {
                uint64_t lanes = __ballot(cw[u] != 0ull);
                while (lanes) {
                    const int l = ctz64(lanes);
                    lanes &= lanes - 1;
                    uint64_t v = readlane_u64(cw[u], l);
                    const int wb = l + 64 * u;                 // stabilizer band
                    if (pv == INT_MAX) {
                        pv = wb * 64 + ctz64(v);
                        v &= v - 1;
                    }
                    while (v && cnt < kRCap) {
                        const int bit = ctz64(v);
                        v &= v - 1;
                        if (lane == 0) srows[sl * kRCap + cnt] = (g.Wr + wb) * 64 + bit;
                        ++cnt;
                    }
                    cnt += __popcll(v);                        // beyond kRCap: counted only
                }
            }
            if (pv == INT_MAX) {
                // deterministic now: evaluated after the chain
                if (lane == 0) {
                    stype[sl] = T_DEAD;
                    cl[k] = -2;
                }
                continue;
            }
            if (lane == 0) {
                stype[sl] = cnt > kRCap ? T_BIG_RANDOM : T_RANDOM;
                spiv[sl] = pv;
                scnt[sl] = cnt;
            }
        }
        __syncthreads();
        // ---- drop entries that turned deterministic, refill from the pending list ----
        if (wave == 0) {
            const int sl = lane < nwin ? wpos[lane] : -1;
            const bool keep = sl >= 0 && stype[sl] != T_DEAD;
            const uint64_t m = __ballot(keep);
            const int nkeep = __popcll(m);
            const uint64_t usedmask = wave_or(keep ? (1ull << sl) : 0ull);
            const int tail = uni(s_tail);
            const int nnew = min(kWin - nkeep, npend - tail);
            const uint64_t freem = ~usedmask;
            const bool fr = (freem >> lane) & 1ull;                   // lane = a free slot
            const int r = __popcll(freem & ((1ull << lane) - 1ull));   // its rank among free slots
            const int kp = __popcll(m & ((1ull << lane) - 1ull));
            // every lane has read what it needs; now write the new order
            __builtin_amdgcn_wave_barrier();
            if (keep) wpos[kp] = sl;
            if (fr && r < nnew) {
                wpos[nkeep + r] = lane;
                sk[lane] = pd[tail + r];
                stype[lane] = T_UNKNOWN;
            }
            if (lane == 0) {
                s_nwin = nkeep + nnew;
                s_tail = tail + nnew;
            }
        }
        __syncthreads();
        const int nw = uni(s_nwin);
        if (nw == 0) break;
        // ---- selection, by wave 0 with one lane per window position t: only analysed
        // entries before the first unknown or big one are eligible; an eligible entry runs iff
        // it is the first owner of all its row pairs.  An entry that does not run must be analysed
        // again iff the pivot of one that runs is among its rows (a row that runs' rowsums touch
        // changes its x at this entry's qubit only by that pivot's, which is then 0); big
        // entries (incomplete row lists) whenever anything runs.
        if (wave == 0) {
            const int t = lane;
            const int sl = t < nw ? wpos[t] : 0;
            const int ty = t < nw ? stype[sl] : T_UNKNOWN;
            const uint64_t um = __ballot(ty == T_UNKNOWN || ty == T_BIG_RANDOM);
            const int bar = um ? min(ctz64(um), nw) : nw;
            const bool elig = t < bar;
            const int cnt = (t < nw && ty == T_RANDOM) ? scnt[sl] : -1;
            const int pv = cnt >= 0 ? spiv[sl] : 0;
            const int* rw = srows + sl * kRCap;
            const int mine = (rounds << 7) | (127 - t);
            if (elig)
                for (int r = 0; r <= cnt; ++r) atomicMax(&owner[r < cnt ? rw[r] - g.NR : pv], mine);
            __builtin_amdgcn_wave_barrier();
            bool ok = elig;
            if (elig)
                for (int r = 0; r <= cnt && ok; ++r)
                    if (owner[r < cnt ? rw[r] - g.NR : pv] != mine) ok = false;
            const uint64_t selm = __ballot(ok);
            if (t < nw) wsel[t] = ok ? 1 : 0;
            if (ok) atomicOr(&pbit[pv >> 5], 1u << (pv & 31));
            __builtin_amdgcn_wave_barrier();
            bool st = false;
            if (!ok && cnt >= 0)
                for (int r = 0; r <= cnt && !st; ++r) {
                    const int q = r < cnt ? rw[r] - g.NR : pv;
                    if ((pbit[q >> 5] >> (q & 31)) & 1u) st = true;
                }
            __builtin_amdgcn_wave_barrier();
            if (ok) atomicAnd(&pbit[pv >> 5], ~(1u << (pv & 31)));
            if (t < nw && (st || (ty == T_BIG_RANDOM && bar > 0))) stype[sl] = T_UNKNOWN;
            if (ok) selpos[__popcll(selm & ((1ull << lane) - 1ull))] = t;
            if (lane == 0) {
                s_bar = bar;
                s_nsel = __popcll(selm);
                s_aff = 0;
            }
        }
        __syncthreads();
        const int bar = uni(s_bar);
        const int nsel = uni(s_nsel);
        // ---- execution ----
        if (bar == 0 && stype[wpos[0]] == T_BIG_RANDOM) {
            block_solo(c, sk[wpos[0]], sm, tid, nt);
            if (tid == 0) {
                wsel[0] = 1;
                count_add(counters, 1, 1ull);
            }
            // a dense update may touch anything: analyse every remaining entry again
            for (int t = tid + 1; t < nw; t += nt) stype[wpos[t]] = T_UNKNOWN;
        } else if (nsel <= kWide) {
            // few targets: stage their pivot rows, spread their rowsums over all waves, and
            // hand their column upkeep to the whole block
            for (int id = tid; id < nsel * g.RS; id += nt) {
                const int j = id / g.RS, w = id - j * g.RS;
                const int ip = spiv[wpos[selpos[j]]];
                wideP[j * g.RS + w] = c.tb[(size_t)(g.NR + ip) * g.RS + w];
            }
            if (tid < nsel) {
                const int ip = spiv[wpos[selpos[tid]]];
                s_rsp[tid] = (int)((c.rs[g.Wr + (ip >> 6)] >> (ip & 63)) & 1ull);
            }
            // word lists of the rowsum rows: wave j writes target j's runs
            for (int j = wave; j < nsel; j += nwaves) {
                const int sl = wpos[selpos[j]];
                uint64_t hm[2], mv[2];
                int wv[2];
                row_runs(srows + sl * kRCap, scnt[sl], lane, hm, wv, mv);
                const int n0 = __popcll(hm[0]);
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    if ((hm[h] >> lane) & 1ull) {
                        const int pos = (h ? n0 : 0) + __popcll(hm[h] & ((1ull << lane) - 1ull));
                        wlw[j * kRCap + pos] = wv[h];
                        wlm[j * kRCap + pos] = mv[h];
                    }
                if (lane == 0) s_wln[j] = n0 + __popcll(hm[1]);
            }
            __syncthreads();
            for (int j = 0; j < nsel; ++j) {
                const int sl = wpos[selpos[j]];
                if (wave >= scnt[sl]) continue;
                uint64_t xp[WPL], zp[WPL];
                load_row_lane<WPL>(wideP + j * g.RS, g.Wc, lane, xp, zp);
                uint64_t pend[1] = {(uint64_t)s_rsp[j]};
                rowsum_rows<WPL>(c, xp, zp, pend, 0, srows + sl * kRCap, scnt[sl], wave, nwaves, lane);
            }
            for (int j = wave; j < nsel; j += nwaves) {
                const int sl = wpos[selpos[j]];
                uint64_t xp[WPL], zp[WPL];
                load_row_lane<WPL>(wideP + j * g.RS, g.Wc, lane, xp, zp);
                random_epilogue<WPL>(c, sk[sl], c.tq[sk[sl]], spiv[sl], s_rsp[j], xp, zp, srows + sl * kRCap, scnt[sl], lane,
                                aff, &s_aff, j);
            }
            __syncthreads();
            // column upkeep of the batch: (entry, word) pairs over the block; the extra slot
            // u == maxw clears the pivot's bit
            const int naff = min(s_aff, kAffCap);
            int maxw = 0;
            for (int j = 0; j < nsel; ++j) maxw = max(maxw, s_wln[j]);
            for (int id = tid; id < naff * (maxw + 1); id += nt) {
                const int e = id / (maxw + 1), u = id - e * (maxw + 1);
                const int k2 = aff[3 * e], j = aff[3 * e + 2];
                unsigned long long* X2 = (unsigned long long*)(c.X + k2);
                if (u < maxw) {
                    if (u >= s_wln[j]) continue;
                    atomicXor(&X2[(size_t)wlw[j * kRCap + u] * K], (unsigned long long)wlm[j * kRCap + u]);
                } else {
                    const int ip = spiv[wpos[selpos[j]]];
                    atomicAnd(&X2[(size_t)(g.Wr + (ip >> 6)) * K], ~(1ull << (ip & 63)));
                    plist_add(c, sk[wpos[selpos[j]]], k2);
                }
            }
        } else {
            for (int j = wave; j < nsel; j += nwaves) {
                const int sl = wpos[selpos[j]];
                wave_random<WPL>(c, sk[sl], spiv[sl], srows + sl * kRCap, scnt[sl], lane);
            }
        }
        __syncthreads();
        // ---- remove executed entries (their slots become free) ----
        if (wave == 0) {
            const bool keep = lane < nw && !wsel[lane];
            const int sl = lane < nw ? wpos[lane] : 0;
            const uint64_t m = __ballot(keep);
            const int rank = __popcll(m & ((1ull << lane) - 1ull));
            __builtin_amdgcn_wave_barrier();
            if (keep) wpos[rank] = sl;
            if (lane == 0) s_nwin = __popcll(m);
        }
        __syncthreads();
    }
    if (tid == 0) {
        count_add(counters, 0, (unsigned long long)rounds);
        count_add(counters, 4, (unsigned long long)s_lcnt[0]);
        count_add(counters, 5, (unsigned long long)s_lcnt[1]);
    }
}

// ------------------------------------------------------------------------------------------
// Destabilizer replay of a measurement layer: grid (Wr destabilizer bands, S copies), 512
// threads.  In op order, every target the chain ran did, to each destabilizer D with x at its
// qubit, rowsum(D, P) with its old pivot row P (sign r_D <- r_D ^ r_P ^ (i-power / 2), the
// per-shot parts XOR), and replaced its pivot's own destabilizer by P.  Only rows with x at
// some run target at layer start, or a pivot's partner, can be touched.
//
// Which targets hit D depends only on D's x bits at the run targets' qubits; applying P flips
// exactly the bits of the pending targets the chain listed for P (a target run earlier has no
// x in P: P commutes with its Z), and replacing D by P sets them to P's.  So the hits of all
// 64 rows of the band are found at once, bit-sliced: word V[j] holds the band's x bits at run
// target j, and one wave walks the run targets in order with the next 64 words in a ring of
// lanes (flips to words within the ring land in registers, flips beyond it are LDS atomics),
// leaving H[j] = the rows target j hits (in place of V[j]).  Runs of targets that hit nothing
// are skipped a ring at a time.  Then every wave takes rows: a row's events (its replacement,
// if it is a partner, and the hits after it) are read off H with ballots and applied to its
// x and z words with kReplayAhead pivot rows in flight, summing the i-powers per lane (every
// step's power is even, so the halves add); the signs of the events after the replacement
// XOR in any order and are taken in parallel over the lanes.  When a pivot's list overflowed
// or the lists do not fit in LDS, a wave instead tests its row's live bits 64 run targets at a
// time and applies each hit before testing again.
// ------------------------------------------------------------------------------------------
constexpr int kReplayEvents = 512;     // events a wave collects before applying them
// pivot rows in flight per wave while events are applied (a ring of register buffers)
template <int WPL> struct ReplayRing { static constexpr int depth = WPL <= 2 ? 16 : WPL == 3 ? 12 : 8; };
constexpr int kReplayInline = 3;       // list entries kept in a target's descriptor

// Dynamic LDS of the replay.  With lists (ent_cap >= 0): per-shot deltas, partner table, run
// targets, then per run target its x word V (H after the walk) and its descriptor, the
// target -> run index map, the per-wave event lists, then ent_cap entries of the long lists.
// Without: the first three only.
struct ReplayLds {
    int acc, prow, rk, V, desc, jmap, ev, ent;      // byte offsets
    int small_bytes;                                // end of the form without lists
    int fixed_bytes;                                // end of the form with lists, before entries
};

__host__ __device__ inline ReplayLds replay_lds_layout(int K, int nrdw, int nwaves)
{
    ReplayLds L;
    int o = 0;
    L.acc = o; o += nwaves * nrdw * 8;
    L.prow = o; o += 64 * 4;
    L.rk = o; o += ((K * 4 + 7) / 8) * 8;
    L.small_bytes = o;
    L.V = o; o += K * 8;
    L.desc = o; o += K * 8;
    L.jmap = o; o += ((K * 2 + 7) / 8) * 8;
    L.ev = o; o += nwaves * kReplayEvents * 4;
    L.ent = o;
    L.fixed_bytes = o;
    return L;
}

// Whether the run-index map (16-bit) covers every target.
__host__ __device__ inline bool replay_walk_fits(int K) { return K <= 32767; }

// Row words of this lane (word lane + 64 t, WPL slots).  No load is conditional, so that the
// loads of rows in flight are waited for one by one: the last slot's lanes past Wc load word 0
// instead (any address of the row does) and the caller masks them with the tail mask.
template <int WPL>
__device__ __forceinline__ void replay_load(const uint64_t* row, int Wc, int lane, uint64_t* x, uint64_t* z)
{
#pragma unroll
    for (int t = 0; t < WPL; ++t) {
        const int cw = (t < WPL - 1 || lane + 64 * t < Wc) ? lane + 64 * t : 0;
        x[t] = row[cw];
        z[t] = row[Wc + cw];
    }
}

// Descriptor of run target j: bits 0..47 up to kReplayInline later run indices of its list
// (16 bits each) or, for a longer list, its offset in the entry area (bits 0..31); bits 48..52
// the list length; bits 53..59 its partner row in the band + 1 (0: the partner is elsewhere).
__device__ __forceinline__ int desc_len(uint64_t d) { return (int)((d >> 48) & 31); }
__device__ __forceinline__ int desc_partner(uint64_t d) { return (int)((d >> 53) & 127) - 1; }

template <int WPL>
__global__ void __launch_bounds__(512)
k_replay(Geom g, uint64_t* __restrict__ tab, uint64_t* __restrict__ rs, uint64_t* __restrict__ rd,
         const uint64_t* __restrict__ Xcol, int K, const int* __restrict__ tq,
         const int* __restrict__ plog_p, const uint64_t* __restrict__ plog_row,
         const int* __restrict__ plog_rs, const uint64_t* __restrict__ plog_rd,
         const uint16_t* __restrict__ plist, const int* __restrict__ pcnt, const int* __restrict__ povf,
         const int* __restrict__ ran, int ent_cap, int* __restrict__ err, unsigned long long* __restrict__ counters)
{
    if (*ran == 0) return;                             // no random target ran in this layer
    extern __shared__ uint64_t rsm[];
    const int band = blk_x(g), s = blk_y(g);
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
    const int Wc = g.Wc, RS = g.RS, NB = g.NB;
    const int nrdw = (g.bpc + 63) >> 6;
    const uint64_t tail = lane + 64 * (WPL - 1) < Wc ? ~0ull : 0ull;   // last slot in the row
    const ReplayLds LL = replay_lds_layout(K, nrdw, nwaves);
    char* base = (char*)rsm;
    const bool lists = ent_cap >= 0;                     // LDS holds the list form
    uint64_t* acc = (uint64_t*)(base + LL.acc);          // nwaves x nrdw per-shot sign deltas
    int* prow = (int*)(base + LL.prow);                  // per row of the band: see below
    int* rk = (int*)(base + LL.rk);
    uint64_t* V = lists ? (uint64_t*)(base + LL.V) : nullptr;
    uint64_t* desc = lists ? (uint64_t*)(base + LL.desc) : nullptr;
    int16_t* jmap = lists ? (int16_t*)(base + LL.jmap) : nullptr;
    int* evs = lists ? (int*)(base + LL.ev) : nullptr;
    uint16_t* ent = lists ? (uint16_t*)(base + LL.ent) : nullptr;
    __shared__ int s_cnt[16], s_crow[64], s_ncand, s_next;
    __shared__ unsigned long long s_cand;
    __shared__ unsigned int s_rc[4];   // work counters, flushed once per block
    const int* lp = plog_p + (size_t)s * K;
    const uint16_t* pl = plist + (size_t)s * K * kPListCap;
    const int* pc = pcnt + (size_t)s * K;
    const uint64_t* X = Xcol + (size_t)s * NB * K + (size_t)band * K;
    uint64_t* tb = tab + (size_t)s * 2 * g.NR * RS;
    uint64_t* rsc = rs + (size_t)s * NB;

    // run targets in op order (stable compaction)
    if (tid == 0) {
        s_cand = 0;
        s_next = 0;
        s_rc[0] = s_rc[1] = s_rc[2] = s_rc[3] = 0;
    }
    for (int r = tid; r < 64; r += nt) prow[r] = -1;
    __syncthreads();
    int R = 0;
    for (int k0 = 0; k0 < K; k0 += nt) {
        const int k = k0 + tid;
        const bool f = k < K && lp[k] >= 0;
        const uint64_t m = __ballot(f);
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) s_cnt[wave] = __popcll(m);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < nwaves; ++w) {
            if (w < wave) before += s_cnt[w];
            total += s_cnt[w];
        }
        if (f) rk[R + before + rank] = k;
        R += total;
        __syncthreads();
    }
    if (R == 0) return;
    // the list form holds for this copy when no pending list overflowed and the long lists fit
    bool walk = lists && povf[s] == 0;
    uint64_t cand = 0;
    if (walk) {
        for (int k = tid; k < K; k += nt) jmap[k] = -1;
        __syncthreads();
        for (int j = tid; j < R; j += nt) jmap[rk[j]] = (int16_t)j;
        __syncthreads();
        // descriptors (list entries as run indices; entries that did not run are dropped),
        // x words, partners; long lists go to ent at offsets from an exclusive scan
        int T = 0;
        for (int j0 = 0; j0 < R; j0 += nt) {
            const int j = j0 + tid;
            int len = 0, n2 = 0, pr = -1;
            const uint16_t* lst = nullptr;
            if (j < R) {
                const int k = rk[j];
                lst = pl + (size_t)k * kPListCap;
                n2 = min(pc[k], kPListCap);
                for (int e = 0; e < n2; ++e) len += jmap[lst[e]] >= 0 ? 1 : 0;
                const uint64_t xw = X[k];
                V[j] = xw;
                cand |= xw;
                const int p = lp[k];
                if ((p >> 6) == band) {
                    pr = p & 63;
                    prow[pr] = j;
                    cand |= 1ull << pr;
                }
            }
            const int big = len > kReplayInline ? len : 0;
            const int ex = wave_excl_scan(big, lane);
            if (lane == 0) s_cnt[wave] = wave_sum(big);
            __syncthreads();
            int before = 0, total = 0;
            for (int w = 0; w < nwaves; ++w) {
                if (w < wave) before += s_cnt[w];
                total += s_cnt[w];
            }
            if (j < R) {
                uint64_t d = ((uint64_t)len << 48) | ((uint64_t)(pr + 1) << 53);
                const int o = T + before + ex;
                if (big) d |= (uint32_t)o;
                for (int e = 0, n = 0; e < n2; ++e) {
                    const int jj = jmap[lst[e]];
                    if (jj < 0) continue;
                    if (!big) d |= (uint64_t)jj << (16 * n);
                    else if (o + n < ent_cap) ent[o + n] = (uint16_t)jj;
                    ++n;
                }
                desc[j] = d;
            }
            T += total;
            __syncthreads();
        }
        walk = T <= ent_cap;
    } else {
        for (int j = tid; j < R; j += nt) {
            const int k = rk[j];
            cand |= X[k];
            const int p = lp[k];
            if ((p >> 6) == band) {
                cand |= 1ull << (p & 63);
                prow[p & 63] = k;
            }
        }
    }
    cand = wave_or(cand);
    if (lane == 0 && cand) atomicOr(&s_cand, (unsigned long long)cand);
    __syncthreads();

    if (walk) {
        // bit-sliced walk, 64 run targets at a time: lane l holds target j0 + l (its word and
        // descriptor); flips to targets of the same 64 land in registers, later ones are LDS
        // atomics made before those targets are read.  A row's bits only ever change by its
        // own hits and replacement, so each wave walks its own slice of the 64 rows (bits gm of
        // every word) on its own: its updates touch no other wave's bits.
        const int rpw = 64 / nwaves;
        const uint64_t gm = (rpw == 64 ? ~0ull : ((1ull << rpw) - 1ull)) << (rpw * wave);
        for (int j0 = 0; j0 < R; j0 += 64) {
            const int jl = j0 + lane;
            const uint64_t raw = jl < R ? V[jl] & gm : 0ull;
            uint64_t val = raw;
            const uint64_t dsc = jl < R ? desc[jl] : 0ull;
            const int pl_ = desc_partner(dsc);
            const uint64_t pm = __ballot(jl < R && pl_ >= 0 && ((gm >> pl_) & 1ull));
            int off = 0;
            while (true) {
                // next target from off on that hits a row or has its partner here
                const uint64_t am = (__ballot(val != 0ull) | pm) & (off < 64 ? ~0ull << off : 0ull);
                if (!am) break;
                const int cj = ctz64(am);
                const uint64_t cur = readlane_u64(val, cj);
                const uint64_t d = readlane_u64(dsc, cj);
                const int len = desc_len(d), prd = desc_partner(d);
                const int pr = (prd >= 0 && ((gm >> prd) & 1ull)) ? prd : -1;
                const uint64_t bpr = pr >= 0 ? 1ull << pr : 0ull;
                const uint64_t hit = cur & ~bpr;
                if (lane == cj) val = hit;                  // H[j]
                if (pr >= 0) {
                    // the partner's bits at later targets become P's: cleared here, set below
                    if (lane > cj) val &= ~bpr;
                    for (int w = j0 + 64 + lane; w < R; w += 64) atomicAnd((unsigned long long*)&V[w], ~bpr);
                }
                for (int e = 0; e < len; ++e) {
                    const int j2 = len <= kReplayInline ? (int)((d >> (16 * e)) & 0xffff) : (int)ent[(uint32_t)d + e];
                    if (j2 < j0 + 64) {
                        if (lane == j2 - j0) val = (val ^ hit) | bpr;
                    } else if (lane == 0) {
                        if (hit) atomicXor((unsigned long long*)&V[j2], hit);
                        if (bpr) atomicOr((unsigned long long*)&V[j2], bpr);
                    }
                }
                off = cj + 1;
            }
            // H of the 64 in this wave's bits (0 where nothing hit)
            if (jl < R && (raw ^ val)) atomicXor((unsigned long long*)&V[jl], raw ^ val);
        }
    }
    if (tid == 0) {
        uint64_t c = s_cand;
        int nc = 0;
        while (c) {
            s_crow[nc++] = ctz64(c);
            c &= c - 1;
        }
        s_ncand = nc;
    }
    __syncthreads();
    const int ncand = s_ncand;

    uint64_t* myacc = acc + (size_t)wave * nrdw;
    int* ev = lists ? evs + (size_t)wave * kReplayEvents : nullptr;
    int nrows = 0, applied = 0, trows = 0, tev = 0;
    while (true) {
        int jr = 0;
        if (lane == 0) jr = atomicAdd(&s_next, 1);
        jr = __shfl(jr, 0, 64);
        if (jr >= ncand) break;
        ++nrows;
        const int r = s_crow[jr];
        const int i = band * 64 + r;                   // destabilizer index
        uint64_t* row = tb + (size_t)i * RS;
        uint64_t x[WPL], z[WPL];
        replay_load<WPL>(row, Wc, lane, x, z);
        x[WPL - 1] &= tail;
        z[WPL - 1] &= tail;
        int sh = (int)((rsc[band] >> r) & 1ull);
        const int sh0 = sh;
        for (int u = lane; u < nrdw; u += 64) myacc[u] = 0;
        bool mod = false;
        // Phase of the rowsums since the last replacement, telescoped: with |u| the number of
        // qubits where a row has both x and z, rowsum(D, P) raises i to |P| + |D| + 2 z_P.x_D
        // - |P D| (mod 4), so the steps from D0 to Dn sum to sum|P| + |D0| - |Dn| + 2 sum z_P.x_D,
        // and only the parity of the last sum matters: its terms XOR into cr.  G holds
        // sum|P| + |D0| per lane.
        int G = 0;
        uint64_t cr[WPL];
#pragma unroll
        for (int t = 0; t < WPL; ++t) {
            G += __popcll(x[t] & z[t]);
            cr[t] = 0;
        }
        auto phase = [&]() {
            int v = G;
#pragma unroll
            for (int t = 0; t < WPL; ++t) v += 2 * __popcll(cr[t]) - __popcll(x[t] & z[t]);
            return wave_sum(v);
        };
        // D := P_k, signs included (the per-shot deltas make rd's bits equal P's)
        auto replace_signs = [&](int kk) {
            const uint64_t* Pd = plog_rd + ((size_t)s * K + kk) * nrdw;
            sh = plog_rs[(size_t)s * K + kk];
            for (int b0 = 0; b0 < g.bpc; b0 += 64) {
                const int b = b0 + lane;
                const bool cb = b < g.bpc && ((rd[(size_t)(s * g.bpc + b) * NB + band] >> r) & 1ull);
                const uint64_t m = __ballot(cb);
                if (lane == 0) myacc[b0 >> 6] = m ^ Pd[b0 >> 6];
            }
        };
        // x and z words of one event: replace (G so far applies to the row being replaced) or
        // multiply in (the pivot row's last slot is masked here, at use)
        auto step = [&](bool repl, const uint64_t* px, const uint64_t* pz) {
            if (repl) {
                const int Gs = phase();
                if (lane == 0 && (Gs & 1)) atomicOr(err, 8);
                G = 0;
#pragma unroll
                for (int t = 0; t < WPL; ++t) {
                    const uint64_t m = t == WPL - 1 ? tail : ~0ull;
                    x[t] = px[t] & m;
                    z[t] = pz[t] & m;
                    G += __popcll(x[t] & z[t]);
                    cr[t] = 0;
                }
            } else {
#pragma unroll
                for (int t = 0; t < WPL; ++t) {
                    const uint64_t m = t == WPL - 1 ? tail : ~0ull;
                    const uint64_t a = px[t] & m, b = pz[t] & m;
                    cr[t] ^= b & x[t];
                    G += __popcll(a & b);
                    x[t] ^= a;
                    z[t] ^= b;
                }
                ++applied;
            }
        };
        if (walk) {
            // events: the replacement (if this row is a partner), then the hits after it
            const int jp = prow[r];
            int jn = jp >= 0 ? jp : 0;                 // next run index to read off H
            bool first = jp >= 0;
            const uint64_t* prow0 = plog_row + (size_t)s * K * RS;
            while (true) {
                int nev = 0;
                if (first) {
                    if (lane == 0) ev[0] = rk[jp] | (1 << 30);
                    nev = 1;
                    jn = jp + 1;
                    first = false;
                }
                while (jn < R && nev + 64 <= kReplayEvents) {
                    const int jj = jn + lane;
                    const bool h = jj < R && ((V[jj] >> r) & 1ull);
                    const uint64_t hm = __ballot(h);
                    if (h) ev[nev + __popcll(hm & ((1ull << lane) - 1ull))] = rk[jj];
                    nev += __popcll(hm);
                    jn += 64;
                }
                if (nev == 0) break;
                mod = true;
                // apply in order, the next kReplayAhead pivot rows in flight (a ring of register
                // buffers rotated by the unrolled loop; loads past the end repeat the last row)
                constexpr int kReplayAhead = ReplayRing<WPL>::depth;
                uint64_t px[kReplayAhead][WPL], pz[kReplayAhead][WPL];
#pragma unroll
                for (int u = 0; u < kReplayAhead; ++u)
                    replay_load<WPL>(prow0 + (size_t)(ev[min(u, nev - 1)] & 0x3fffffff) * RS, Wc, lane, px[u], pz[u]);
                int lastrep = -1;
                for (int e0 = 0; e0 < nev; e0 += kReplayAhead) {
#pragma unroll
                    for (int u = 0; u < kReplayAhead; ++u) {
                        const int e = e0 + u;
                        if (e < nev) {
                            const bool rp = (ev[e] >> 30) & 1;
                            if (rp) lastrep = e;
                            step(rp, px[u], pz[u]);
                        }
                        const int en = min(e + kReplayAhead, nev - 1);
                        replay_load<WPL>(prow0 + (size_t)(ev[en] & 0x3fffffff) * RS, Wc, lane, px[u], pz[u]);
                    }
                }
                // signs: from the last replacement on (XOR over events, in any order)
                if (lastrep >= 0) replace_signs(ev[lastrep] & 0x3fffffff);
                int par = 0;
                for (int e = lastrep + 1 + lane; e < nev; e += 64)
                    par ^= plog_rs[(size_t)s * K + (ev[e] & 0x3fffffff)];
                sh ^= __popcll(__ballot(par & 1)) & 1;
                for (int u = 0; u < nrdw; ++u) {
                    uint64_t a = 0;
                    for (int e = lastrep + 1 + lane; e < nev; e += 64)
                        a ^= plog_rd[((size_t)s * K + (ev[e] & 0x3fffffff)) * nrdw + u];
                    a = wave_xor(a);
                    if (lane == 0) myacc[u] ^= a;
                }
                if (jn >= R) break;
            }
        } else {
            // walk by testing D's live x bits 64 run targets at a time
            ++trows;
            for (int j0 = 0; j0 < R; j0 += 64) {
                const int jj = j0 + lane;
                int k = 0, a = 0, p = -1;
                if (jj < R) {
                    k = rk[jj];
                    a = tq[k];
                    p = lp[k];
                }
                int from = 0;
                while (true) {
                    const int wa = a >> 6, src = wa & 63, slot = wa >> 6;
                    uint64_t vv = 0;
#pragma unroll
                    for (int t = 0; t < WPL; ++t) {
                        const uint64_t o = shfl_u64(x[t], src);
                        if (slot == t) vv = o;
                    }
                    const bool hit = jj < R && lane >= from && ((((vv >> (a & 63)) & 1ull) != 0) || p == i);
                    const uint64_t hm = __ballot(hit);
                    if (!hm) break;
                    const int l = ctz64(hm);
                    const int kk = __shfl(k, l, 64), pkk = __shfl(p, l, 64);
                    uint64_t px[WPL], pz[WPL];
                    replay_load<WPL>(plog_row + ((size_t)s * K + kk) * RS, Wc, lane, px, pz);
                    const bool repl = pkk == i;
                    step(repl, px, pz);
                    if (repl) {
                        replace_signs(kk);
                    } else {
                        sh ^= plog_rs[(size_t)s * K + kk];
                        const uint64_t* Pd = plog_rd + ((size_t)s * K + kk) * nrdw;
                        for (int u = lane; u < nrdw; u += 64) myacc[u] ^= Pd[u];
                    }
                    mod = true;
                    ++tev;
                    from = l + 1;
                }
            }
        }
        if (mod) {
            const int Gs = phase();
            if (lane == 0 && (Gs & 1)) atomicOr(err, 8);
            sh ^= (Gs >> 1) & 1;
#pragma unroll
            for (int t = 0; t < WPL; ++t) {
                const int cw = lane + 64 * t;
                if (cw < Wc) {
                    row[cw] = x[t];
                    row[Wc + cw] = z[t];
                }
            }
            if (lane == 0 && sh != sh0) atomicXor((unsigned long long*)&rsc[band], 1ull << r);
            for (int b = lane; b < g.bpc; b += 64)
                if ((myacc[b >> 6] >> (b & 63)) & 1ull)
                    atomicXor((unsigned long long*)&rd[(size_t)(s * g.bpc + b) * NB + band], 1ull << r);
        }
    }
    if (lane == 0 && nrows) {
        atomicAdd(&s_rc[0], (unsigned int)applied);
        atomicAdd(&s_rc[1], (unsigned int)nrows);
        atomicAdd(&s_rc[2], (unsigned int)trows);
        atomicAdd(&s_rc[3], (unsigned int)tev);
    }
    __syncthreads();
    if (tid == 0 && s_rc[1]) {
        if (s_rc[0]) count_add(counters, 8, (unsigned long long)s_rc[0]);
        count_add(counters, 9, (unsigned long long)s_rc[1]);
        if (s_rc[2]) count_add(counters, 10, (unsigned long long)s_rc[2]);
        if (s_rc[3]) count_add(counters, 11, (unsigned long long)s_rc[3]);
    }
}

// ------------------------------------------------------------------------------------------
// End of a measurement layer: resets (X on the qubit when the outcome is 1: every row with z
// at the qubit flips sign -- applied once for the whole layer, which is exact because sign
// flips commute with rowsum and with the other measurements of the layer) and the record.
// Block per (sign word w, group of up to kResetShots shots, chunk of kResetChunk targets), a
// wave per shot and its lanes over the chunk's targets.  The waves of a block read the same
// column words at about the same time, so a band's column comes from L2 once per block (the
// other waves hit in L1), not once per shot; the chunks keep enough blocks in flight.
// ------------------------------------------------------------------------------------------
constexpr int kResetShots = 16;
constexpr int kResetChunk = 1024;

__global__ void __launch_bounds__(64 * kResetShots)
k_reset_record(Geom g, uint64_t* __restrict__ rd, const uint64_t* __restrict__ Zcol,
               const uint8_t* __restrict__ obuf, int K, int do_reset, uint8_t* __restrict__ record,
               long long rec_stride, long long rec_off, int do_record)
{
    const int w = blk_x(g);
    const int lane = threadIdx.x & 63;
    const int b = blk_y(g) * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
    if (b >= g.B) return;                       // (no block barrier below)
    const int s = b / g.bpc;
    const int kc = (g.rev ? (int)gridDim.z - 1 - (int)blockIdx.z : (int)blockIdx.z) * kResetChunk;
    const int ke = min(K, kc + kResetChunk);
    const uint8_t* ob = obuf + (size_t)b * K;
    const uint64_t* Zc = Zcol + ((size_t)s * g.NB + w) * K;
    uint64_t acc = 0;
    // four targets per lane at a time, every load unconditional so they are all in flight
    for (int k0 = kc + lane; k0 < ke; k0 += 4 * 64) {
        uint8_t o[4];
        uint64_t z[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * 64;
            o[u] = k < ke ? ob[k] : (uint8_t)0;
            z[u] = (do_reset && k < ke) ? Zc[k] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u * 64;
            if (o[u]) acc ^= z[u];
            if (do_record && w == 0 && k < ke) record[(size_t)b * rec_stride + rec_off + k] = o[u];
        }
    }
    if (do_reset) {
        acc = wave_xor(acc);
        if (lane == 0 && acc) atomicXor((unsigned long long*)&rd[(size_t)b * g.NB + w], (unsigned long long)acc);
    }
}

// Pack the byte-per-measurement record into bits, LSB first, ceil(M/8) bytes per shot.
__global__ void k_pack(const uint8_t* __restrict__ rec, long long M, int B, uint8_t* __restrict__ out)
{
    const long long nbytes = (M + 7) / 8;
    const long long total = nbytes * B;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
         idx += (long long)gridDim.x * blockDim.x) {
        const long long b = idx / nbytes, j = idx - b * nbytes;
        uint8_t v = 0;
        for (int t = 0; t < 8; ++t) {
            const long long m = j * 8 + t;
            if (m < M && rec[b * M + m]) v |= (uint8_t)(1u << t);
        }
        out[idx] = v;
    }
}

}  // namespace stabdev
