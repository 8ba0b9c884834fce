// stab_commute.hip -- pairwise commutation of bit-packed Pauli strings (Sec. 3.2: the
// grouping check).  Two strings commute group-wise iff the parity of
// sum_q (x1_q z2_q + z1_q x2_q) is even, and qubit-wise iff every single-qubit term of that
// sum is 0.  Strings are stored like tableau rows: ceil(n/64) x-words, then as many z-words.
//
// Layout of the work: a block owns 64 strings B_j (one per lane: lane = j within the tile) and
// 64 strings A_i (16 per wave).  A tile of A words is staged in LDS and read as broadcasts;
// each lane keeps a chunk of its B_j words in registers; per (i, j) the two accumulators are a
// 64-bit XOR (group-wise) and a 64-bit OR (qubit-wise), reduced to one bit at the end and
// packed 64 columns per word with a ballot.  The work is VALU-bound (10 int32 operations per
// string pair and 64-bit word); nothing is a dense contraction MFMA could take.
//
// Included by stab_api.hip (same translation unit).

namespace stabdev {

constexpr int kCommThreads = 256;
constexpr int kCommRowsPerWave = 16;
constexpr int kCommRows = kCommRowsPerWave * (kCommThreads / 64);   // A strings per block
constexpr int kCommChunk = 4;                                        // x (and z) words per pass

__global__ void __launch_bounds__(kCommThreads)
k_commute(const uint64_t* __restrict__ A, int na, const uint64_t* __restrict__ B, int nb, int W,
          uint64_t* __restrict__ gc, uint64_t* __restrict__ qwc)
{
    __shared__ uint64_t sa[kCommRows][2 * kCommChunk + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = blockIdx.x * 64 + lane;
    const int i0 = blockIdx.y * kCommRows;
    const int nbw = (nb + 63) >> 6;
    const int RS = 2 * W;
    uint64_t accg[kCommRowsPerWave], accq[kCommRowsPerWave];
#pragma unroll
    for (int r = 0; r < kCommRowsPerWave; ++r) accg[r] = accq[r] = 0;

    for (int w0 = 0; w0 < W; w0 += kCommChunk) {
        const int nw = min(kCommChunk, W - w0);
        // B_j chunk in registers
        uint64_t xb[kCommChunk], zb[kCommChunk];
#pragma unroll
        for (int t = 0; t < kCommChunk; ++t) {
            const bool in = j < nb && t < nw;
            xb[t] = in ? B[(size_t)j * RS + w0 + t] : 0ull;
            zb[t] = in ? B[(size_t)j * RS + W + w0 + t] : 0ull;
        }
        // A tile chunk in LDS: row r, x words at [t], z words at [kCommChunk + t]
        for (int e = tid; e < kCommRows * 2 * kCommChunk; e += kCommThreads) {
            const int r = e / (2 * kCommChunk), c = e - r * (2 * kCommChunk);
            const int t = c < kCommChunk ? c : c - kCommChunk;
            const int i = i0 + r;
            uint64_t v = 0;
            if (i < na && t < nw) v = A[(size_t)i * RS + (c < kCommChunk ? 0 : W) + w0 + t];
            sa[r][c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kCommRowsPerWave; ++r) {
            const uint64_t* ar = sa[wave * kCommRowsPerWave + r];
            uint64_t g = 0, q = 0;
#pragma unroll
            for (int t = 0; t < kCommChunk; ++t) {
                const uint64_t m = (ar[t] & zb[t]) ^ (ar[kCommChunk + t] & xb[t]);
                g ^= m;
                q |= m;
            }
            accg[r] ^= g;
            accq[r] |= q;
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < kCommRowsPerWave; ++r) {
        const int i = i0 + wave * kCommRowsPerWave + r;
        const uint64_t bg = __ballot(j < nb && (__popcll(accg[r]) & 1));
        const uint64_t bq = __ballot(j < nb && accq[r] != 0);
        if (lane == 0 && i < na) {
            if (gc) gc[(size_t)i * nbw + blockIdx.x] = bg;
            if (qwc) qwc[(size_t)i * nbw + blockIdx.x] = bq;
        }
    }
}

}  // namespace stabdev
