/*
 * chp_oracle.c -- plain CPU reference of the STABSim tableau method (TEST INFRASTRUCTURE ONLY).
 *
 * This file is the oracle that the HIP library is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the product path never does.
 * It shares no code, header, table or constant with the HIP library.
 *
 * It is written to be obviously correct, not fast:
 *   - the tableau is row-major: row i holds x_i[0..n-1] and z_i[0..n-1] as packed bits plus
 *     a sign byte r_i.  Rows 0..n-1 are the destabilizers, rows n..2n-1 the stabilizers and
 *     row 2n the scratch row (CHP formalism, Sec. 2.3 of the paper);
 *   - gates loop over every row and apply the per-row bit rule of Table 1, with the
 *     Aaronson-Gottesman phase rules where the table is incomplete (see below);
 *   - a measurement follows Sec. 2.4: pivot = the first stabilizer row with x at the
 *     measured qubit; random case = rowsum into every other anticommuting row, move the
 *     pivot row to its destabilizer, replace it by Z_a with a random sign; deterministic case
 *     = clear the scratch row and rowsum(scratch, n+i) for each destabilizer i that has x at
 *     the qubit, in increasing i, the outcome being the scratch sign;
 *   - rowsum and its helper g are the rowsum algorithm of Appendix A.2, term by term.
 *
 * Readings of the paper taken here (each pinned by a test against 2x2/4x4 matrix algebra):
 *   - Phase gate: the sign update uses x*z from BEFORE the z update (Table 1 lists the z
 *     update first; read literally that gives the wrong sign for Y).
 *   - CNOT: r ^= x_c z_t (x_t ^ z_c ^ 1), the Aaronson-Gottesman rule; Table 1 prints only
 *     x_c z_t, which is wrong for e.g. Y_c Z_t.
 *   - X, Y, Z gates ("derived" Cliffords, Sec. 2.4): sign flips r ^= z, r ^= x^z, r ^= x.
 *   - Initial state |0...0>: destabilizer i = +X_i, stabilizer i = +Z_i.
 *   - Reset (MR, R): measure, then apply X when the outcome is 1.
 *   - T1T2 (exact relaxation + dephasing, Sec. 4.2): per target, reset with probability t0
 *     (its measurement outcome, if random, is u1 >> 63), else Z with probability t1 - t0.
 *   - rowsum with an odd phase sum leaves r_h unchanged (it only happens for the destabilizer
 *     of the pivot, which is overwritten right after).
 *
 * Randomness: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3", SC'11), key = (seed, shot), counter = (instruction index, target index, 0, 0).
 * The op-stream format and the noise/outcome draws are described in circuits.py.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* instruction kinds of the op-stream format */
enum { K_TICK = 0, K_H, K_S, K_X, K_Y, K_Z, K_CX, K_M, K_MR, K_R, K_DEP1, K_DEP2, K_PAULI1,
       K_T1T2, K_COUNT };

typedef struct {
    uint32_t kind;
    uint32_t ntargets;
    uint64_t t0, t1, t2;
} oinstr;

/* ------------------------------------------------------------------------------------------ */
/* Philox4x64-10 (SC'11, Sec. 4 / Random123): 10 rounds of two 64x64->128 multiplies with     */
/* the published multipliers, and a Weyl sequence on the key between rounds.                  */
/* ------------------------------------------------------------------------------------------ */
static void mul128(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void oracle_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        if (round > 0) { k0 += W0; k1 += W1; }
        mul128(M0, c0, &hi0, &lo0);
        mul128(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint64_t shot, uint64_t instr, uint64_t pos, uint64_t u[4])
{
    uint64_t ctr[4] = {instr, pos, 0, 0};
    uint64_t key[2] = {seed, shot};
    oracle_philox4x64_10(ctr, key, u);
}

static uint64_t mulhi64(uint64_t a, uint64_t b)
{
    uint64_t hi, lo;
    mul128(a, b, &hi, &lo);
    return hi;
}

/* ------------------------------------------------------------------------------------------ */
/* Tableau                                                                                    */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int n;
    int words;        /* 64-bit words per row per component */
    uint64_t *x;      /* (2n+1) * words */
    uint64_t *z;
    uint8_t *r;       /* 2n+1 */
} otab;

static int getx(const otab *t, int row, int col) { return (int)((t->x[(size_t)row * t->words + col / 64] >> (col % 64)) & 1u); }
static int getz(const otab *t, int row, int col) { return (int)((t->z[(size_t)row * t->words + col / 64] >> (col % 64)) & 1u); }

static void setx(otab *t, int row, int col, int v)
{
    uint64_t *w = &t->x[(size_t)row * t->words + col / 64];
    uint64_t m = 1ULL << (col % 64);
    *w = v ? (*w | m) : (*w & ~m);
}

static void setz(otab *t, int row, int col, int v)
{
    uint64_t *w = &t->z[(size_t)row * t->words + col / 64];
    uint64_t m = 1ULL << (col % 64);
    *w = v ? (*w | m) : (*w & ~m);
}

otab *oracle_tab_new(int n)
{
    if (n <= 0) return NULL;
    otab *t = (otab *)calloc(1, sizeof(otab));
    if (!t) return NULL;
    t->n = n;
    t->words = (n + 63) / 64;
    size_t rows = (size_t)2 * n + 1;
    t->x = (uint64_t *)calloc(rows * t->words, sizeof(uint64_t));
    t->z = (uint64_t *)calloc(rows * t->words, sizeof(uint64_t));
    t->r = (uint8_t *)calloc(rows, 1);
    if (!t->x || !t->z || !t->r) {
        free(t->x); free(t->z); free(t->r); free(t);
        return NULL;
    }
    /* |0...0>: destabilizer i = X_i, stabilizer i = Z_i, all signs + */
    for (int i = 0; i < n; ++i) {
        setx(t, i, i, 1);
        setz(t, n + i, i, 1);
    }
    return t;
}

void oracle_tab_free(otab *t)
{
    if (!t) return;
    free(t->x); free(t->z); free(t->r); free(t);
}

/* g of the rowsum algorithm (Appendix A.2): the power of i picked up when the Pauli with bits
 * (x1, z1) multiplies the one with bits (x2, z2). */
int oracle_g(int x1, int z1, int x2, int z2)
{
    if (x1 == 0 && z1 == 0) return 0;
    if (x1 == 1 && z1 == 1) return z2 - x2;
    if (x1 == 1 && z1 == 0) return z2 * (2 * x2 - 1);
    return x2 * (1 - 2 * z2); /* x1 == 0, z1 == 1 */
}

/* rowsum(h, i) (Appendix A.2): row h <- row i * row h, with the sign from the mod-4 sum. */
void oracle_rowsum(otab *t, int h, int i)
{
    long sum = 2L * t->r[h] + 2L * t->r[i];
    for (int j = 0; j < t->n; ++j)
        sum += oracle_g(getx(t, i, j), getz(t, i, j), getx(t, h, j), getz(t, h, j));
    long m = ((sum % 4) + 4) % 4;
    if (m == 0) t->r[h] = 0;
    else if (m == 2) t->r[h] = 1;
    for (int j = 0; j < t->n; ++j) {
        setx(t, h, j, getx(t, i, j) ^ getx(t, h, j));
        setz(t, h, j, getz(t, i, j) ^ getz(t, h, j));
    }
}

/* Clifford gates (Table 1): the same bit rule on every row at the gate's column(s).  Rows
 * evolve independently under gates, so an instruction's targets are applied in order to one
 * row before moving to the next row (the row-per-thread view of Sec. 3.1). */
static void row_h(otab *t, int i, int a)
{
    int x = getx(t, i, a), z = getz(t, i, a);
    t->r[i] ^= (uint8_t)(x & z);
    setx(t, i, a, z);
    setz(t, i, a, x);
}

static void row_s(otab *t, int i, int a)
{
    int x = getx(t, i, a), z = getz(t, i, a);
    t->r[i] ^= (uint8_t)(x & z);   /* pre-gate z */
    setz(t, i, a, z ^ x);
}

static void row_cx(otab *t, int i, int c, int tg)
{
    int xc = getx(t, i, c), zc = getz(t, i, c), xt = getx(t, i, tg), zt = getz(t, i, tg);
    t->r[i] ^= (uint8_t)(xc & zt & (xt ^ zc ^ 1));
    setx(t, i, tg, xt ^ xc);
    setz(t, i, c, zc ^ zt);
}

static void gates(otab *t, uint32_t kind, const int32_t *tg, uint32_t nt)
{
    for (int i = 0; i < 2 * t->n; ++i) {
        if (kind == K_H) for (uint32_t q = 0; q < nt; ++q) row_h(t, i, tg[q]);
        else if (kind == K_S) for (uint32_t q = 0; q < nt; ++q) row_s(t, i, tg[q]);
        else for (uint32_t q = 0; q < nt; q += 2) row_cx(t, i, tg[q], tg[q + 1]);
    }
}

/* Pauli P in {1=X, 2=Y, 3=Z} on qubit a: flips the sign of every row it anticommutes with. */
static void pauli(otab *t, int a, int P)
{
    if (P == 0) return;
    for (int i = 0; i < 2 * t->n; ++i) {
        int x = getx(t, i, a), z = getz(t, i, a);
        int anti = (P == 1) ? z : (P == 3) ? x : (x ^ z);
        t->r[i] ^= (uint8_t)anti;
    }
}

/* Z measurement of qubit a (Sec. 2.4).  Returns the outcome; *was_random tells the branch.
 * rand_bit is the outcome used if the measurement is random. */
static int measure(otab *t, int a, int rand_bit, int *was_random)
{
    int n = t->n;
    int p = -1;
    for (int i = n; i < 2 * n; ++i)
        if (getx(t, i, a)) { p = i; break; }
    if (p >= 0) {
        for (int i = 0; i < 2 * n; ++i)
            if (i != p && getx(t, i, a)) oracle_rowsum(t, i, p);
        /* destabilizer p-n <- stabilizer p */
        memcpy(&t->x[(size_t)(p - n) * t->words], &t->x[(size_t)p * t->words], sizeof(uint64_t) * t->words);
        memcpy(&t->z[(size_t)(p - n) * t->words], &t->z[(size_t)p * t->words], sizeof(uint64_t) * t->words);
        t->r[p - n] = t->r[p];
        /* stabilizer p <- (-1)^outcome Z_a */
        for (int j = 0; j < n; ++j) { setx(t, p, j, 0); setz(t, p, j, 0); }
        setz(t, p, a, 1);
        t->r[p] = (uint8_t)(rand_bit & 1);
        *was_random = 1;
        return rand_bit & 1;
    }
    int s = 2 * n;
    for (int j = 0; j < n; ++j) { setx(t, s, j, 0); setz(t, s, j, 0); }
    t->r[s] = 0;
    for (int i = 0; i < n; ++i)
        if (getx(t, i, a)) oracle_rowsum(t, s, i + n);
    *was_random = 0;
    return t->r[s];
}

/* ------------------------------------------------------------------------------------------ */
/* Op-stream execution                                                                        */
/* ------------------------------------------------------------------------------------------ */

/* Execute instructions [0, ninstr) of a stream on one tableau.  instr_base is added to the
 * instruction index for the RNG counter.  Writes one byte per recorded measurement into rec
 * (if non-NULL) and, optionally, a flag per measurement target saying whether it was random.
 * Returns the number of recorded measurements, or -1 on a malformed stream. */
long oracle_exec(otab *t, const oinstr *ins, long ninstr, const int32_t *targets, long ntargets,
                 uint64_t seed, uint64_t shot, uint64_t instr_base,
                 uint8_t *rec, uint8_t *rand_flags, long *nflags)
{
    long off = 0, nrec = 0, nf = 0;
    int n = t->n;
    for (long k = 0; k < ninstr; ++k) {
        uint32_t kind = ins[k].kind, nt = ins[k].ntargets;
        if (kind >= K_COUNT || off + (long)nt > ntargets) return -1;
        const int32_t *tg = targets + off;
        for (uint32_t q = 0; q < nt; ++q)
            if (tg[q] < 0 || tg[q] >= n) return -1;
        if ((kind == K_CX || kind == K_DEP2) && (nt % 2)) return -1;
        uint64_t idx = instr_base + (uint64_t)k;
        uint64_t u[4];
        switch (kind) {
        case K_TICK: break;
        case K_H: case K_S: gates(t, kind, tg, nt); break;
        case K_X: for (uint32_t q = 0; q < nt; ++q) pauli(t, tg[q], 1); break;
        case K_Y: for (uint32_t q = 0; q < nt; ++q) pauli(t, tg[q], 2); break;
        case K_Z: for (uint32_t q = 0; q < nt; ++q) pauli(t, tg[q], 3); break;
        case K_CX:
            for (uint32_t q = 0; q < nt; q += 2)
                if (tg[q] == tg[q + 1]) return -1;
            gates(t, kind, tg, nt);
            break;
        case K_M: case K_MR: case K_R:
            for (uint32_t q = 0; q < nt; ++q) {
                draw(seed, shot, idx, q, u);
                int was_random = 0;
                int out = measure(t, tg[q], (int)(u[0] >> 63), &was_random);
                if (rand_flags) rand_flags[nf] = (uint8_t)was_random;
                nf++;
                if (kind != K_R) { if (rec) rec[nrec] = (uint8_t)out; nrec++; }
                if (kind != K_M && out) pauli(t, tg[q], 1);
            }
            break;
        case K_DEP1:
            for (uint32_t q = 0; q < nt; ++q) {
                draw(seed, shot, idx, q, u);
                if (u[0] < ins[k].t0) pauli(t, tg[q], (int)(1 + mulhi64(u[1], 3)));
            }
            break;
        case K_DEP2:
            for (uint32_t q = 0; q < nt; q += 2) {
                draw(seed, shot, idx, q / 2, u);
                if (u[0] < ins[k].t0) {
                    int kk = (int)(1 + mulhi64(u[1], 15));
                    pauli(t, tg[q], kk >> 2);
                    pauli(t, tg[q + 1], kk & 3);
                }
            }
            break;
        case K_PAULI1:
            for (uint32_t q = 0; q < nt; ++q) {
                draw(seed, shot, idx, q, u);
                if (u[0] < ins[k].t0) pauli(t, tg[q], 1);
                else if (u[0] < ins[k].t1) pauli(t, tg[q], 2);
                else if (u[0] < ins[k].t2) pauli(t, tg[q], 3);
            }
            break;
        case K_T1T2:
            /* relaxation then dephasing as a mixture: reset with probability t0, Z with
             * probability t1 - t0, else nothing; the reset's measurement draws u1 >> 63 */
            for (uint32_t q = 0; q < nt; ++q) {
                draw(seed, shot, idx, q, u);
                if (u[0] < ins[k].t0) {
                    int was_random = 0;
                    if (measure(t, tg[q], (int)(u[1] >> 63), &was_random)) pauli(t, tg[q], 1);
                } else if (u[0] < ins[k].t1) {
                    pauli(t, tg[q], 3);
                }
            }
            break;
        default: return -1;
        }
        off += nt;
    }
    if (nflags) *nflags = nf;
    return nrec;
}

/* Row-major export of rows 0..2n-1: x, z as one byte per bit ([2n][n]), r as [2n]. */
void oracle_tab_get(const otab *t, uint8_t *x, uint8_t *z, uint8_t *r)
{
    int n = t->n;
    for (int i = 0; i < 2 * n; ++i) {
        for (int j = 0; j < n; ++j) {
            if (x) x[(size_t)i * n + j] = (uint8_t)getx(t, i, j);
            if (z) z[(size_t)i * n + j] = (uint8_t)getz(t, i, j);
        }
        if (r) r[i] = t->r[i];
    }
}

/* Overwrite row i (0 <= i <= 2n, 2n = scratch) with the given bits, for unit tests. */
void oracle_tab_set_row(otab *t, int i, const uint8_t *x, const uint8_t *z, int r)
{
    for (int j = 0; j < t->n; ++j) { setx(t, i, j, x[j] & 1); setz(t, i, j, z[j] & 1); }
    t->r[i] = (uint8_t)(r & 1);
}

void oracle_tab_get_row(const otab *t, int i, uint8_t *x, uint8_t *z, uint8_t *r)
{
    for (int j = 0; j < t->n; ++j) { x[j] = (uint8_t)getx(t, i, j); z[j] = (uint8_t)getz(t, i, j); }
    *r = t->r[i];
}

/* Run `shots` independent shots (shot ids first_shot .. first_shot+shots-1) of a stream from
 * |0...0>.  rec: [shots][nrec] bytes.  tab_x/tab_z/tab_r (optional): final tableau of each shot,
 * [shots][2n][n] / [shots][2n].  Shots run in parallel with OpenMP when compiled with it.
 * Returns nrec, or -1 on error. */
long oracle_run(const oinstr *ins, long ninstr, const int32_t *targets, long ntargets, int n,
                long shots, uint64_t first_shot, uint64_t seed, uint8_t *rec, long nrec_expected,
                uint8_t *tab_x, uint8_t *tab_z, uint8_t *tab_r)
{
    long err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : err)
    for (long s = 0; s < shots; ++s) {
        otab *t = oracle_tab_new(n);
        if (!t) { err += 1; continue; }
        long got = oracle_exec(t, ins, ninstr, targets, ntargets, seed, first_shot + (uint64_t)s, 0,
                               rec ? rec + (size_t)s * nrec_expected : NULL, NULL, NULL);
        if (got != nrec_expected) err += 1;
        if (tab_x || tab_z || tab_r)
            oracle_tab_get(t, tab_x ? tab_x + (size_t)s * 2 * n * n : NULL,
                           tab_z ? tab_z + (size_t)s * 2 * n * n : NULL,
                           tab_r ? tab_r + (size_t)s * 2 * n : NULL);
        oracle_tab_free(t);
    }
    return err ? -1 : nrec_expected;
}

/* Threads OpenMP would use (1 when built without it). */
int oracle_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
