/*
 * sanitize_driver.c -- runs the oracle (chp_oracle.c) on an op stream read from a file, so the
 * oracle can be built as a standalone program with AddressSanitizer and UndefinedBehaviorSanitizer
 * (TEST INFRASTRUCTURE ONLY: the CPU test suite builds and runs it; the product never does).
 *
 * Input file: 7 int64 (n, shots, first_shot, seed, ninstr, ntargets, nrec), then ninstr
 * 32-byte instructions (kind u32, ntargets u32, t0 u64, t1 u64, t2 u64), then ntargets int32.
 * Output file: shots * nrec record bytes (0/1), then each shot's final tableau (x, z as
 * [2n][n] bytes, r as [2n]).  Exit status 0 on success, 2 on bad input, 3 on an oracle error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct { uint32_t kind, ntargets; uint64_t t0, t1, t2; } dinstr;

long oracle_run(const void *ins, long ninstr, const int32_t *targets, long ntargets, int n,
                long shots, uint64_t first_shot, uint64_t seed, uint8_t *rec, long nrec_expected,
                uint8_t *tab_x, uint8_t *tab_z, uint8_t *tab_r);

int main(int argc, char **argv)
{
    if (argc != 3) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t h[7];
    if (fread(h, sizeof h, 1, f) != 1) { fclose(f); return 2; }
    const int n = (int)h[0];
    const long shots = (long)h[1], ninstr = (long)h[4], ntg = (long)h[5], nrec = (long)h[6];
    if (n < 1 || shots < 1 || ninstr < 0 || ntg < 0 || nrec < 0) { fclose(f); return 2; }
    dinstr *ins = (dinstr *)malloc(sizeof(dinstr) * (size_t)(ninstr ? ninstr : 1));
    int32_t *tg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ntg ? ntg : 1));
    const size_t sq = (size_t)shots * 2 * (size_t)n * (size_t)n;
    uint8_t *rec = (uint8_t *)calloc((size_t)shots * (size_t)(nrec ? nrec : 1), 1);
    uint8_t *tx = (uint8_t *)malloc(sq), *tz = (uint8_t *)malloc(sq);
    uint8_t *tr = (uint8_t *)malloc((size_t)shots * 2 * (size_t)n);
    int rc = 0;
    if (!ins || !tg || !rec || !tx || !tz || !tr) rc = 2;
    else if (fread(ins, sizeof(dinstr), (size_t)ninstr, f) != (size_t)ninstr) rc = 2;
    else if (fread(tg, sizeof(int32_t), (size_t)ntg, f) != (size_t)ntg) rc = 2;
    fclose(f);
    if (rc == 0 && oracle_run(ins, ninstr, tg, ntg, n, shots, (uint64_t)h[2], (uint64_t)h[3], rec, nrec,
                              tx, tz, tr) != nrec)
        rc = 3;
    if (rc == 0) {
        FILE *o = fopen(argv[2], "wb");
        if (!o) rc = 2;
        else {
            fwrite(rec, 1, (size_t)shots * (size_t)nrec, o);
            fwrite(tx, 1, sq, o);
            fwrite(tz, 1, sq, o);
            fwrite(tr, 1, (size_t)shots * 2 * (size_t)n, o);
            fclose(o);
        }
    }
    free(ins); free(tg); free(rec); free(tx); free(tz); free(tr);
    return rc;
}
