/*
 * Seeded synthetic inputs, host side.
 *
 * This file holds no arithmetic of the graph method; it only produces the
 * random numbers and R-MAT edge keys that both the CPU oracle and the GPU
 * library consume as inputs.
 *
 * Counter-based generator: Philox4x32-10 as defined by Salmon, Moraes, Dror
 * and Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 128-bit
 * counter and a 64-bit key, ten rounds of two 32x32->64 multiplies with the
 * key bumped by the Weyl constants between rounds.
 *
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM'04): edge k picks one quadrant per
 * level with probabilities a/b/c/d; the quadrant draw for level l uses word
 * (l mod 4) of Philox(key = seed, counter = (k_lo, k_hi, l/4, 0)).
 */
#include <stdint.h>
#include <stddef.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

static inline void philox_round(uint32_t c[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * c[0];
    uint64_t p1 = (uint64_t)PHILOX_M1 * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void rmatgen_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k[0] += PHILOX_W0;
            k[1] += PHILOX_W1;
        }
        philox_round(c, k);
    }
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

/* Block b of stream `stream`: Philox(key = seed, counter = (b_lo, b_hi, stream, 0)).
 * Fills out[0 .. count) with the words of blocks first_block, first_block+1, ... */
void rmatgen_philox_stream(uint64_t seed, uint32_t stream, uint64_t first_word,
                           int64_t count, uint32_t* out) {
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for schedule(static)
    for (int64_t w = 0; w < count; ++w) {
        uint64_t word = first_word + (uint64_t)w;
        uint64_t b = word >> 2;
        uint32_t ctr[4] = {(uint32_t)b, (uint32_t)(b >> 32), stream, 0u};
        uint32_t r[4];
        rmatgen_philox4x32_10(ctr, key, r);
        out[w] = r[word & 3];
    }
}

/* Raw R-MAT edge keys (u << 32 | v) for edges first .. first+count-1.
 * thr[0..2] are the cumulative quadrant thresholds A, A+B, A+B+C in units of 2^-32. */
void rmatgen_rmat_keys(int scale, uint64_t seed, uint64_t first, int64_t count,
                       uint32_t thrA, uint32_t thrAB, uint32_t thrABC, uint64_t* keys) {
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < count; ++e) {
        uint64_t k = first + (uint64_t)e;
        uint32_t u = 0, v = 0;
        uint32_t r[4] = {0, 0, 0, 0};
        for (int l = 0; l < scale; ++l) {
            if ((l & 3) == 0) {
                uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), (uint32_t)(l >> 2), 0u};
                rmatgen_philox4x32_10(ctr, key, r);
            }
            uint32_t x = r[l & 3];
            uint32_t q = x < thrA ? 0u : (x < thrAB ? 1u : (x < thrABC ? 2u : 3u));
            u = (u << 1) | (q >> 1);
            v = (v << 1) | (q & 1u);
        }
        keys[e] = ((uint64_t)u << 32) | (uint64_t)v;
    }
}
