/* Host-only memory and undefined-behaviour check of the oracle's C code:
 * random simple graphs (n = 0, 1, 2, 7, 40, 120, three densities each),
 * every oracle entry point at h = 1..4, with random alive masks, repeated
 * vertex ids in the list call, a trace capacity too small for the peel, the
 * certificate over all vertices (which must pass on the oracle's own cores)
 * and the sampling peel.  Built with gcc -fsanitize=address,undefined by
 * tests/test_oracle_sanitized.py; exits 0 on success. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
int oracle_check_csr(uint32_t n, const uint64_t *row_ptr, const uint32_t *col);
int oracle_hdeg(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, const uint8_t *alive, uint32_t h, uint32_t *deg);
int oracle_hdeg_list(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, const uint8_t *alive, uint32_t h,
                     const uint32_t *verts, uint64_t count, uint32_t *deg_out, uint64_t *te_out, int threads);
int oracle_peel(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t h, uint32_t *core, uint32_t *round,
                uint32_t *trace_k, uint32_t *trace_p, uint32_t *trace_a, uint64_t trace_cap, uint64_t *rounds_out);
int oracle_certificate(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t h, const uint32_t *c,
                       const uint32_t *rho, const uint32_t *verts, uint64_t count, uint64_t *fail_out, int threads);
int oracle_peel_sampled(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t h, const uint8_t *sampled,
                        uint32_t *core, uint32_t *est_out);

static uint64_t rs = 88172645463325252ull;
static uint32_t rnd(void) { rs ^= rs << 13; rs ^= rs >> 7; rs ^= rs << 17; return (uint32_t)rs; }

/* random simple undirected graph as CSR */
static void make(uint32_t n, uint32_t m, uint64_t **rp, uint32_t **col) {
    uint8_t *adj = calloc((size_t)n * n + 1, 1);
    for (uint32_t e = 0; e < m && n > 1; e++) {
        uint32_t a = rnd() % n, b = rnd() % n;
        if (a != b) adj[(size_t)a * n + b] = adj[(size_t)b * n + a] = 1;
    }
    *rp = malloc((n + 1) * sizeof(uint64_t));
    uint64_t nnz = 0;
    for (uint32_t a = 0; a < n; a++) for (uint32_t b = 0; b < n; b++) nnz += adj[(size_t)a * n + b];
    *col = malloc((nnz ? nnz : 1) * sizeof(uint32_t));
    uint64_t k = 0;
    for (uint32_t a = 0; a < n; a++) {
        (*rp)[a] = k;
        for (uint32_t b = 0; b < n; b++) if (adj[(size_t)a * n + b]) (*col)[k++] = b;
    }
    (*rp)[n] = k;
    free(adj);
}

int main(void) {
    uint32_t sizes[] = {0, 1, 2, 7, 40, 120};
    for (int si = 0; si < 6; si++) {
        uint32_t n = sizes[si];
        for (int rep = 0; rep < 3; rep++) {
            uint64_t *rp; uint32_t *col;
            make(n, n * (rep + 1), &rp, &col);
            if (oracle_check_csr(n, rp, col) != 0) { printf("csr invalid n=%u\n", n); return 1; }
            uint32_t nn = n ? n : 1;
            uint32_t *deg = malloc(nn * 4), *core = malloc(nn * 4), *round = malloc(nn * 4), *est = malloc(nn * 4);
            uint8_t *alive = malloc(nn), *samp = malloc(nn);
            uint32_t *verts = malloc(nn * 2 * 4), *dl = malloc(nn * 2 * 4);
            uint64_t *te = malloc(nn * 2 * 8);
            for (uint32_t i = 0; i < n; i++) { alive[i] = rnd() % 4 != 0; samp[i] = rnd() % 3 == 0; }
            for (uint32_t i = 0; i < 2 * n; i++) verts[i] = rnd() % n;
            for (uint32_t h = 1; h <= 4; h++) {
                if (oracle_hdeg(n, rp, col, NULL, h, deg)) return 2;
                if (oracle_hdeg(n, rp, col, alive, h, deg)) return 2;
                if (oracle_hdeg_list(n, rp, col, alive, h, verts, 2 * (uint64_t)n, dl, te, 3)) return 3;
                uint32_t tk[4], tp[4], ta[4];
                uint64_t rounds = 0;
                int rc = oracle_peel(n, rp, col, h, core, round, tk, tp, ta, 4, &rounds);
                if (rc != 0 && rc != -2) return 4;
                uint64_t fail[3] = {0, 0, 0};
                if (oracle_certificate(n, rp, col, h, core, round, NULL, n, fail, 2)) return 5;
                if (fail[0] || fail[1] || fail[2]) { printf("certificate violation n=%u h=%u\n", n, h); return 6; }
                if (oracle_peel_sampled(n, rp, col, h, samp, core, est)) return 7;
            }
            free(deg); free(core); free(round); free(est); free(alive); free(samp); free(verts); free(dl); free(te);
            free(rp); free(col);
        }
    }
    printf("oracle sanitizer run ok\n");
    return 0;
}
