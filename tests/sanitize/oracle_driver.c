/* Drives the oracle (instance, costs, QUBO, energies, schedule, annealing with
 * and without a stored J, enumeration, brute force, Held-Karp, seed sampling,
 * replica exchange)
 * for a build under AddressSanitizer and UndefinedBehaviorSanitizer. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

uint32_t orc_init_bit(uint32_t seed, uint32_t inst, uint32_t r, int t, int c);
int32_t orc_free_cells(int32_t rows, int32_t cols, int32_t depot, const uint8_t *nofly, int32_t *F);
int32_t orc_cost_matrix(int32_t cols, int32_t depot, int32_t m, const int32_t *F, int32_t scale, int32_t *W);
int64_t orc_literal_energy(int32_t m, const int32_t *W, int32_t P, int32_t closed, const uint8_t *x);
void orc_build_qubo(int32_t m, const int32_t *W, int32_t P, int32_t closed, int32_t *J, int32_t *b, int64_t *c0);
int64_t orc_qubo_energy(int32_t N, const int32_t *J, const int32_t *b, int64_t c0, const uint8_t *x);
int32_t orc_dmax(double T0);
void orc_thresholds(double T0, double T1, int32_t S, int32_t Dmax, uint32_t *thr);
int32_t orc_anneal(int32_t m, const int32_t *J, const int32_t *W, int32_t P, const int32_t *b, int64_t c0,
                   int32_t S, int32_t Dmax, const uint32_t *thr, uint32_t seed, uint32_t inst, int32_t n_rep,
                   const int32_t *rep_ids, const uint8_t *init_x, const int32_t *start_sweep, int32_t check_every,
                   uint8_t *final_x, int64_t *final_E, int64_t *best_E, int32_t *best_sweep, uint8_t *best_x,
                   uint64_t *accepts, uint64_t *draws, int64_t *mismatches, int32_t n_threads);
int32_t orc_enum_min(int32_t m, const int32_t *J, const int32_t *b, int64_t c0, int64_t *min_E, int64_t *n_min,
                     uint8_t *argmin, int64_t *min_infeasible);
int32_t orc_tour_brute(int32_t m, const int32_t *W, int32_t closed, int64_t *best, int64_t *n_opt);
int64_t orc_held_karp(int32_t m, const int32_t *W, int32_t closed);
int32_t orc_sample_seed(int32_t m, const uint16_t *q, uint32_t seed, uint32_t inst, uint32_t r, uint8_t *x);
int32_t orc_pt_dx(double T_hot, double T_cold, int32_t K, int32_t cap, int32_t *DX);
void orc_pt_tables(double T_hot, double T_cold, int32_t K, const int32_t *DX, int32_t stride, uint32_t *xthr);
int32_t orc_pt_exchange(int32_t K, int32_t R, int32_t N, uint32_t round, uint32_t seed, uint32_t inst,
                        const int32_t *DX, int32_t stride, const uint32_t *xthr, uint8_t *x, int64_t *E,
                        uint64_t *swaps);
int32_t orc_pt_anneal(int32_t m, const int32_t *J, const int32_t *W, int32_t P, const int32_t *b, int64_t c0,
                      int32_t K, int32_t S, int32_t interval, int32_t Dmax, const uint32_t *thr,
                      const int32_t *DX, int32_t stride, const uint32_t *xthr,
                      uint32_t seed, uint32_t inst, int32_t n_chain, const int32_t *chain_ids,
                      uint8_t *final_x, int64_t *final_E, int64_t *best_E, int32_t *best_sweep, uint8_t *best_x,
                      uint64_t *accepts, uint64_t *draws, uint64_t *swaps, int32_t n_threads);

#define CHECK(c)                                                                \
    do {                                                                        \
        if (!(c)) {                                                             \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);     \
            return 1;                                                           \
        }                                                                       \
    } while (0)

static int field(int rows, int cols, int closed, int with_J)
{
    uint8_t *nf = calloc((size_t)rows * cols, 1);
    int32_t *F = malloc(sizeof(int32_t) * (size_t)rows * cols);
    int32_t m = orc_free_cells(rows, cols, 0, nf, F);
    CHECK(m == rows * cols - 1);
    int32_t N = m * m;
    int32_t *W = malloc(sizeof(int32_t) * (size_t)(m + 1) * (m + 1));
    int32_t wmax = orc_cost_matrix(cols, 0, m, F, 10, W);
    int32_t P = 2 * wmax;
    int32_t *b = malloc(sizeof(int32_t) * (size_t)N);
    int32_t *J = with_J ? malloc(sizeof(int32_t) * (size_t)N * N) : NULL;
    int64_t c0 = 0;
    orc_build_qubo(m, W, P, closed, J, b, &c0);
    uint8_t *x = calloc((size_t)N, 1);
    for (int32_t t = 0; t < m; t++) x[t * m + (t * 7 + 3) % m] = 1;
    int64_t lit = orc_literal_energy(m, W, P, closed, x);
    if (J) CHECK(orc_qubo_energy(N, J, b, c0, x) == lit);

    const int32_t S = 12, n = 3;
    int32_t Dmax = orc_dmax(80.0);
    uint32_t *thr = malloc(sizeof(uint32_t) * (size_t)S * (Dmax + 1));
    orc_thresholds(80.0, 0.5, S, Dmax, thr);
    int32_t reps[3] = {0, 4, 9}, start[3] = {0, 3, S};
    uint8_t *fx = malloc((size_t)n * N), *bx = malloc((size_t)n * N);
    int64_t fE[3], bE[3], mis[3];
    int32_t bs[3];
    uint64_t acc[3], drw[3];
    CHECK(orc_anneal(m, J, W, P, b, c0, S, Dmax, thr, 5, 2, n, reps, NULL, start, 4, fx, fE, bE, bs, bx, acc, drw,
                     mis, 1) == 0);
    for (int i = 0; i < n; i++) CHECK(mis[i] == 0);

    /* marginals: m cells x 128 steps of uint16 weights */
    uint16_t *q = malloc(sizeof(uint16_t) * (size_t)m * 128);
    for (int32_t k = 0; k < m * 128; k++) q[k] = (uint16_t)(1 + (k * 37) % 500);
    CHECK(orc_sample_seed(m, q, 9, 2, 1, x) == 0);
    for (int32_t t = 0; t < m; t++) {
        int32_t ones = 0;
        for (int32_t c = 0; c < m; c++) ones += x[t * m + c];
        CHECK(ones == 1);
    }
    if (m <= 9) {
        int64_t best = 0, nopt = 0;
        CHECK(orc_tour_brute(m, W, closed, &best, &nopt) == 0);
        CHECK(orc_held_karp(m, W, closed) == best);
    }
    free(nf); free(F); free(W); free(b); free(J); free(x); free(thr); free(fx); free(bx); free(q);
    return 0;
}

int main(void)
{
    if (field(3, 3, 1, 1) || field(3, 4, 0, 1) || field(4, 4, 1, 0) || field(6, 6, 1, 0)) return 1;
    /* 2^9 enumeration on the 2x2 field */
    {
        int32_t F[4], W[16], b[9], J[81];
        uint8_t nf[4] = {0, 0, 0, 0}, arg[9];
        int32_t m = orc_free_cells(2, 2, 0, nf, F);
        CHECK(m == 3);
        int32_t wmax = orc_cost_matrix(2, 0, m, F, 10, W);
        int64_t c0 = 0, mn = 0, nmin = 0, minf = 0;
        orc_build_qubo(m, W, 2 * wmax, 1, J, b, &c0);
        CHECK(orc_enum_min(m, J, b, c0, &mn, &nmin, arg, &minf) == 0 && mn < minf);
    }
    /* replica exchange: ladder tables and a few rounds */
    {
        enum { K = 6, R = 7, N = 5 };
        int32_t DX[K];
        int32_t mx = orc_pt_dx(90.0, 2.0, K, 1 << 22, DX);
        CHECK(mx > 1);
        uint32_t *xt = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(K - 1) * (size_t)(mx + 1));
        orc_pt_tables(90.0, 2.0, K, DX, mx + 1, xt);
        uint8_t x[K * R * N];
        int64_t E[K * R];
        uint64_t sw[K - 1] = {0};
        for (int i = 0; i < K * R * N; i++) x[i] = (uint8_t)(i & 1);
        for (int i = 0; i < K * R; i++) E[i] = (int64_t)((i * 37) % 101) - 20;
        for (uint32_t rnd = 0; rnd < 5; rnd++) CHECK(orc_pt_exchange(K, R, N, rnd, 3, 1, DX, mx + 1, xt, x, E, sw) == 0);
        /* a whole tempering run of two chains on the 3x3 field (J computed on the fly) */
        {
            int32_t F[9], W[100], b[64];
            uint8_t nf[9] = {0};
            int32_t m = orc_free_cells(3, 3, 0, nf, F);
            int32_t wmax = orc_cost_matrix(3, 0, m, F, 10, W);
            int64_t c0 = 0;
            int32_t *Jf = (int32_t *)malloc(sizeof(int32_t) * 64 * 64);
            orc_build_qubo(m, W, 2 * wmax, 1, Jf, b, &c0);
            int32_t Dm = orc_dmax(90.0);
            uint32_t *tt = (uint32_t *)calloc((size_t)K * (size_t)(Dm + 1), sizeof(uint32_t));
            for (int k = 0; k < K; k++) orc_thresholds(90.0 - 10.0 * k, 90.0 - 10.0 * k, 1, Dm, tt + (size_t)k * (Dm + 1));
            int32_t ch[2] = {0, 5};
            uint8_t fx[2 * K * 64], bx[2 * K * 64];
            int64_t fE[2 * K], bE2[2 * K];
            int32_t bs2[2 * K];
            uint64_t ac[2 * K], dr[2 * K], sw2[2 * (K - 1)];
            CHECK(orc_pt_anneal(m, NULL, W, 2 * wmax, b, c0, K, 12, 2, Dm, tt, DX, mx + 1, xt, 1, 0, 2, ch, fx, fE, bE2,
                                bs2, bx, ac, dr, sw2, 1) == 0);
            free(tt);
            free(Jf);
        }
        free(xt);
    }
    printf("oracle driver: clean\n");
    return 0;
}
