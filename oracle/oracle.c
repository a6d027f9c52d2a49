/*
 * oracle.c -- plain, slow CPU reference for the UAV coverage-path QUBO annealer.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code with the HIP path.
 *
 * What it computes (paper: "GPU-Accelerated Quantum Annealing-Inspired UAV Path
 * Planning for Smart Agriculture"):
 *   - the travel-time matrix between cell centres (Sec. II, system model),
 *   - the one-hot, time-indexed QUBO H_total = H_dist + P (H_visit + H_time)
 *     (Sec. III-B, eqs. (3)-(6)), in the closed-tour reading with the start cell
 *     fixed at step 0 (Sec. II, fixed start x_{0,0} = 1),
 *   - single-flip Metropolis annealing over independent replicas (the solver of
 *     Sec. III-C / Alg. 1 and the parallel-annealing description of Sec. IV-A;
 *     the paper gives no solver internals, so the sweep order, acceptance rule,
 *     schedule and random-number addressing below are this project's reading),
 *   - exact checkers: 2^N enumeration, brute force over tours, Held-Karp DP.
 *
 * Everything is written for clarity: dense int32 J built from its definition
 * (or, for fields too large to store it, each coefficient evaluated from the
 * same definition where it is used), O(N) field updates, no blocking or
 * fusion.  The only parallelism is an OpenMP loop over independent replicas.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator, from its published definition      */
/* (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,   */
/* 3", SC'11): 10 rounds of two 32x32->64 multiplies with fixed multipliers,  */
/* xor with the other half of the counter and the round key; the key is       */
/* advanced by two Weyl constants between rounds.                             */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Random word for site (t, c) (t = 1..m, c = 0..m-1).  Four consecutive steps
 * of one cell share a Philox call: counter word 0 = c + 65536 * ((t-1) / 4),
 * the word used is (t-1) mod 4.  Words 1..3 of the counter and the key are the
 * caller's (stream, sweep, replica, instance) address. */
static uint32_t site_word(int t, int c, uint32_t w1, uint32_t w2, uint32_t w3,
                          uint32_t seed, uint32_t stream)
{
    uint32_t ctr[4] = { (uint32_t)c + 65536u * (uint32_t)((t - 1) >> 2), w1, w2, w3 };
    uint32_t key[2] = { seed, stream };
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[(t - 1) & 3];
}

/* Acceptance draw u(inst, r, s, t, c): stream 0, counter {., s, r, inst}. */
uint32_t orc_accept_word(uint32_t seed, uint32_t inst, uint32_t r, uint32_t s, int t, int c)
{
    return site_word(t, c, s, r, inst, seed, 0u);
}

/* Initial bit: top bit of the stream-1 word, counter {., r, inst, 0}. */
uint32_t orc_init_bit(uint32_t seed, uint32_t inst, uint32_t r, int t, int c)
{
    return site_word(t, c, r, inst, 0u, seed, 1u) >> 31;
}

/* ------------------------------------------------------------------------ */
/* Instance and travel costs (Sec. II).                                       */
/* Cells c_{i,j} are numbered row-major, g = i*cols + j.  Travel time between */
/* cell centres is t_ij = d_ij * tau (Euclidean distance); with a 5 m cell and */
/* 5 m/s it is sqrt(q) seconds for q = di^2 + dj^2 in cell units.  Costs are   */
/* integers: w = round(scale * sqrt(q)) (scale 10 = deciseconds).             */
/* ------------------------------------------------------------------------ */
int32_t orc_cost(int32_t cols, int32_t ga, int32_t gb, int32_t scale)
{
    int32_t di = ga / cols - gb / cols, dj = ga % cols - gb % cols;
    double q = (double)di * di + (double)dj * dj;
    return (int32_t)lround((double)scale * sqrt(q));
}

/* Free cells F: every cell that is neither the depot nor a no-fly cell, in
 * increasing row-major index.  Returns m = |F|, writes F if non-NULL. */
int32_t orc_free_cells(int32_t rows, int32_t cols, int32_t depot, const uint8_t *nofly, int32_t *F)
{
    int32_t m = 0;
    for (int32_t g = 0; g < rows * cols; g++) {
        if (g == depot) continue;
        if (nofly && nofly[g]) continue;
        if (F) F[m] = g;
        m++;
    }
    return m;
}

/* Cost matrix over the visit list V = [depot, F_0, .., F_{m-1}]:
 * W[a*(m+1)+b] = w(V_a, V_b).  Returns w_max over all pairs. */
int32_t orc_cost_matrix(int32_t cols, int32_t depot, int32_t m, const int32_t *F,
                        int32_t scale, int32_t *W)
{
    int32_t wmax = 0;
    for (int32_t a = 0; a <= m; a++) {
        int32_t ga = a == 0 ? depot : F[a - 1];
        for (int32_t b = 0; b <= m; b++) {
            int32_t gb = b == 0 ? depot : F[b - 1];
            int32_t w = orc_cost(cols, ga, gb, scale);
            W[a * (m + 1) + b] = w;
            if (w > wmax) wmax = w;
        }
    }
    return wmax;
}

/* ------------------------------------------------------------------------ */
/* Literal Hamiltonian, eqs. (3)-(6), evaluated by loops on the full step x  */
/* cell occupation matrix.  Steps 0 and m+1 are pinned to the depot (fixed   */
/* start; closed tour returns to it); steps 1..m are the free variables      */
/* x[(t-1)*m + c].  closed = 0 drops the return leg (open path, eq. (1a)).    */
/*   H_dist  = sum_t sum_{a,b} w(a,b) X[t][a] X[t+1][b]                       */
/*   H_visit = sum_c (1 - sum_t X[t][c])^2     over free cells c              */
/*   H_time  = sum_t (1 - sum_c X[t][c])^2     over free steps t              */
/*   H = H_dist + P (H_visit + H_time)                                        */
/* ------------------------------------------------------------------------ */
int64_t orc_literal_energy(int32_t m, const int32_t *W, int32_t P, int32_t closed, const uint8_t *x)
{
    int32_t steps = m + 2, cells = m + 1;
    uint8_t *X = (uint8_t *)calloc((size_t)steps * cells, 1);
    X[0 * cells + 0] = 1;                       /* step 0 at the depot */
    if (closed) X[(m + 1) * cells + 0] = 1;     /* step m+1 back at the depot */
    for (int32_t t = 1; t <= m; t++)
        for (int32_t c = 0; c < m; c++)
            X[t * cells + (c + 1)] = x[(t - 1) * m + c];

    int64_t hdist = 0;
    for (int32_t t = 0; t + 1 < steps; t++)
        for (int32_t a = 0; a < cells; a++)
            for (int32_t b = 0; b < cells; b++)
                hdist += (int64_t)W[a * cells + b] * X[t * cells + a] * X[(t + 1) * cells + b];

    int64_t hvisit = 0;
    for (int32_t c = 1; c < cells; c++) {
        int64_t s = 0;
        for (int32_t t = 1; t <= m; t++) s += X[t * cells + c];
        hvisit += (1 - s) * (1 - s);
    }
    int64_t htime = 0;
    for (int32_t t = 1; t <= m; t++) {
        int64_t s = 0;
        for (int32_t c = 1; c < cells; c++) s += X[t * cells + c];
        htime += (1 - s) * (1 - s);
    }
    free(X);
    return hdist + (int64_t)P * (hvisit + htime);
}

/* ------------------------------------------------------------------------ */
/* QUBO form E(x) = c0 + sum_k b_k x_k + sum_{k<l} J_kl x_k x_l, obtained by  */
/* expanding eqs. (3)-(6) with x^2 = x:                                       */
/*   c0 = 2 P m                                                               */
/*   b_{t,c} = -2P + [t=1] w(depot,c) + [t=m, closed] w(c,depot)              */
/*   J_{(t,c),(t',c')} = 2P [t=t'] + 2P [c=c'] + w(c,c') [|t-t'| = 1]         */
/* Variable index k = (t-1)*m + c.                                            */
/* ------------------------------------------------------------------------ */
int32_t orc_J(int32_t m, const int32_t *W, int32_t P, int32_t k, int32_t l)
{
    if (k == l) return 0;
    int32_t t = k / m, c = k % m, t2 = l / m, c2 = l % m;
    int32_t v = 0;
    if (t == t2) v += 2 * P;
    if (c == c2) v += 2 * P;
    if (t - t2 == 1 || t2 - t == 1) v += W[(c + 1) * (m + 1) + (c2 + 1)];
    return v;
}

int32_t orc_b(int32_t m, const int32_t *W, int32_t P, int32_t closed, int32_t k)
{
    int32_t t = k / m + 1, c = k % m;
    int32_t v = -2 * P;
    if (t == 1) v += W[0 * (m + 1) + (c + 1)];
    if (t == m && closed) v += W[(c + 1) * (m + 1) + 0];
    return v;
}

void orc_build_qubo(int32_t m, const int32_t *W, int32_t P, int32_t closed,
                    int32_t *J /* N*N or NULL */, int32_t *b /* N */, int64_t *c0)
{
    int32_t N = m * m;
    for (int32_t k = 0; k < N; k++) {
        b[k] = orc_b(m, W, P, closed, k);
        if (J)
            for (int32_t l = 0; l < N; l++) J[(int64_t)k * N + l] = orc_J(m, W, P, k, l);
    }
    *c0 = 2LL * P * m;
}

int64_t orc_qubo_energy(int32_t N, const int32_t *J, const int32_t *b, int64_t c0, const uint8_t *x)
{
    int64_t e = c0;
    for (int32_t k = 0; k < N; k++) {
        if (!x[k]) continue;
        e += b[k];
        for (int32_t l = k + 1; l < N; l++)
            if (x[l]) e += J[(int64_t)k * N + l];
    }
    return e;
}

/* J_kl from the stored matrix, or from its definition when none is stored.  */
static inline int32_t J_at(const int32_t *J, int32_t N, int32_t m, const int32_t *W, int32_t P,
                           int32_t k, int32_t l)
{
    return J ? J[(int64_t)k * N + l] : orc_J(m, W, P, k, l);
}

/* E(x) = c0 + sum_k b_k x_k + sum_{k<l} J_kl x_k x_l, J stored or not. */
static int64_t qubo_energy_any(int32_t m, const int32_t *J, const int32_t *W, int32_t P, const int32_t *b,
                               int64_t c0, const uint8_t *x)
{
    int32_t N = m * m;
    int64_t e = c0;
    for (int32_t k = 0; k < N; k++) {
        if (!x[k]) continue;
        e += b[k];
        for (int32_t l = k + 1; l < N; l++)
            if (x[l]) e += J_at(J, N, m, W, P, k, l);
    }
    return e;
}

/* ------------------------------------------------------------------------ */
/* Schedule and acceptance thresholds.                                       */
/* T_s = T0 (T1/T0)^(s/(S-1)) (geometric; S = 1 gives T0).                    */
/* thr[s][d] = min(2^32-1, floor(2^32 exp(-d/T_s))) for d >= 1; thr[s][0] is  */
/* unused (a non-positive energy change is always accepted).                 */
/* Dmax = least d >= 1 with thr[0][d] = 0; a change is clamped to Dmax, where */
/* every row is zero because T_s <= T0.                                       */
/* ------------------------------------------------------------------------ */
double orc_temperature(double T0, double T1, int32_t S, int32_t s)
{
    if (S <= 1) return T0;
    return T0 * pow(T1 / T0, (double)s / (double)(S - 1));
}

static uint32_t thr_value(int32_t d, double T)
{
    double v = ldexp(exp(-(double)d / T), 32);
    double f = floor(v);
    if (f >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)f;
}

int32_t orc_dmax(double T0)
{
    int32_t d = 1;
    while (thr_value(d, T0) != 0) d++;
    return d;
}

void orc_thresholds(double T0, double T1, int32_t S, int32_t Dmax, uint32_t *thr /* S*(Dmax+1) */)
{
    for (int32_t s = 0; s < S; s++) {
        double T = orc_temperature(T0, T1, S, s);
        thr[(int64_t)s * (Dmax + 1) + 0] = 0xFFFFFFFFu;
        for (int32_t d = 1; d <= Dmax; d++)
            thr[(int64_t)s * (Dmax + 1) + d] = thr_value(d, T);
    }
}

/* ------------------------------------------------------------------------ */
/* The annealer.  For each replica r (independently):                        */
/*   x  <- initial state (Bernoulli(1/2) bits from stream 1, or given)       */
/*   h_k = b_k + sum_{l != k} J_kl x_l ;  E = E(x)                            */
/*   best_E <- +inf                                                          */
/*   for s = start .. S-1:                                                   */
/*     for k = 0 .. N-1 (t-major order):                                     */
/*       dE = (1 - 2 x_k) h_k                                                */
/*       accept if dE <= 0, else draw u = u(inst,r,s,t,c) and accept iff     */
/*         u < thr[s][min(dE, Dmax)]  (no draw when that entry is 0)         */
/*       on accept: x_k ^= 1, h_l += (x_k' - x_k) J_kl for l != k, E += dE   */
/*     at the end of the sweep: if E < best_E then best_E, best_sweep, best_x */
/* ------------------------------------------------------------------------ */
static int64_t field_energy_mismatch(int32_t m, const int32_t *J, const int32_t *W, int32_t P, const int32_t *b,
                                     int64_t c0, const uint8_t *x, const int32_t *h, int64_t E)
{
    int32_t N = m * m;
    int64_t bad = 0;
    for (int32_t k = 0; k < N; k++) {
        int64_t v = b[k];
        for (int32_t l = 0; l < N; l++)
            if (l != k && x[l]) v += J_at(J, N, m, W, P, k, l);
        if (v != h[k]) bad++;
    }
    if (qubo_energy_any(m, J, W, P, b, c0, x) != E) bad++;
    return bad;
}

/* One in-order sweep s of replica r over all N sites with table row `row`
 * (the loop body of the annealer above); updates x, h, E and the counters. */
static void sweep_once(int32_t m, const int32_t *J, const int32_t *W, int32_t P, const uint32_t *row, int32_t Dmax,
                       uint32_t seed, uint32_t inst, uint32_t r, int32_t s, uint8_t *x, int32_t *h, int64_t *E,
                       uint64_t *acc, uint64_t *drw)
{
    int32_t N = m * m;
    for (int32_t k = 0; k < N; k++) {
        int32_t t = k / m + 1, c = k % m;
        int32_t dE = x[k] ? -h[k] : h[k];
        int accept;
        if (dE <= 0) {
            accept = 1;
        } else {
            uint32_t th = row[dE < Dmax ? dE : Dmax];
            if (th == 0) {
                accept = 0;
            } else {
                (*drw)++;
                accept = orc_accept_word(seed, inst, r, (uint32_t)s, t, c) < th;
            }
        }
        if (accept) {
            int32_t delta = x[k] ? -1 : 1;
            x[k] ^= 1;
            for (int32_t l = 0; l < N; l++)
                if (l != k) h[l] += delta * J_at(J, N, m, W, P, k, l);
            *E += dE;
            (*acc)++;
        }
    }
}

/* J may be NULL: then every coefficient comes from orc_J(m, W, P, ., .). */
int32_t orc_anneal(int32_t m, const int32_t *J, const int32_t *W, int32_t P, const int32_t *b, int64_t c0,
                   int32_t S, int32_t Dmax, const uint32_t *thr,
                   uint32_t seed, uint32_t inst, int32_t n_rep, const int32_t *rep_ids,
                   const uint8_t *init_x, const int32_t *start_sweep, int32_t check_every,
                   uint8_t *final_x, int64_t *final_E, int64_t *best_E, int32_t *best_sweep,
                   uint8_t *best_x, uint64_t *accepts, uint64_t *draws, int64_t *mismatches,
                   int32_t n_threads)
{
    int32_t N = m * m;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int32_t i = 0; i < n_rep; i++) {
        uint32_t r = (uint32_t)rep_ids[i];
        uint8_t *x = final_x + (int64_t)i * N;
        uint8_t *bx = best_x + (int64_t)i * N;
        int32_t *h = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));

        for (int32_t k = 0; k < N; k++) {
            int32_t t = k / m + 1, c = k % m;
            x[k] = init_x ? init_x[(int64_t)i * N + k] : (uint8_t)orc_init_bit(seed, inst, r, t, c);
        }
        for (int32_t k = 0; k < N; k++) {
            int32_t v = b[k];
            for (int32_t l = 0; l < N; l++)
                if (l != k && x[l]) v += J_at(J, N, m, W, P, k, l);
            h[k] = v;
        }
        int64_t E = qubo_energy_any(m, J, W, P, b, c0, x);
        int64_t bE = INT64_MAX;
        int32_t bs = -1;
        uint64_t acc = 0, drw = 0;
        int64_t bad = 0;
        memcpy(bx, x, (size_t)N);
        int32_t s0 = start_sweep ? start_sweep[i] : 0;

        for (int32_t s = s0; s < S; s++) {
            sweep_once(m, J, W, P, thr + (int64_t)s * (Dmax + 1), Dmax, seed, inst, r, s, x, h, &E, &acc, &drw);
            if (E < bE) {
                bE = E;
                bs = s;
                memcpy(bx, x, (size_t)N);
            }
            if (check_every > 0 && ((s - s0 + 1) % check_every == 0 || s == S - 1))
                bad += field_energy_mismatch(m, J, W, P, b, c0, x, h, E);
        }
        final_E[i] = E;
        best_E[i] = bE;
        best_sweep[i] = bs;
        accepts[i] = acc;
        draws[i] = drw;
        if (mismatches) mismatches[i] = bad;
        free(h);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Exact checkers.                                                           */
/* ------------------------------------------------------------------------ */

/* Minimum of E over all 2^N states by direct evaluation of every state
 * (N <= 24).  Returns the minimum, the number of minimisers and the first
 * minimiser (in counting order); also the minimum over states that are not
 * permutation matrices (INT64_MAX if none). */
int32_t orc_enum_min(int32_t m, const int32_t *J, const int32_t *b, int64_t c0,
                     int64_t *min_E, int64_t *n_min, uint8_t *argmin, int64_t *min_infeasible)
{
    int32_t N = m * m;
    if (N > 24) return -1;
    int64_t best = INT64_MAX, cnt = 0, binf = INT64_MAX;
    uint64_t arg = 0;
    uint8_t *x = (uint8_t *)malloc((size_t)(N > 0 ? N : 1));
    for (uint64_t v = 0; v < (1ull << N); v++) {
        for (int32_t k = 0; k < N; k++) x[k] = (uint8_t)((v >> k) & 1);
        int64_t e = orc_qubo_energy(N, J, b, c0, x);
        if (e < best) { best = e; cnt = 1; arg = v; }
        else if (e == best) cnt++;
        int feasible = 1;
        for (int32_t t = 0; t < m && feasible; t++) {
            int s = 0;
            for (int32_t c = 0; c < m; c++) s += x[t * m + c];
            if (s != 1) feasible = 0;
        }
        for (int32_t c = 0; c < m && feasible; c++) {
            int s = 0;
            for (int32_t t = 0; t < m; t++) s += x[t * m + c];
            if (s != 1) feasible = 0;
        }
        if (!feasible && e < binf) binf = e;
    }
    for (int32_t k = 0; k < N; k++) argmin[k] = (uint8_t)((arg >> k) & 1);
    *min_E = best;
    *n_min = cnt;
    *min_infeasible = binf;
    free(x);
    return 0;
}

/* Brute force over all m! visiting orders (m <= 11): cost of the tour
 * depot -> F[p_1] -> ... -> F[p_m] (-> depot when closed). */
static int64_t tour_cost(int32_t m, const int32_t *W, int32_t closed, const int32_t *p)
{
    int64_t c = W[0 * (m + 1) + (p[0] + 1)];
    for (int32_t i = 0; i + 1 < m; i++) c += W[(p[i] + 1) * (m + 1) + (p[i + 1] + 1)];
    if (closed) c += W[(p[m - 1] + 1) * (m + 1) + 0];
    return c;
}

int32_t orc_tour_brute(int32_t m, const int32_t *W, int32_t closed, int64_t *best, int64_t *n_opt)
{
    if (m < 1 || m > 11) return -1;
    int32_t p[11], cidx[11];
    for (int32_t i = 0; i < m; i++) { p[i] = i; cidx[i] = 0; }
    int64_t b = tour_cost(m, W, closed, p), cnt = 1;
    /* Heap's algorithm, iterative form. */
    int32_t i = 0;
    while (i < m) {
        if (cidx[i] < i) {
            int32_t j = (i % 2 == 0) ? 0 : cidx[i];
            int32_t tmp = p[j]; p[j] = p[i]; p[i] = tmp;
            int64_t c = tour_cost(m, W, closed, p);
            if (c < b) { b = c; cnt = 1; }
            else if (c == b) cnt++;
            cidx[i]++;
            i = 0;
        } else {
            cidx[i] = 0;
            i++;
        }
    }
    *best = b;
    *n_opt = cnt;
    return 0;
}

/* Held-Karp dynamic programme (textbook): best[S][j] = cheapest path from the
 * depot through the set S of free cells ending at j.  m <= 24; a path has at
 * most 25 legs of at most 2^24 each here, so the table holds int32 (1.6 GB at
 * m = 24).  Returns -1 if m is out of range or the table cannot be allocated. */
int64_t orc_held_karp(int32_t m, const int32_t *W, int32_t closed)
{
    if (m < 1 || m > 24) return -1;
    for (int32_t i = 0; i < (m + 1) * (m + 1); i++)
        if (W[i] < 0 || W[i] >= (1 << 24)) return -1;
    const int32_t INF = INT32_MAX;
    uint32_t full = (1u << m);
    int32_t *dp = (int32_t *)malloc(sizeof(int32_t) * (size_t)full * (size_t)m);
    if (!dp) return -1;
    for (uint64_t i = 0; i < (uint64_t)full * m; i++) dp[i] = INF;
    for (int32_t j = 0; j < m; j++) dp[(1u << j) * (uint64_t)m + j] = W[0 * (m + 1) + (j + 1)];
    for (uint32_t set = 1; set < full; set++) {
        for (int32_t j = 0; j < m; j++) {
            if (!(set & (1u << j))) continue;
            int32_t cur = dp[(uint64_t)set * m + j];
            if (cur == INF) continue;
            for (int32_t k = 0; k < m; k++) {
                if (set & (1u << k)) continue;
                uint32_t ns = set | (1u << k);
                int32_t v = cur + W[(j + 1) * (m + 1) + (k + 1)];
                if (v < dp[(uint64_t)ns * m + k]) dp[(uint64_t)ns * m + k] = v;
            }
        }
    }
    int64_t best = INT64_MAX;
    for (int32_t j = 0; j < m; j++) {
        int64_t v = dp[(uint64_t)(full - 1) * m + j];
        if (closed) v += W[(j + 1) * (m + 1) + 0];
        if (v < best) best = v;
    }
    free(dp);
    return best;
}

/* ------------------------------------------------------------------------ */
/* Warm-start seed sampler (integer).  For t = 1..m: W = sum over unvisited  */
/* cells of q[c][t-1]; u = word 0 of Philox({t, r, inst, 0}, {seed, 4});     */
/* target = floor(u W / 2^32); step t goes to the first unvisited cell (in   */
/* free-list order) whose running sum of weights exceeds the target.         */
/* q is m rows (cells) of 128 steps; x receives the m x m permutation state. */
/* ------------------------------------------------------------------------ */
int32_t orc_sample_seed(int32_t m, const uint16_t *q, uint32_t seed, uint32_t inst, uint32_t r, uint8_t *x)
{
    uint8_t used[256];
    if (m < 1 || m > 128) return -1;
    memset(used, 0, sizeof used);
    memset(x, 0, (size_t)m * m);
    for (int32_t t = 1; t <= m; t++) {
        uint64_t W = 0;
        for (int32_t c = 0; c < m; c++)
            if (!used[c]) W += q[c * 128 + (t - 1)];
        uint32_t ctr[4] = { (uint32_t)t, r, inst, 0u }, key[2] = { seed, 4u }, out[4];
        orc_philox4x32_10(ctr, key, out);
        uint64_t target = ((uint64_t)out[0] * W) >> 32;
        uint64_t run = 0;
        int32_t pick = -1;
        for (int32_t c = 0; c < m; c++) {
            if (used[c]) continue;
            run += q[c * 128 + (t - 1)];
            if (run > target) { pick = c; break; }
        }
        if (pick < 0) return -2;
        used[pick] = 1;
        x[(t - 1) * m + pick] = 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Replica exchange (parallel tempering), an extension of the paper's many-  */
/* replica search (Sec. III-C): the paper runs independent replicas; here K  */
/* of them per chain index r sit at fixed temperatures and trade states.     */
/*                                                                          */
/* Ladder: T_k = T_hot (T_cold/T_hot)^(k/(K-1)), k = 0..K-1 (hottest first;  */
/* K = 1 gives T_hot).  Slot k sweeps at the constant temperature T_k, its   */
/* draws addressed by the instance id inst + k (inst: the chain set's id).   */
/* Exchange between slots k and k+1 of chain r (states x, x', energies E,    */
/* E'): the swap is accepted with probability                               */
/*   min(1, exp((1/T_{k+1} - 1/T_k) (E' - E))),                              */
/* the Metropolis rule on the product of the two Boltzmann weights.  In       */
/* integers: with db = 1/T_{k+1} - 1/T_k (> 0) and d = E' - E, accept when    */
/* d >= 0; otherwise with a = -d draw u and accept iff                       */
/*   u < xthr[k][min(a, DX_k)],  xthr[k][a] = min(2^32-1, floor(2^32 e^{-a db}))*/
/* (no draw when that entry is 0).  DX_k = least a >= 1 with a zero entry.   */
/* u = word 0 of Philox({k, round, r, inst}, {seed, 5}).                     */
/* Round e exchanges the pairs (k, k+1) with k = e mod 2, 4, ...             */
/* ------------------------------------------------------------------------ */
double orc_pt_temperature(double T_hot, double T_cold, int32_t K, int32_t k)
{
    if (K <= 1) return T_hot;
    return T_hot * pow(T_cold / T_hot, (double)k / (double)(K - 1));
}

static uint32_t xthr_value(int64_t a, double db)
{
    double f = floor(ldexp(exp(-(double)a * db), 32));
    if (f >= 4294967295.0) return 0xFFFFFFFFu;
    return (uint32_t)f;
}

/* DX[k] for the K-1 pairs; returns the largest, or -1 when a pair's db is not
 * positive or a DX exceeds cap. */
int32_t orc_pt_dx(double T_hot, double T_cold, int32_t K, int32_t cap, int32_t *DX)
{
    int32_t mx = 1;
    for (int32_t k = 0; k + 1 < K; k++) {
        double db = 1.0 / orc_pt_temperature(T_hot, T_cold, K, k + 1) - 1.0 / orc_pt_temperature(T_hot, T_cold, K, k);
        if (!(db > 0.0)) return -1;
        int32_t a = 1;
        while (xthr_value(a, db) != 0) {
            if (++a > cap) return -1;
        }
        DX[k] = a;
        if (a > mx) mx = a;
    }
    return mx;
}

/* xthr[k][a] for a = 0..DX[k] (row stride `stride` >= max DX + 1; entries past
 * DX[k] are zero). */
void orc_pt_tables(double T_hot, double T_cold, int32_t K, const int32_t *DX, int32_t stride, uint32_t *xthr)
{
    for (int32_t k = 0; k + 1 < K; k++) {
        double db = 1.0 / orc_pt_temperature(T_hot, T_cold, K, k + 1) - 1.0 / orc_pt_temperature(T_hot, T_cold, K, k);
        uint32_t *row = xthr + (int64_t)k * stride;
        for (int32_t a = 0; a < stride; a++) row[a] = a <= DX[k] ? xthr_value(a, db) : 0u;
    }
}

uint32_t orc_pt_word(uint32_t seed, uint32_t inst, uint32_t r, uint32_t round, int32_t k)
{
    uint32_t ctr[4] = { (uint32_t)k, round, r, inst }, key[2] = { seed, 5u }, out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[0];
}

/* One exchange round over chains 0..R-1.  x: [K][R][N] bytes, E: [K][R].
 * swaps[k] (may be NULL) counts accepted exchanges of pair k. */
int32_t orc_pt_exchange(int32_t K, int32_t R, int32_t N, uint32_t round, uint32_t seed, uint32_t inst,
                        const int32_t *DX, int32_t stride, const uint32_t *xthr,
                        uint8_t *x, int64_t *E, uint64_t *swaps)
{
    uint8_t *tmp = (uint8_t *)malloc((size_t)(N > 0 ? N : 1));
    for (int32_t k = (int32_t)(round & 1u); k + 1 < K; k += 2) {
        for (int32_t r = 0; r < R; r++) {
            int64_t *Eh = E + (int64_t)k * R + r, *Ec = E + (int64_t)(k + 1) * R + r;
            int64_t d = *Ec - *Eh;
            int accept;
            if (d >= 0) {
                accept = 1;
            } else {
                int64_t a = -d;
                uint32_t th = xthr[(int64_t)k * stride + (a < DX[k] ? a : DX[k])];
                accept = th != 0 && orc_pt_word(seed, inst, (uint32_t)r, round, k) < th;
            }
            if (!accept) continue;
            uint8_t *xh = x + ((int64_t)k * R + r) * N, *xc = x + ((int64_t)(k + 1) * R + r) * N;
            memcpy(tmp, xh, (size_t)N);
            memcpy(xh, xc, (size_t)N);
            memcpy(xc, tmp, (size_t)N);
            int64_t t = *Eh; *Eh = *Ec; *Ec = t;
            if (swaps) swaps[k]++;
        }
    }
    free(tmp);
    return 0;
}

/* Parallel tempering of the chains chain_ids[0..n_chain-1], each independent
 * of the others: slot k of chain r starts from the stream-1 bits of instance
 * inst + k and sweeps with table row thr[k] (a constant temperature; entries
 * up to Dmax, zero past the slot's own cutoff) and instance id inst + k; after
 * sweep s, when (s + 1) is a multiple of `interval` and s + 1 < S, exchange
 * round e = (s + 1) / interval - 1 runs on the chain's pairs (k = e mod 2,
 * k + 2, ...) with the rule of orc_pt_exchange, swapping states, fields and
 * energies.  Each slot keeps its best at its sweep ends.  Outputs per chain i
 * and slot k at [i][k]; swaps per chain and pair at [i][k]. */
int32_t orc_pt_anneal(int32_t m, const int32_t *J, const int32_t *W, int32_t P, const int32_t *b, int64_t c0,
                      int32_t K, int32_t S, int32_t interval, int32_t Dmax, const uint32_t *thr,
                      const int32_t *DX, int32_t stride, const uint32_t *xthr,
                      uint32_t seed, uint32_t inst, int32_t n_chain, const int32_t *chain_ids,
                      uint8_t *final_x, int64_t *final_E, int64_t *best_E, int32_t *best_sweep, uint8_t *best_x,
                      uint64_t *accepts, uint64_t *draws, uint64_t *swaps, int32_t n_threads)
{
    int32_t N = m * m;
    if (K < 1 || interval < 1) return -1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int32_t i = 0; i < n_chain; i++) {
        uint32_t r = (uint32_t)chain_ids[i];
        uint8_t *xs = final_x + (int64_t)i * K * N;
        uint8_t *bxs = best_x + (int64_t)i * K * N;
        int32_t *hs = (int32_t *)malloc(sizeof(int32_t) * (size_t)K * (size_t)(N > 0 ? N : 1));
        int32_t *htmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
        uint8_t *xtmp = (uint8_t *)malloc((size_t)(N > 0 ? N : 1));
        int64_t *Es = final_E + (int64_t)i * K, *bE = best_E + (int64_t)i * K;
        int32_t *bs = best_sweep + (int64_t)i * K;
        uint64_t *acc = accepts + (int64_t)i * K, *drw = draws + (int64_t)i * K;
        uint64_t *sw = swaps ? swaps + (int64_t)i * (K > 1 ? K - 1 : 1) : NULL;
        for (int32_t k = 0; k < K; k++) {
            uint8_t *x = xs + (int64_t)k * N;
            int32_t *h = hs + (int64_t)k * N;
            for (int32_t v = 0; v < N; v++) x[v] = (uint8_t)orc_init_bit(seed, inst + (uint32_t)k, r, v / m + 1, v % m);
            for (int32_t v = 0; v < N; v++) {
                int32_t f = b[v];
                for (int32_t l = 0; l < N; l++)
                    if (l != v && x[l]) f += J_at(J, N, m, W, P, v, l);
                h[v] = f;
            }
            Es[k] = qubo_energy_any(m, J, W, P, b, c0, x);
            bE[k] = INT64_MAX;
            bs[k] = -1;
            acc[k] = drw[k] = 0;
            memcpy(bxs + (int64_t)k * N, x, (size_t)N);
        }
        if (sw)
            for (int32_t k = 0; k + 1 < K; k++) sw[k] = 0;
        for (int32_t s = 0; s < S; s++) {
            for (int32_t k = 0; k < K; k++) {
                uint8_t *x = xs + (int64_t)k * N;
                sweep_once(m, J, W, P, thr + (int64_t)k * (Dmax + 1), Dmax, seed, inst + (uint32_t)k, r, s, x,
                           hs + (int64_t)k * N, &Es[k], &acc[k], &drw[k]);
                if (Es[k] < bE[k]) {
                    bE[k] = Es[k];
                    bs[k] = s;
                    memcpy(bxs + (int64_t)k * N, x, (size_t)N);
                }
            }
            if (K < 2 || (s + 1) % interval != 0 || s + 1 >= S) continue;
            uint32_t e = (uint32_t)((s + 1) / interval - 1);
            for (int32_t k = (int32_t)(e & 1u); k + 1 < K; k += 2) {
                int64_t d = Es[k + 1] - Es[k];
                int accept;
                if (d >= 0) {
                    accept = 1;
                } else {
                    int64_t a = -d;
                    uint32_t th = xthr[(int64_t)k * stride + (a < DX[k] ? a : DX[k])];
                    accept = th != 0 && orc_pt_word(seed, inst, r, e, k) < th;
                }
                if (!accept) continue;
                uint8_t *x0 = xs + (int64_t)k * N, *x1 = xs + (int64_t)(k + 1) * N;
                int32_t *h0 = hs + (int64_t)k * N, *h1 = hs + (int64_t)(k + 1) * N;
                memcpy(xtmp, x0, (size_t)N); memcpy(x0, x1, (size_t)N); memcpy(x1, xtmp, (size_t)N);
                memcpy(htmp, h0, sizeof(int32_t) * (size_t)N); memcpy(h0, h1, sizeof(int32_t) * (size_t)N);
                memcpy(h1, htmp, sizeof(int32_t) * (size_t)N);
                int64_t t = Es[k]; Es[k] = Es[k + 1]; Es[k + 1] = t;
                if (sw) sw[k]++;
            }
        }
        free(hs);
        free(htmp);
        free(xtmp);
    }
    return 0;
}
