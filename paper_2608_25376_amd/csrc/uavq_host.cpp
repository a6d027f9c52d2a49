// Host side of libuavq: QUBO construction, schedule table, host energy and
// path decoding, plan packing and the C entry points.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "uavq_internal.h"

namespace uavq {

static thread_local std::string g_err;

int set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// floor(sqrt(v)) for v >= 0, exact for all 64-bit inputs used here.
static int64_t isqrt64(int64_t v) {
    int64_t r = (int64_t)std::sqrt((double)v);
    while (r > 0 && r * r > v) r--;
    while ((r + 1) * (r + 1) <= v) r++;
    return r;
}

// round(scale * sqrt(q)) = floor((isqrt(4 scale^2 q) + 1) / 2); exact because
// 4 scale^2 q is even, so scale*sqrt(q) is never a half-integer.
static int32_t travel_cost(int32_t cols, int32_t ga, int32_t gb, int32_t scale) {
    int64_t di = ga / cols - gb / cols, dj = ga % cols - gb % cols;
    int64_t q = di * di + dj * dj;
    return (int32_t)((isqrt64(4LL * scale * scale * q) + 1) >> 1);
}

static double temperature(double T0, double T1, int32_t S, int32_t s) {
    return S <= 1 ? T0 : T0 * std::pow(T1 / T0, (double)s / (double)(S - 1));
}

static uint32_t threshold(int32_t d, double T) {
    double v = std::floor(std::ldexp(std::exp(-(double)d / T), 32));
    return v >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)v;
}

// Rows s = 0..S-1 of the acceptance table, entries 0..Dmax of each, row s at
// dst + s * stride.  exp(-k/T) decreases in k, so past a row's first zero
// every entry is zero and needs no exp.
static void fill_schedule(double T0, double T1, int32_t S, int32_t Dmax, uint32_t *dst, size_t stride) {
    for (int32_t s = 0; s < S; s++) {
        const double T = temperature(T0, T1, S, s);
        uint32_t *row = dst + (size_t)s * stride;
        row[0] = 0xFFFFFFFFu;
        int32_t k = 1;
        for (; k <= Dmax; k++)
            if ((row[k] = threshold(k, T)) == 0) break;
        for (; k <= Dmax; k++) row[k] = 0;
    }
}

}  // namespace uavq

using namespace uavq;

extern "C" {

const char *uavq_last_error(void) { return g_err.c_str(); }

int32_t uavq_version(void) { return 101; }

int uavq_qubo_build(const uavq_grid *g, uavq_qubo **out) {
    if (!g || !out) return set_error(UAVQ_EINVAL, "qubo_build: null argument");
    *out = nullptr;
    if (g->rows < 1 || g->cols < 1 || (int64_t)g->rows * g->cols > 65536)
        return set_error(UAVQ_EINVAL, "qubo_build: grid %dx%d out of range", g->rows, g->cols);
    int32_t cells = g->rows * g->cols;
    if (g->depot < 0 || g->depot >= cells) return set_error(UAVQ_EINVAL, "qubo_build: start cell out of range");
    if (g->nofly && g->nofly[g->depot]) return set_error(UAVQ_EINVAL, "qubo_build: start cell is no-fly");
    int32_t scale = g->cost_scale ? g->cost_scale : 10;
    if (scale < 1 || scale > 10000) return set_error(UAVQ_EINVAL, "qubo_build: cost_scale out of range");

    uavq_qubo *q = new (std::nothrow) uavq_qubo();
    if (!q) return set_error(UAVQ_ENOMEM, "qubo_build: out of memory");
    q->rows = g->rows; q->cols = g->cols; q->depot = g->depot; q->scale = scale;
    q->closed = (g->flags & UAVQ_OPEN_PATH) ? 0 : 1;
    for (int32_t c = 0; c < cells; c++)
        if (c != g->depot && !(g->nofly && g->nofly[c])) q->F.push_back(c);
    int32_t m = (int32_t)q->F.size();
    if (m < 1) { delete q; return set_error(UAVQ_EINVAL, "qubo_build: no cell to visit"); }
    q->m = m;
    q->N = m * m;
    q->row_words = (m + 31) / 32;

    // visit list V = [start, F...]; W over V x V
    q->W.assign((size_t)(m + 1) * (m + 1), 0);
    int32_t wmax = 0;
    for (int32_t a = 0; a <= m; a++) {
        int32_t ga = a ? q->F[a - 1] : g->depot;
        for (int32_t b = 0; b <= m; b++) {
            int32_t gb = b ? q->F[b - 1] : g->depot;
            int32_t w = travel_cost(g->cols, ga, gb, scale);
            q->W[(size_t)a * (m + 1) + b] = w;
            wmax = std::max(wmax, w);
        }
    }
    q->wmax = wmax;
    if (wmax > 65535) { delete q; return set_error(UAVQ_ETOOBIG, "qubo_build: w_max %d > 65535", wmax); }
    int32_t P = g->penalty ? g->penalty : 2 * wmax;
    if (P <= wmax) { delete q; return set_error(UAVQ_EINVAL, "qubo_build: penalty %d <= w_max %d", P, wmax); }
    // Every local field and energy change the kernels form is an int32: with
    // R_t, C_c <= m and travel rows <= m w_max, |h| + |k 2P| stays below
    // 2P (3m + 2) + 2 m w_max, kept under 2^30 (and 2P within 24 bits).
    if (P > (1 << 20) || 2LL * P * (3LL * m + 2) + 2LL * m * wmax >= (1LL << 30)) {
        delete q;
        return set_error(UAVQ_EINVAL, "qubo_build: penalty %d too large for m = %d", P, m);
    }
    q->P = P;
    q->c0 = 2LL * P * m;
    q->D16.resize((size_t)m * m);
    q->ddep16.resize(m);
    for (int32_t c = 0; c < m; c++) {
        q->ddep16[c] = (uint16_t)q->W[c + 1];
        for (int32_t c2 = 0; c2 < m; c2++)
            q->D16[(size_t)c * m + c2] = (uint16_t)q->W[(size_t)(c + 1) * (m + 1) + c2 + 1];
    }
    if (wmax <= 255) {   // the byte copies the LDS-resident kernels and the MFMA refresh read
        q->D.assign(q->D16.begin(), q->D16.end());
        q->ddep.assign(q->ddep16.begin(), q->ddep16.end());
    }
    q->b.resize(q->N);
    for (int32_t t = 1; t <= m; t++)
        for (int32_t c = 0; c < m; c++) {
            int32_t v = -2 * P;
            if (t == 1) v += q->ddep16[c];
            if (t == m && q->closed) v += q->ddep16[c];
            q->b[(size_t)(t - 1) * m + c] = v;
        }
    if (g->flags & UAVQ_DENSE) {
        // J <= 2P + w_max must split into two int8 limbs (J & 127, J >> 7 <= 127)
        if (q->N > 46340 || 2 * P + wmax > 16383) {
            delete q;
            return set_error(UAVQ_ETOOBIG, "qubo_build: dense J too large (N=%d, P=%d)", m * m, P);
        }
        try {
            q->J.assign((size_t)q->N * q->N, 0);
        } catch (...) {
            delete q;
            return set_error(UAVQ_ENOMEM, "qubo_build: dense J allocation failed");
        }
        // same step: 2P between different cells; same cell: 2P between
        // different steps; adjacent steps: travel cost between the cells.
        for (int32_t t = 0; t < m; t++)
            for (int32_t c = 0; c < m; c++) {
                int16_t *row = &q->J[(size_t)(t * m + c) * q->N];
                for (int32_t c2 = 0; c2 < m; c2++)
                    if (c2 != c) row[t * m + c2] += (int16_t)(2 * P);
                for (int32_t t2 = 0; t2 < m; t2++)
                    if (t2 != t) row[t2 * m + c] += (int16_t)(2 * P);
                for (int32_t dt = -1; dt <= 1; dt += 2) {
                    int32_t t2 = t + dt;
                    if (t2 < 0 || t2 >= m) continue;
                    for (int32_t c2 = 0; c2 < m; c2++) row[t2 * m + c2] += (int16_t)q->D16[(size_t)c * m + c2];
                }
            }
    }
    *out = q;
    return UAVQ_OK;
}

void uavq_qubo_free(uavq_qubo *q) { delete q; }

int uavq_qubo_info(const uavq_qubo *q, uavq_qubo_info_t *info) {
    if (!q || !info) return set_error(UAVQ_EINVAL, "qubo_info: null argument");
    info->m = q->m;
    info->n_vars = q->N;
    info->P = q->P;
    info->w_max = q->wmax;
    info->c0 = q->c0;
    info->closed = q->closed;
    info->has_dense = q->J.empty() ? 0 : 1;
    info->row_words = q->row_words;
    info->state_words = q->m * q->row_words;
    return UAVQ_OK;
}

int uavq_qubo_free_cells(const uavq_qubo *q, int32_t *F) {
    if (!q || !F) return set_error(UAVQ_EINVAL, "qubo_free_cells: null argument");
    std::memcpy(F, q->F.data(), sizeof(int32_t) * q->F.size());
    return UAVQ_OK;
}

int uavq_qubo_costs(const uavq_qubo *q, int32_t *W) {
    if (!q || !W) return set_error(UAVQ_EINVAL, "qubo_costs: null argument");
    std::memcpy(W, q->W.data(), sizeof(int32_t) * q->W.size());
    return UAVQ_OK;
}

int uavq_qubo_export(const uavq_qubo *q, int32_t *b, int32_t *J) {
    if (!q || !b) return set_error(UAVQ_EINVAL, "qubo_export: null argument");
    std::memcpy(b, q->b.data(), sizeof(int32_t) * q->b.size());
    if (J) {
        if (q->J.empty()) return set_error(UAVQ_EINVAL, "qubo_export: built without UAVQ_DENSE");
        for (size_t i = 0; i < q->J.size(); i++) J[i] = q->J[i];
    }
    return UAVQ_OK;
}

// E = c0 + sum_k b_k x_k + P sum_t R_t (R_t - 1) + P sum_c C_c (C_c - 1)
//     + sum_{t=1}^{m-1} sum_{c,c'} D[c][c'] x_{t,c} x_{t+1,c'}
// (R_t, C_c the step and cell occupation counts): the pair sum of the
// expanded form grouped by the three kinds of coupling.
int uavq_energy_eval(const uavq_qubo *q, const uint32_t *x, int64_t n, int64_t *E) {
    if (!q || (n > 0 && (!x || !E)) || n < 0) return set_error(UAVQ_EINVAL, "energy_eval: bad argument");
    const int32_t m = q->m, W = q->row_words, sw = m * W;
    std::vector<int32_t> colcnt(m);
    std::vector<int32_t> ones, prev;
    for (int64_t i = 0; i < n; i++) {
        const uint32_t *s = x + i * sw;
        int64_t e = q->c0;
        std::fill(colcnt.begin(), colcnt.end(), 0);
        prev.clear();
        for (int32_t t = 1; t <= m; t++) {
            ones.clear();
            for (int32_t c = 0; c < m; c++)
                if ((s[(size_t)(t - 1) * W + (c >> 5)] >> (c & 31)) & 1u) ones.push_back(c);
            int64_t R = (int64_t)ones.size();
            e += (int64_t)q->P * R * (R - 1);
            for (int32_t c : ones) {
                e += q->b[(size_t)(t - 1) * m + c];
                colcnt[c]++;
                for (int32_t cp : prev) e += q->D16[(size_t)cp * m + c];
            }
            prev.swap(ones);
        }
        for (int32_t c = 0; c < m; c++) e += (int64_t)q->P * colcnt[c] * (colcnt[c] - 1);
        E[i] = e;
    }
    return UAVQ_OK;
}

int uavq_decode_path(const uavq_qubo *q, const uint32_t *x, int32_t *path, int64_t *cost) {
    if (!q || !x || !path || !cost) return set_error(UAVQ_EINVAL, "decode_path: null argument");
    const int32_t m = q->m, W = q->row_words;
    std::vector<int32_t> order(m, -1);
    std::vector<char> used(m, 0);
    for (int32_t t = 1; t <= m; t++) {
        for (int32_t c = 0; c < m; c++) {
            if (!((x[(size_t)(t - 1) * W + (c >> 5)] >> (c & 31)) & 1u)) continue;
            if (order[t - 1] >= 0 || used[c])
                return set_error(UAVQ_EINFEASIBLE, "decode_path: step %d or cell %d occupied twice", t, c);
            order[t - 1] = c;
            used[c] = 1;
        }
        if (order[t - 1] < 0) return set_error(UAVQ_EINFEASIBLE, "decode_path: step %d empty", t);
    }
    int64_t total = q->ddep16[order[0]];
    path[0] = q->depot;
    for (int32_t t = 0; t < m; t++) {
        path[t + 1] = q->F[order[t]];
        if (t > 0) total += q->D16[(size_t)order[t - 1] * m + order[t]];
    }
    if (q->closed) {
        total += q->ddep16[order[m - 1]];
        path[m + 1] = q->depot;
    } else {
        path[m + 1] = -1;
    }
    *cost = total;
    return UAVQ_OK;
}

// Per-cell features of the warm-start network (16 per free cell, free-list order).
int uavq_mlp_features(const uavq_qubo *q, float *X) {
    if (!q || !X) return set_error(UAVQ_EINVAL, "mlp_features: null argument");
    const int32_t R = q->rows, Cn = q->cols, m = q->m;
    std::vector<uint8_t> freecell((size_t)R * Cn, 0);
    freecell[q->depot] = 1;
    for (int32_t g : q->F) freecell[g] = 1;
    const int32_t side = std::max(R, Cn);
    const double den = side > 1 ? (double)(side - 1) : 1.0;
    const int32_t i0 = q->depot / Cn, j0 = q->depot % Cn;
    for (int32_t c = 0; c < m; c++) {
        const int32_t i = q->F[c] / Cn, j = q->F[c] % Cn;
        float *f = X + (size_t)c * 16;
        f[0] = (float)(i / den);
        f[1] = (float)(j / den);
        f[2] = (float)((i - i0) / den);
        f[3] = (float)((j - j0) / den);
        f[4] = (float)(std::sqrt((double)(i - i0) * (i - i0) + (double)(j - j0) * (j - j0)) / (std::sqrt(2.0) * den));
        int nf1 = 0, nf2 = 0;
        int ring_free[9] = {0}, ring_all[9] = {0};
        for (int32_t a = 0; a < R; a++)
            for (int32_t b = 0; b < Cn; b++) {
                const int32_t d = std::max(std::abs(a - i), std::abs(b - j));
                if (d == 0 || d > 8) continue;
                const bool fr = freecell[(size_t)a * Cn + b] != 0;
                if (!fr && d == 1) nf1++;
                if (!fr && d <= 2) nf2++;
                ring_all[d]++;
                if (fr) ring_free[d]++;
            }
        f[5] = (float)(nf1 / 8.0);
        f[6] = (float)(nf2 / 24.0);
        for (int r = 1; r <= 8; r++) f[6 + r] = ring_all[r] ? (float)((double)ring_free[r] / ring_all[r]) : 0.0f;
        f[15] = (float)(m / 99.0);
    }
    return UAVQ_OK;
}

int uavq_schedule(double T0, double T1, int32_t S, int32_t *Dmax, uint32_t *thr) {
    if (!Dmax || S < 1 || !(T1 > 0.0) || !(T1 <= T0) || !std::isfinite(T0) || T0 > 1e7)
        return set_error(UAVQ_EINVAL, "schedule: need S >= 1 and 0 < T1 <= T0 (finite)");
    int32_t d = 1;
    while (threshold(d, T0) != 0) d++;
    *Dmax = d;
    if (thr) fill_schedule(T0, T1, S, d, thr, (size_t)d + 1);
    return UAVQ_OK;
}

// ------------------------------------------------------- replica exchange --

static uint32_t exchange_threshold(int64_t a, double db) {
    double v = std::floor(std::ldexp(std::exp(-(double)a * db), 32));
    return v >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)v;
}

int uavq_pt_ladder(double T_hot, double T_cold, int32_t K, double *T, int32_t *DX, int32_t *max_dx, uint32_t *xthr,
                   int32_t stride) {
    if (!T || !max_dx || (K > 1 && !DX)) return set_error(UAVQ_EINVAL, "pt_ladder: null argument");
    if (K < 1 || K > 4096) return set_error(UAVQ_EINVAL, "pt_ladder: K = %d outside 1..4096", K);
    if (!std::isfinite(T_hot) || !(T_hot > 0.0) || T_hot > 1e7 ||
        (K > 1 && (!std::isfinite(T_cold) || !(T_cold > 0.0) || !(T_cold < T_hot))))
        return set_error(UAVQ_EINVAL, "pt_ladder: need 0 < T_cold < T_hot (finite)");
    for (int32_t k = 0; k < K; k++) T[k] = temperature(T_hot, T_cold, K, k);
    constexpr int32_t kCap = 1 << 22;
    int32_t mx = 1;
    for (int32_t k = 0; k + 1 < K; k++) {
        const double db = 1.0 / T[k + 1] - 1.0 / T[k];
        if (!(db > 0.0)) return set_error(UAVQ_ETOOBIG, "pt_ladder: slots %d and %d share a temperature", k, k + 1);
        int32_t a = 1;
        while (exchange_threshold(a, db) != 0)
            if (++a > kCap) return set_error(UAVQ_ETOOBIG, "pt_ladder: exchange table of pair %d exceeds 2^22", k);
        DX[k] = a;
        mx = std::max(mx, a);
    }
    *max_dx = mx;
    if (!xthr) return UAVQ_OK;
    if (stride < mx + 1) return set_error(UAVQ_EINVAL, "pt_ladder: stride %d < max DX + 1 = %d", stride, mx + 1);
    for (int32_t k = 0; k + 1 < K; k++) {
        const double db = 1.0 / T[k + 1] - 1.0 / T[k];
        uint32_t *row = xthr + (size_t)k * stride;
        for (int32_t a = 0; a < stride; a++) row[a] = a <= DX[k] ? exchange_threshold(a, db) : 0u;
    }
    return UAVQ_OK;
}

// ------------------------------------------------------------------ plans --

// Chunk class of an instance: ceil(m/64), and at least kByteChunks + 1 when
// its costs do not fit a byte (only those classes read 16-bit costs).
static int inst_class(const uavq_qubo *q, bool dense) {
    if (dense) return 1;
    const int c = (q->m + 63) / 64;
    return q->wmax > 255 ? std::max(c, kByteChunks + 1) : c;
}

// Replicas per workgroup by chunk class: eight for three chunks (one
// table-row copy per sweep serves eight replicas; measured on the 12x12 field:
// 371 ms against 377 with four and 374 with sixteen), four otherwise (two
// chunks with eight: the 256-field batch took 774 ms against 738, its last
// workgroups running longer alone).
static int default_waves_per_block(int chunks) {
    return chunks == 3 ? 8 : 4;
}

int uavq_plan_create(const uavq_qubo *const *q, int32_t n_inst, const uint32_t *inst_ids,
                     const uavq_anneal_params *p, uavq_plan **out) {
    if (!out || !p || n_inst < 0 || (n_inst > 0 && (!q || !inst_ids)))
        return set_error(UAVQ_EINVAL, "plan_create: bad argument");
    *out = nullptr;
    if (p->replicas < 1 || p->replicas > (1 << 20)) return set_error(UAVQ_EINVAL, "plan_create: replicas out of range");
    if (p->sweeps < 1) return set_error(UAVQ_EINVAL, "plan_create: sweeps must be >= 1");
    if (p->waves_per_block < 0 || p->waves_per_block > 16)
        return set_error(UAVQ_EINVAL, "plan_create: waves_per_block must be 0..16");
    const bool dense = (p->flags & UAVQ_KERNEL_DENSE) != 0;
    for (int32_t i = 0; i < n_inst; i++) {
        if (!q[i]) return set_error(UAVQ_EINVAL, "plan_create: null qubo %d", i);
        if (dense && q[i]->J.empty()) return set_error(UAVQ_EINVAL, "plan_create: dense kernel needs UAVQ_DENSE (instance %d)", i);
        if (dense && q[i]->N > 4096)
            return set_error(UAVQ_ETOOBIG, "plan_create: dense kernel holds at most 4096 variables (N = %d)", q[i]->N);
        if (!dense && q[i]->m > kMaxM)
            return set_error(UAVQ_ETOOBIG, "plan_create: m = %d exceeds the factored kernel's %d", q[i]->m, kMaxM);
    }
    int32_t Dmax = 0;
    int rc = uavq_schedule(p->T0, p->T1, p->sweeps, &Dmax, nullptr);
    if (rc) return rc;
    // per-instance schedules; the table width covers the hottest
    std::vector<double> sT(2 * (size_t)std::max(n_inst, 1));
    for (int32_t i = 0; i < n_inst; i++) {
        sT[2 * i] = p->inst_T ? p->inst_T[2 * i] : p->T0;
        sT[2 * i + 1] = p->inst_T ? p->inst_T[2 * i + 1] : p->T1;
        int32_t di = 0;
        if (uavq_schedule(sT[2 * i], sT[2 * i + 1], p->sweeps, &di, nullptr))
            return set_error(UAVQ_EINVAL, "plan_create: schedule of instance %d needs 0 < T1 <= T0 (finite)", i);
        Dmax = std::max(Dmax, di);
    }

    uavq_plan *pl = new (std::nothrow) uavq_plan();
    if (!pl) return set_error(UAVQ_ENOMEM, "plan_create: out of memory");
    pl->p = *p;
    pl->p.inst_T = nullptr;   // the caller's array is read above only
    pl->n_inst = n_inst;
    pl->S = p->sweeps;
    pl->Dmax = Dmax;
    pl->dense = dense ? 1 : 0;
    pl->variant = (p->flags & UAVQ_VARIANT_ROWMASK) ? UAVQ_VARIANT_ROWMASK : 0;
    if (p->tune) pl->variant = p->tune->variant_flags & UAVQ_VARIANT_ROWMASK;
    pl->no_producer = (p->flags & UAVQ_VARIANT_NOPRODUCER) ? 1 : 0;
    if (p->tune) pl->no_producer = (p->tune->variant_flags & UAVQ_VARIANT_NOPRODUCER) ? 1 : 0;
    pl->generic_chunk = (p->flags & UAVQ_VARIANT_GENERIC) ? 1 : 0;
    if (p->tune) pl->generic_chunk = (p->tune->variant_flags & UAVQ_VARIANT_GENERIC) ? 1 : 0;
    pl->stop_frozen = (p->flags & UAVQ_STOP_FROZEN) ? 1 : 0;
    pl->reduce_at_end = (p->flags & UAVQ_REDUCE_AT_END) ? 1 : 0;
    pl->concurrent = (p->flags & UAVQ_CONCURRENT_CLASSES) ? 1 : 0;
    if (p->tune) pl->concurrent |= (p->tune->variant_flags & UAVQ_CONCURRENT_CLASSES) ? 1 : 0;
    pl->persistent = (p->flags & UAVQ_PERSISTENT) ? 1 : 0;
    pl->graph = (p->flags & UAVQ_GRAPH) ? 1 : 0;
    const int32_t S = p->sweeps, R = p->replicas;

    // Distinct schedules share their rows: S rows for a cooling schedule, one
    // row for a constant temperature.  Device copy with rows padded to a
    // multiple of 4 entries (16-byte rows).
    pl->thr_stride = (Dmax + 2 + 3) & ~3;   // entries 0..Dmax, then zeros (at least one)
    pl->sched_T = sT;
    std::vector<int32_t> sched_of(std::max(n_inst, 1), 0), sched_row, sched_rows;
    std::vector<double> uT;
    for (int32_t i = 0; i < n_inst; i++) {
        size_t j = 0;
        while (j < sched_row.size() && !(uT[2 * j] == sT[2 * i] && uT[2 * j + 1] == sT[2 * i + 1])) j++;
        if (j == sched_row.size()) {
            uT.push_back(sT[2 * i]);
            uT.push_back(sT[2 * i + 1]);
            const int32_t rows = (S == 1 || sT[2 * i] == sT[2 * i + 1]) ? 1 : S;
            sched_row.push_back(sched_rows.empty() ? 0 : sched_row.back() + sched_rows.back());
            sched_rows.push_back(rows);
        }
        sched_of[i] = (int32_t)j;
    }
    pl->thr_rows = sched_row.empty() ? 1 : sched_row.back() + sched_rows.back();
    if ((double)pl->thr_rows * pl->thr_stride * 4.0 > 4.0 * (1ull << 30)) {
        const int32_t rows = pl->thr_rows, stride = pl->thr_stride;
        delete pl;
        return set_error(UAVQ_ETOOBIG, "plan_create: acceptance tables of %d rows x %d entries exceed 4 GiB", rows,
                         stride);
    }
    std::vector<uint32_t> thr_dev;
    try {
        thr_dev.assign((size_t)pl->thr_rows * pl->thr_stride, 0u);
    } catch (...) {
        delete pl;
        return set_error(UAVQ_ENOMEM, "plan_create: out of host memory for the acceptance tables");
    }
    for (size_t j = 0; j < sched_row.size(); j++)
        fill_schedule(uT[2 * j], uT[2 * j + 1], sched_rows[j], Dmax,
                      thr_dev.data() + (size_t)sched_row[j] * pl->thr_stride, pl->thr_stride);
    std::vector<int32_t> dcut(pl->thr_rows, 1);
    for (int32_t s = 0; s < pl->thr_rows; s++) {
        const uint32_t *row = &thr_dev[(size_t)s * pl->thr_stride];
        int32_t d = 1;
        while (d < Dmax && row[d] != 0) d++;
        dcut[s] = d;
    }
    // a frozen replica stays frozen only if no later row accepts where this one rejects
    for (size_t j = 0; pl->stop_frozen && j < sched_row.size(); j++)
        for (int32_t s = 1; s < sched_rows[j]; s++)
            if (dcut[sched_row[j] + s] > dcut[sched_row[j] + s - 1]) {
                delete pl;
                return set_error(UAVQ_EINVAL, "plan_create: UAVQ_STOP_FROZEN needs a draw cutoff that never grows");
            }

    // replica and state layout, per-instance descriptors
    pl->rep_offset.assign(n_inst + 1, 0);
    pl->state_offset.assign(n_inst + 1, 0);
    pl->inst_state_off.assign(n_inst + 1, 0);
    pl->desc.resize(n_inst);
    pl->max_m = 0;
    for (int32_t i = 0; i < n_inst; i++) {
        const uavq_qubo *qi = q[i];
        int32_t sw = qi->m * qi->row_words;
        pl->rep_offset[i + 1] = pl->rep_offset[i] + R;
        pl->state_offset[i + 1] = pl->state_offset[i] + (int64_t)R * sw;
        pl->inst_state_off[i + 1] = pl->inst_state_off[i] + sw;
        pl->max_m = std::max(pl->max_m, qi->m);
    }
    pl->total_rep = pl->rep_offset[n_inst];
    pl->total_state_words = pl->state_offset[n_inst];

    // blob: thr | dcut | desc | items | inst_state_off | per-instance data
    size_t off = 0;
    pl->thr_off = off;          off = align_up(off + thr_dev.size() * 4, 256);
    pl->dcut_off = off;         off = align_up(off + dcut.size() * 4, 256);
    pl->desc_off = off;         off = align_up(off + sizeof(InstDesc) * (size_t)std::max(n_inst, 1), 256);

    // work items: groups of waves_per_block replicas, ordered by chunk class
    // and, inside a class, by decreasing m (largest first).
    std::vector<int32_t> order(n_inst);
    for (int32_t i = 0; i < n_inst; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return q[a]->m > q[b]->m; });
    pl->items.clear();
    for (int c = 0; c <= kMaxChunks + 1; c++) pl->class_begin[c] = 0;
    for (int cls = 1; cls <= kMaxChunks; cls++) {
        int wpb = p->waves_per_block ? p->waves_per_block : default_waves_per_block(cls);
        if (cls == 1 && !p->waves_per_block) {
            // m <= 64 with more replicas than the chip has SIMDs (so not one wave per SIMD): twelve replicas share
            // a workgroup's table row and cost rows, three waves per SIMD instead of two, where their LDS fits
            // (the 256-field batch's m <= 64 kernel: 334 -> 298 ms)
            int64_t n1 = 0;
            int m1 = 0;
            for (int32_t i = 0; i < n_inst; i++)
                if (inst_class(q[i], dense) == 1) {
                    n1 += R;
                    m1 = std::max(m1, q[i]->m);
                }
            if (n1 > kSimdsPerChip && ylds_lds_bytes_for((size_t)pl->thr_stride, m1, 12) <= 160 * 1024) wpb = 12;
        }
        if (p->tune && p->tune->waves_per_block[cls] > 0) wpb = p->tune->waves_per_block[cls];
        if (cls >= 4 && wpb > kWideMaxWaves) wpb = kWideMaxWaves;   // those kernels' block limit
        if (wpb < 1 || wpb > 16) {
            delete pl;
            return set_error(UAVQ_EINVAL, "plan_create: waves per block %d out of range", wpb);
        }
        pl->waves_per_block[cls] = wpb;
        pl->class_begin[cls] = (int32_t)pl->items.size();
        for (int32_t i : order) {
            if (inst_class(q[i], dense) != cls) continue;
            for (int32_t r0 = 0; r0 < R; r0 += wpb) pl->items.push_back({i, r0, std::min(wpb, R - r0), 0});
        }
    }
    pl->waves_per_block[0] = pl->waves_per_block[1];
    pl->class_begin[kMaxChunks + 1] = (int32_t)pl->items.size();
    pl->items_off = off;        off = align_up(off + sizeof(WorkItem) * std::max<size_t>(pl->items.size(), 1), 256);
    pl->inst_state_off_off = off; off = align_up(off + 8 * (size_t)(n_inst + 1), 256);

    for (int32_t i = 0; i < n_inst; i++) {
        const uavq_qubo *qi = q[i];
        InstDesc &d = pl->desc[i];
        d.m = qi->m; d.P = qi->P; d.closed = qi->closed; d.row_words = qi->row_words;
        d.state_words = qi->m * qi->row_words;
        d.nrep = R;
        d.c0 = qi->c0;
        const size_t cb = inst_class(qi, dense) > kByteChunks ? 2 : 1;   // bytes per cost entry
        // 16-bit matrices are read from global memory, lanes past m up to 64 kMaxChunks entries beyond the end
        d.d_off = (int64_t)off;     off = align_up(off + cb * qi->D16.size() + (cb == 2 ? 2 * 64 * kMaxChunks : 0), 16);
        d.ddep_off = (int64_t)off;  off = align_up(off + cb * qi->ddep16.size(), 256);
        if (dense) {
            const size_t Np = ((size_t)qi->N + 31) / 32 * 32;
            d.J_off = (int64_t)off;     off = align_up(off + qi->J.size() * 2, 256);
            d.Jlimb_off = (int64_t)off; off = align_up(off + 2 * Np * Np, 256);
            d.b_off = (int64_t)off;     off = align_up(off + qi->b.size() * 4, 256);
        } else {
            d.J_off = -1;
            d.Jlimb_off = -1;
            d.b_off = -1;
        }
        d.rep_base = pl->rep_offset[i];
        d.state_off = pl->state_offset[i];
        d.inst_id = inst_ids[i];
        d.chunks = inst_class(qi, dense);
        d.wide = qi->wmax > 255 ? 1 : 0;
        d.wmax = qi->wmax;
        const int32_t sj = sched_of[i];
        d.sched_row = sched_row[sj];
        d.sched_step = sched_rows[sj] > 1 ? 1 : 0;
        d.tl2_a = (float)std::log2(sT[2 * i] * 0.69314718055994531);
        d.tl2_b = d.sched_step ? (float)(std::log2(sT[2 * i + 1] / sT[2 * i]) / (S - 1)) : 0.0f;
    }
    pl->blob_bytes = align_up(off, 256);
    try {
        pl->blob.assign(pl->blob_bytes, 0);
    } catch (...) {
        delete pl;
        return set_error(UAVQ_ENOMEM, "plan_create: out of host memory");
    }
    uint8_t *B = pl->blob.data();
    std::memcpy(B + pl->thr_off, thr_dev.data(), thr_dev.size() * 4);
    std::memcpy(B + pl->dcut_off, dcut.data(), dcut.size() * 4);
    if (n_inst) std::memcpy(B + pl->desc_off, pl->desc.data(), sizeof(InstDesc) * n_inst);
    if (!pl->items.empty()) std::memcpy(B + pl->items_off, pl->items.data(), sizeof(WorkItem) * pl->items.size());
    std::memcpy(B + pl->inst_state_off_off, pl->inst_state_off.data(), 8 * (size_t)(n_inst + 1));
    for (int32_t i = 0; i < n_inst; i++) {
        const uavq_qubo *qi = q[i];
        const InstDesc &d = pl->desc[i];
        if (d.chunks > kByteChunks) {
            std::memcpy(B + d.d_off, qi->D16.data(), 2 * qi->D16.size());
            std::memcpy(B + d.ddep_off, qi->ddep16.data(), 2 * qi->ddep16.size());
        } else {
            std::memcpy(B + d.d_off, qi->D.data(), qi->D.size());
            std::memcpy(B + d.ddep_off, qi->ddep.data(), qi->ddep.size());
        }
        if (dense) {
            std::memcpy(B + d.J_off, qi->J.data(), qi->J.size() * 2);
            std::memcpy(B + d.b_off, qi->b.data(), qi->b.size() * 4);
            // int8 limbs J = lo + 128 hi for the MFMA field refresh (rows padded to Np)
            const size_t N = (size_t)qi->N, Np = (N + 31) / 32 * 32;
            int8_t *lo = reinterpret_cast<int8_t *>(B + d.Jlimb_off), *hi = lo + Np * Np;
            for (size_t k = 0; k < N; k++)
                for (size_t l = 0; l < N; l++) {
                    const int v = qi->J[k * N + l];
                    lo[k * Np + l] = (int8_t)(v & 127);
                    hi[k * Np + l] = (int8_t)(v >> 7);
                }
        }
    }
    pl->e_init_off = pl->blob_bytes;
    size_t wsoff = align_up(pl->e_init_off + 8 * (size_t)std::max<int64_t>(pl->total_rep, 1), 256);
    pl->dense_xb_off = pl->dense_h_off = 0;
    if (dense) {
        size_t xb = 0, hb = 0;
        for (int32_t i = 0; i < n_inst; i++) {
            const size_t N = (size_t)q[i]->N, Np = (N + 31) / 32 * 32;
            xb = std::max(xb, (size_t)R * Np);
            hb = std::max(hb, (size_t)R * N * 4);
        }
        pl->dense_xb_off = wsoff; wsoff = align_up(wsoff + xb, 256);
        pl->dense_h_off = wsoff;  wsoff = align_up(wsoff + hb, 256);
    }
    pl->queue_off = wsoff;
    wsoff = align_up(wsoff + 4 * (kMaxChunks + 2), 256);
    pl->ws_bytes = wsoff;
    *out = pl;
    return UAVQ_OK;
}

void uavq_plan_free(uavq_plan *plan) {
    if (!plan) return;
    plan_destroy_events(plan);
    delete plan;
}

int uavq_plan_info(const uavq_plan *pl, uavq_plan_info_t *info) {
    if (!pl || !info) return set_error(UAVQ_EINVAL, "plan_info: null argument");
    info->ws_bytes = pl->ws_bytes;
    info->total_replicas = pl->total_rep;
    info->total_state_words = pl->total_state_words;
    info->n_inst = pl->n_inst;
    info->Dmax = pl->Dmax;
    return UAVQ_OK;
}

int uavq_plan_layout(const uavq_plan *pl, int64_t *rep_offset, int64_t *state_offset) {
    if (!pl) return set_error(UAVQ_EINVAL, "plan_layout: null plan");
    if (rep_offset) std::memcpy(rep_offset, pl->rep_offset.data(), 8 * (size_t)(pl->n_inst + 1));
    if (state_offset) std::memcpy(state_offset, pl->state_offset.data(), 8 * (size_t)(pl->n_inst + 1));
    return UAVQ_OK;
}

}  // extern "C"
