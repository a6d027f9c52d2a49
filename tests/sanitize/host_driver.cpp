// Drives the host half of libuavq (QUBO build, costs, export, host energy,
// decode, features, schedule, plan layout, per-instance schedules, the
// tempering ladder and their error paths) for a build
// under AddressSanitizer and UndefinedBehaviorSanitizer.  No device call is
// made; the one device-side symbol the host half references is stubbed.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "uavq.h"

extern "C" void plan_destroy_events(uavq_plan *) {}

#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                      \
        }                                                                  \
    } while (0)

static uint64_t g_rng = 0x9E3779B97F4A7C15ull;
static uint32_t rnd() {
    g_rng ^= g_rng << 13;
    g_rng ^= g_rng >> 7;
    g_rng ^= g_rng << 17;
    return (uint32_t)(g_rng >> 16);
}

struct Field {
    int rows, cols, pct, flags;
};

static int one_field(const Field &f, std::vector<uavq_qubo *> &keep) {
    std::vector<uint8_t> nf((size_t)f.rows * f.cols, 0);
    for (size_t k = 1; k < nf.size(); k++) nf[k] = (int)(rnd() % 100) < f.pct;
    uavq_grid g{};
    g.rows = f.rows;
    g.cols = f.cols;
    g.nofly = nf.data();
    g.flags = (uint32_t)f.flags;
    uavq_qubo *q = nullptr;
    const int rc = uavq_qubo_build(&g, &q);
    if (rc == UAVQ_EINVAL) return 0;   // e.g. every cell drawn no-fly
    CHECK(rc == UAVQ_OK && q);
    uavq_qubo_info_t info{};
    CHECK(uavq_qubo_info(q, &info) == UAVQ_OK);
    const int m = info.m, N = info.n_vars, W = info.row_words, SW = info.state_words;
    CHECK(N == m * m && SW == m * W);
    std::vector<int32_t> F(m), costs((size_t)(m + 1) * (m + 1)), b(N);
    CHECK(uavq_qubo_free_cells(q, F.data()) == UAVQ_OK);
    CHECK(uavq_qubo_costs(q, costs.data()) == UAVQ_OK);
    if (info.has_dense) {
        std::vector<int32_t> J((size_t)N * N);
        CHECK(uavq_qubo_export(q, b.data(), J.data()) == UAVQ_OK);
    } else {
        CHECK(uavq_qubo_export(q, b.data(), nullptr) == UAVQ_OK);
    }
    // random states and permutation states: energies, decode
    const int n = 5;
    std::vector<uint32_t> x((size_t)n * SW, 0u);
    for (int s = 0; s < n; s++) {
        uint32_t *xs = x.data() + (size_t)s * SW;
        if (s < 2) {
            for (int t = 0; t < m; t++)
                for (int c = 0; c < m; c++)
                    if (rnd() & 1u) xs[t * W + (c >> 5)] |= 1u << (c & 31);
        } else {
            std::vector<int> perm(m);
            for (int i = 0; i < m; i++) perm[i] = i;
            for (int i = m - 1; i > 0; i--) std::swap(perm[i], perm[rnd() % (uint32_t)(i + 1)]);
            for (int t = 0; t < m; t++) xs[t * W + (perm[t] >> 5)] |= 1u << (perm[t] & 31);
        }
    }
    std::vector<int64_t> E(n);
    CHECK(uavq_energy_eval(q, x.data(), n, E.data()) == UAVQ_OK);
    std::vector<int32_t> path(m + 2);
    int64_t cost = 0;
    for (int s = 2; s < n; s++) {
        CHECK(uavq_decode_path(q, x.data() + (size_t)s * SW, path.data(), &cost) == UAVQ_OK);
        CHECK(cost == E[s]);
    }
    std::vector<float> X((size_t)m * 16);
    CHECK(uavq_mlp_features(q, X.data()) == UAVQ_OK);
    keep.push_back(q);
    return 0;
}

int main() {
    const Field fields[] = {{1, 2, 0, 0},  {3, 3, 0, UAVQ_DENSE}, {3, 4, 0, UAVQ_OPEN_PATH | UAVQ_DENSE},
                            {5, 5, 20, UAVQ_DENSE}, {2, 9, 30, UAVQ_OPEN_PATH}, {8, 8, 10, 0},
                            {12, 12, 0, 0}, {16, 16, 5, UAVQ_OPEN_PATH}, {19, 19, 3, 0}, {4, 4, 100, 0}};
    std::vector<uavq_qubo *> qs;
    for (const Field &f : fields)
        if (one_field(f, qs)) return 1;

    // error paths
    uavq_qubo *bad = nullptr;
    uavq_grid g{};
    g.rows = 1;
    g.cols = 1;
    CHECK(uavq_qubo_build(&g, &bad) == UAVQ_EINVAL && bad == nullptr);
    CHECK(std::strlen(uavq_last_error()) > 0);
    g.rows = 30;
    g.cols = 30;
    g.cost_scale = 10000;   // w_max = round(10^4 * 29 sqrt 2) does not fit 16 bits
    CHECK(uavq_qubo_build(&g, &bad) == UAVQ_ETOOBIG && bad == nullptr);
    g.cost_scale = 0;
    CHECK(uavq_qubo_build(nullptr, &bad) == UAVQ_EINVAL);
    CHECK(uavq_decode_path(qs[1], nullptr, nullptr, nullptr) == UAVQ_EINVAL);

    // schedule: query, then the table
    int32_t Dmax = 0;
    CHECK(uavq_schedule(200.0, 0.5, 300, &Dmax, nullptr) == UAVQ_OK && Dmax > 0);
    std::vector<uint32_t> thr((size_t)300 * (Dmax + 1));
    CHECK(uavq_schedule(200.0, 0.5, 300, &Dmax, thr.data()) == UAVQ_OK);
    CHECK(uavq_schedule(1.0, 2.0, 10, &Dmax, nullptr) == UAVQ_EINVAL);

    // plans over every instance (all chunk classes), their layout and errors
    std::vector<uint32_t> ids(qs.size());
    for (size_t i = 0; i < qs.size(); i++) ids[i] = (uint32_t)(100 + i);
    uavq_anneal_params p{};
    p.replicas = 37;
    p.sweeps = 20;
    p.T0 = 50.0;
    p.T1 = 0.5;
    p.seed = 3;
    for (int wpb : {0, 1, 3, 16}) {
        p.waves_per_block = wpb;
        uavq_plan *pl = nullptr;
        CHECK(uavq_plan_create(qs.data(), (int32_t)qs.size(), ids.data(), &p, &pl) == UAVQ_OK && pl);
        uavq_plan_info_t pi{};
        CHECK(uavq_plan_info(pl, &pi) == UAVQ_OK && pi.total_replicas == 37 * (int64_t)qs.size());
        std::vector<int64_t> ro(qs.size() + 1), so(qs.size() + 1);
        CHECK(uavq_plan_layout(pl, ro.data(), so.data()) == UAVQ_OK);
        CHECK(ro.back() == pi.total_replicas && so.back() == pi.total_state_words);
        uavq_plan_free(pl);
    }
    // per-instance schedules: cooling, constant and repeated ones share rows
    {
        std::vector<double> iT(2 * qs.size());
        for (size_t i = 0; i < qs.size(); i++) {
            iT[2 * i] = (i % 3 == 0) ? 80.0 : (i % 3 == 1 ? 25.0 : 120.0);
            iT[2 * i + 1] = (i % 3 == 1) ? 25.0 : 0.5;
        }
        p.waves_per_block = 0;
        p.inst_T = iT.data();
        for (uint32_t fl : {0u, (uint32_t)UAVQ_STOP_FROZEN}) {
            p.flags = fl;
            uavq_plan *pl = nullptr;
            CHECK(uavq_plan_create(qs.data(), (int32_t)qs.size(), ids.data(), &p, &pl) == UAVQ_OK && pl);
            uavq_plan_info_t pi{};
            CHECK(uavq_plan_info(pl, &pi) == UAVQ_OK && pi.Dmax > 0);
            uavq_plan_free(pl);
        }
        p.flags = 0;
        iT[1] = 90.0;   // T1 > T0
        uavq_plan *pl = nullptr;
        CHECK(uavq_plan_create(qs.data(), (int32_t)qs.size(), ids.data(), &p, &pl) == UAVQ_EINVAL && !pl);
        p.inst_T = nullptr;
    }

    // tempering ladder: query, fill, errors
    {
        const int K = 9;
        double T[K];
        int32_t DX[K], mx = 0;
        CHECK(uavq_pt_ladder(150.0, 1.0, K, T, DX, &mx, nullptr, 0) == UAVQ_OK && mx > 1);
        std::vector<uint32_t> xt((size_t)(K - 1) * (mx + 1));
        CHECK(uavq_pt_ladder(150.0, 1.0, K, T, DX, &mx, xt.data(), mx + 1) == UAVQ_OK);
        CHECK(uavq_pt_ladder(150.0, 1.0, K, T, DX, &mx, xt.data(), mx) == UAVQ_EINVAL);
        CHECK(uavq_pt_ladder(150.0, 150.0, K, T, DX, &mx, nullptr, 0) == UAVQ_EINVAL);
        CHECK(uavq_pt_ladder(150.0, 1.0, 0, T, DX, &mx, nullptr, 0) == UAVQ_EINVAL);
        CHECK(uavq_pt_ladder(150.0, 1.0, 1, T, nullptr, &mx, nullptr, 0) == UAVQ_OK && T[0] == 150.0);
    }

    uavq_plan *pl = nullptr;
    p.replicas = 0;
    CHECK(uavq_plan_create(qs.data(), (int32_t)qs.size(), ids.data(), &p, &pl) == UAVQ_EINVAL && !pl);
    p.replicas = 4;
    p.flags = UAVQ_KERNEL_DENSE;   // instances without the dense J
    CHECK(uavq_plan_create(qs.data(), (int32_t)qs.size(), ids.data(), &p, &pl) == UAVQ_EINVAL && !pl);

    for (uavq_qubo *q : qs) uavq_qubo_free(q);
    std::printf("host driver: %zu instances, clean\n", qs.size());
    return 0;
}
