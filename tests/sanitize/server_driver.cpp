// Drives the request server's host logic (fmg_server.hip built for the host
// against the HIP stand-in) from several client threads at once: requests of
// uneven size, some larger than max_batch (served as parts), to four fake
// models, with and without graph replay, with every model admitted and with a
// budget for two of them and idle models swapped in and out.  Every served
// row must equal the fake prediction of its query, each request must be
// counted once, and no prediction may run on a model that is not resident.
// Prints "server runs clean" and exits 0 when all of that holds.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "fastmuygps.h"
#include "fmg_internal.h"

int fake_violations();

namespace {

struct FakeModelSpec {
    int d, ell, prec;
    int64_t n;
    uint64_t bytes;
};

template <typename T>
bool check_rows(const std::vector<T> &Z, const std::vector<T> &out, int B, const FakeModelSpec &s) {
    for (int q = 0; q < B; ++q) {
        T sum = 0;
        for (int j = 0; j < s.d; ++j) sum += Z[(size_t)q * s.d + j];
        for (int c = 0; c < s.ell; ++c)
            if (out[(size_t)q * s.ell + c] != (T)(c + 1) * sum + (T)s.n) return false;
    }
    return true;
}

template <typename T>
bool one_request(fmg_server *S, int32_t id, const FakeModelSpec &s, int B, std::mt19937_64 &rng,
                 int64_t *queries) {
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    std::vector<T> Z((size_t)B * s.d), out((size_t)B * s.ell, (T)-7);
    for (auto &z : Z) z = (T)u(rng);
    fmg_ticket t = nullptr;
    if (fastmuygps_server_submit(S, id, Z.data(), B, out.data(), 0, &t) != FMG_OK) return false;
    double ms = -1.0;
    if (fastmuygps_server_wait(t, &ms) != FMG_OK || ms < 0.0) return false;
    *queries += B;
    return check_rows(Z, out, B, s);
}

bool run(bool graphs, bool swap) {
    const FakeModelSpec specs[4] = {{8, 3, FMG_PREC_MIXED, 6000, 300u << 20},
                                    {5, 2, FMG_PREC_FP32, 4000, 200u << 20},
                                    {3, 1, FMG_PREC_FP64, 1500, 250u << 20},
                                    {16, 2, FMG_PREC_FP32, 9000, 350u << 20}};
    fmg_server_opts opts{};
    opts.slots = 3;
    opts.max_batch = 512;
    opts.use_graphs = graphs ? 1 : 0;
    opts.swap_idle = swap ? 1 : 0;
    uint64_t budget = 0;  // the whole (fake) device
    if (swap) {
        fmg_server *probe = nullptr;
        if (fastmuygps_server_create(0, &opts, &probe) != FMG_OK) return false;
        fmg_server_stats st{};
        fastmuygps_server_stats(probe, &st);
        fastmuygps_server_destroy(probe);
        budget = st.hbm_resident + (700u << 20);  // room for two of the four models
    }
    fmg_server *S = nullptr;
    if (fastmuygps_server_create(budget, &opts, &S) != FMG_OK) return false;
    std::vector<fmg_model *> models;
    std::vector<int32_t> ids;
    for (const FakeModelSpec &s : specs) {
        fmg_model *M = new fmg_model();
        M->n = s.n;
        M->d = s.d;
        M->ell = s.ell;
        M->k = 16;
        M->prec = s.prec;
        M->bytes = s.bytes;
        M->resident = true;
        int32_t id = -1;
        const fmg_status st = fastmuygps_server_add_model(S, M, &id);
        if (st != FMG_OK && st != FMG_E_BUSY) return false;
        models.push_back(M);
        ids.push_back(id);
    }
    std::atomic<int64_t> submitted{0}, served_q{0};
    std::atomic<bool> ok{true};
    std::vector<std::thread> clients;
    for (int c = 0; c < 4; ++c) {
        clients.emplace_back([&, c] {
            std::mt19937_64 rng(1000 + 17 * c + (graphs ? 1 : 0) + (swap ? 2 : 0));
            std::uniform_int_distribution<int> pick(0, 3);
            std::uniform_real_distribution<double> lb(0.0, std::log(1300.0));
            int64_t q = 0;
            for (int r = 0; r < 60 && ok; ++r) {
                const int mi = pick(rng);
                const int B = 1 + (int)std::exp(lb(rng));
                const bool good = specs[mi].prec == FMG_PREC_FP64
                                      ? one_request<double>(S, ids[mi], specs[mi], B, rng, &q)
                                      : one_request<float>(S, ids[mi], specs[mi], B, rng, &q);
                if (!good) {
                    fprintf(stderr, "request failed or wrong (model %d, B %d): %s\n", mi, B,
                            fastmuygps_last_error());
                    ok = false;
                }
                submitted += 1;
            }
            served_q += q;
        });
    }
    for (auto &t : clients) t.join();
    fmg_server_stats st{};
    fastmuygps_server_stats(S, &st);
    fastmuygps_server_destroy(S);
    for (fmg_model *M : models) delete M;
    if (!ok) return false;
    if (st.requests != submitted.load() || st.queries != served_q.load()) {
        fprintf(stderr, "statistics: %lld requests, %lld queries; expected %lld, %lld\n",
                (long long)st.requests, (long long)st.queries, (long long)submitted.load(),
                (long long)served_q.load());
        return false;
    }
    if (swap && st.swaps == 0) {
        fprintf(stderr, "no swap under a budget for two of four models\n");
        return false;
    }
    if (!(st.p50_ms <= st.p99_ms && st.p99_ms <= st.max_ms)) return false;
    printf("graphs %d swap %d: %lld requests, %lld queries, %lld batches, %lld swaps\n", graphs,
           swap, (long long)st.requests, (long long)st.queries, (long long)st.batches,
           (long long)st.swaps);
    return true;
}

}  // namespace

int main() {
    for (int graphs = 0; graphs < 2; ++graphs)
        for (int swap = 0; swap < 2; ++swap)
            if (!run(graphs != 0, swap != 0)) {
                fprintf(stderr, "FAILED (graphs %d, swap %d)\n", graphs, swap);
                return 1;
            }
    if (fake_violations() != 0) {
        fprintf(stderr, "%d predictions on a model that was not resident\n", fake_violations());
        return 1;
    }
    printf("server runs clean\n");
    return 0;
}
