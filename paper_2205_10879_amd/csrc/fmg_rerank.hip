// FP64 re-rank of screened candidates, with an exactness certificate.
//
// For each query row one wavefront recomputes the distance of every screened
// candidate exactly as the ranking defines it (FP64, coordinate order, every
// operation rounded on its own), keeps the k smallest (distance, index) keys
// and then proves that no unscreened training point could have entered them:
//
//   every non-candidate p has screened value S'_p >= T' (the c-th kept value
//   of its split), and the MFMA result differs from the exact
//   ||x~_p - z~||^2 - ||z~||^2 by at most A_q, so
//       ||x~_p - z~|| >= sqrt(T' + ||z~||^2 - A_q);
//   the rounding radii bound the distance to the unrounded points:
//       ||x_p - z|| >= ||x~_p - z~|| - e_max - e_q.
//   If that lower bound exceeds sqrt(D_k), the exact k-th distance, with a
//   relative margin for FP64 rounding, no non-candidate can be among the k
//   nearest, and ties are impossible.
//
// Rows that fail are listed for an exact rescan.
#include "fmg_device.h"
#include "fmg_kernels.h"

namespace fmg {

namespace {

constexpr int RR_WAVES = 4;

__global__ __launch_bounds__(256) void rerank_kernel(RerankArgs a) {
#pragma clang fp contract(off)
    extern __shared__ double zsh[];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int64_t w = (int64_t)blockIdx.x * RR_WAVES + wave;
    if (w >= a.m) return;
    const int64_t q = a.order ? (int64_t)a.order[w] : w;  // query (output row)
    double *z = zsh + wave * a.d;
    const float *__restrict__ X = (const float *)a.X;
    const float *__restrict__ Zc = (const float *)a.Zc;
    for (int c = lane; c < a.d; c += 64) z[c] = (double)Zc[q * a.d + c];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");

    const int64_t cq = w;  // its row of the screen's output
    const int total = a.splits * a.c;
    const double nz = a.nzq[q];
    const double A = a.acc_coef * (2.01 * a.nx_max + nz) + 1.0e-6 * a.nx_max;
    // Lower bound on the exact distance of any point whose screened value is
    // at least S (the certificate's bound).
    auto lower_bound = [&](double S) {
        const double lb2 = S + nz - A;
        return (lb2 > 0.0 ? sqrt(lb2) : 0.0) - a.e_max - a.eq[q];
    };
    XKey list = xkey_empty();
    for (int base = 0; base < total; base += 64) {
        if (base > 0 && a.splits == 1) {
            // One sorted list: once the bound of the next screened value
            // exceeds the current k-th exact distance, no later candidate
            // can enter the k nearest.
            const uint64_t nk = a.cand[cq * a.c + base];
            if (nk == SKEY_EMPTY) break;
            const XKey cur = readlane_x(list, a.k - 1);
            if (cur.p != 0xffffffffu &&
                lower_bound((double)skey_val(nk)) > sqrt(dkey_inv(cur.d)) * (1.0 + 1.0e-12) + 1.0e-300)
                break;
        }
        const int slot = base + lane;
        XKey key = xkey_empty();
        if (slot < total) {
            const int sp = slot / a.c, r = slot % a.c;
            const uint64_t sk = a.cand[((int64_t)sp * a.m + cq) * a.c + r];
            if (sk != SKEY_EMPTY) {
                uint32_t p = skey_idx(sk);
                if (a.cand_idx && p < (uint64_t)a.n_idx) p = a.cand_idx[p];
                const float *__restrict__ xp = X + (int64_t)p * a.d;
                double s = 0.0;
                for (int c = 0; c < a.d; ++c) {
                    const double t = z[c] - (double)xp[c];
                    const double t2 = t * t;
                    s = s + t2;
                }
                key = XKey{dkey(s), p};
            }
        }
        list = wave_merge_x(list, key);
    }

    // certificate
    double tmin = INFINITY;
    for (int sp = 0; sp < a.splits; ++sp) {
        const double t = (double)a.tq[(int64_t)sp * a.m + cq];
        tmin = t < tmin ? t : tmin;
    }
    const XKey kk = readlane_x(list, a.k - 1);
    bool ok;
    if (!(tmin < INFINITY)) {
        ok = kk.p != 0xffffffffu;  // every training point was a candidate
    } else if (kk.p == 0xffffffffu) {
        ok = false;
    } else {
        const double dk = sqrt(dkey_inv(kk.d));
        ok = lower_bound(tmin) > dk * (1.0 + 1.0e-12) + 1.0e-300;
    }

    int32_t *o = a.out + q * (int64_t)a.out_stride;
    if (a.self_first) {
        if (lane == 0) o[0] = (int32_t)q;
        if (lane < a.k) o[1 + lane] = (int32_t)list.p;  // a.k <= 64 others
    } else if (lane < a.k) {
        o[lane] = (int32_t)list.p;
    }
    if (!ok && lane == 0) {
        const int pos = atomicAdd(a.fb_count, 1);
        a.fb_list[pos] = (int32_t)q;
    }
}

}  // namespace

hipError_t launch_rerank(const RerankArgs &a, hipStream_t s) {
    if (a.m <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.m + RR_WAVES - 1) / RR_WAVES);
    const size_t shm = sizeof(double) * RR_WAVES * (size_t)a.d;
    hipLaunchKernelGGL(rerank_kernel, dim3(blocks), dim3(256), shm, s, a);
    return hipGetLastError();
}

}  // namespace fmg
