// Coefficient precompute in FP32 (FP32 and MIXED precision modes):
// Algorithm 2, training loop; Section 3, coefficient equation:
//     K_ab = phi(||x_{N(i)_a} - x_{N(i)_b}||)  (a != b),   K_aa = amp + sigma^2,
//     C[i] = K^{-1} Y(X_{N(i)}).
// One wavefront per training point i; lane a owns row a (k <= KMAX <= 64).
//   1. The k neighbour rows, centred on x_i and rounded to FP32, are staged in
//      LDS.  Their Gram matrix G = Xc Xc^T comes from FP32 MFMA
//      (v_mfma_f32_16x16x4f32) and D_ab = G_aa + G_bb - 2 G_ab (centring
//      keeps the cancellation small).  G is transposed through LDS in halves
//      of 32 columns so that each lane receives its row.
//   2. Right-looking Cholesky in registers, with the forward substitution
//      folded into the same loop; the register window slides one column per
//      step so the loop stays rolled and the code fits the instruction cache.
//   3. Back substitution; solved values are broadcast with v_readlane.
//   4. MIXED only: one refinement step.  The rows, centred on x_i, are exact
//      in FP64; their Gram matrix on FP64 MFMA (v_mfma_f64_16x16x4f64) gives
//      FP64 distances and kernel values, a second FP64 MFMA product gives
//      r = Y_N - (K64 + sigma^2 I) C, and C += solve(L, r) with the FP32
//      factor.
// L is kept in LDS as a packed lower triangle; LDS per wavefront is about
// 15 KB (FP32) or 35 KB (MIXED, d = 40, k = 50, ell = 10).
// A non-positive or non-finite pivot marks the point: its C row is NaN and
// its status is 1.
#include "fmg_device.h"
#include "fmg_kernels.h"

namespace fmg {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Row stride (floats) of the staged coordinates: d rounded up to the MFMA
// k-step of 4, plus one (odd, so that lanes reading different rows spread
// over the LDS banks).
__host__ __device__ __forceinline__ int xs_stride(int d) { return ((d + 3) / 4) * 4 + 1; }

// Row stride (doubles) of the FP64 rows used by the refinement: d rounded up
// to the MFMA k-step, plus one.
__host__ __device__ __forceinline__ int x64_stride(int d) { return ((d + 3) / 4) * 4 + 1; }

// LDS layout (bytes), one wavefront per block.
struct PcLayout {
    int xs_ld;      // floats per staged FP32 row
    int x64_ld;     // doubles per staged FP64 row (refinement)
    int g_ld;       // floats per Gram column (column-major, 32 columns at a time)
    int off_r1;     // staged rows, then Gram halves, then FP64 rows
    int off_l;      // Cholesky factor, packed by rows (row a at a(a+1)/2), 1/L_jj on
                    // the diagonal
    int off_bc;     // broadcast buffer [64][ELLMAX] floats
    int off_nrm;    // [64] floats
    int off_nrm64;  // [64] doubles
    int off_kc;     // refinement: K64 C, [64][ELLMAX] doubles
    int bytes;
};

__host__ __device__ __forceinline__ int imax3(int x, int y, int z) {
    const int m = x > y ? x : y;
    return m > z ? m : z;
}

__host__ __device__ __forceinline__ PcLayout pc_layout(int k, int d, int kmax, int ellmax,
                                                       bool refine) {
    PcLayout L;
    L.xs_ld = xs_stride(d);
    L.x64_ld = x64_stride(d);
    L.g_ld = kmax + 4;
    const int r1 = imax3(k * L.xs_ld * 4, 32 * L.g_ld * 4, refine ? k * L.x64_ld * 8 : 0);
    L.off_r1 = 0;
    L.off_l = (r1 + 15) & ~15;
    L.off_bc = (L.off_l + (k * (k + 1) / 2) * 4 + 15) & ~15;
    L.off_nrm = L.off_bc + 64 * ellmax * 4;
    L.off_nrm64 = L.off_nrm + 64 * 4;
    L.off_kc = L.off_nrm64 + 64 * 8;
    L.bytes = L.off_kc + (refine ? 64 * ellmax * 8 : 0);
    return L;
}

// Stage rows N(i)_b (b < k) centred on x_i (difference in FP64, rounded to
// FP32) into xs[b][0..d), zero padded to xs_ld; lane b loads row b.
__device__ __forceinline__ void stage_rows(const float *__restrict__ X, int d, int k, int64_t i,
                                           int64_t p, float *__restrict__ xs, int ld, int a) {
    const float *__restrict__ xi = X + i * d;
    const float *__restrict__ xp = X + p * d;
    if (a < k) {
        float *row = xs + a * ld;
        for (int c = 0; c < d; ++c) row[c] = (float)((double)xp[c] - (double)xi[c]);
        for (int c = d; c < ld; ++c) row[c] = 0.0f;
    }
}

// Triangular solves with L in LDS as a packed lower triangle, row a at
// a(a+1)/2, whose diagonal slots hold 1/L_jj.  Lane a holds row a of the
// ELLMAX right-hand sides; the value solved at step j is read from lane j
// (v_readlane), so no LDS round trip or barrier sits on the dependency chain.
template <int ELLMAX>
__device__ __forceinline__ void solve_forward(const float *__restrict__ Lm, int k, int ell, int a,
                                              float (&y)[ELLMAX]) {
    const int arow = a * (a + 1) / 2;
    for (int j = 0; j < k; ++j) {
        const float rjj = Lm[j * (j + 1) / 2 + j];
        const float laj = (a > j && a < k) ? Lm[arow + j] : 0.0f;
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) {
            if (c >= ell) break;
            const float zj = readlane_f32(y[c], j) * rjj;
            y[c] = (a == j) ? zj : fmaf(-laj, zj, y[c]);
        }
    }
}

template <int ELLMAX>
__device__ __forceinline__ void solve_backward(const float *__restrict__ Lm, int k, int ell, int a,
                                               float (&y)[ELLMAX]) {
    for (int j = k - 1; j >= 0; --j) {
        const int jrow = j * (j + 1) / 2;
        const float rjj = Lm[jrow + j];
        const float lja = (a < j) ? Lm[jrow + a] : 0.0f;
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) {
            if (c >= ell) break;
            const float xj = readlane_f32(y[c], j) * rjj;
            y[c] = (a == j) ? xj : fmaf(-lja, xj, y[c]);
        }
    }
}

template <int KMAX, int ELLMAX, bool REFINE>
__global__ __launch_bounds__(64) void precompute32_kernel(PrecomputeArgs P) {
    extern __shared__ __align__(16) char smem[];
    const int64_t i = blockIdx.x;
    if (i >= P.n) return;
    const int a = threadIdx.x;
    const int k = P.k, d = P.d, ell = P.ell;
    const PcLayout L = pc_layout(k, d, KMAX, ELLMAX, REFINE);
    float *xs = (float *)(smem + L.off_r1);
    float *G = (float *)(smem + L.off_r1);
    double *x64 = (double *)(smem + L.off_r1);
    float *Lm = (float *)(smem + L.off_l);
    float *bc = (float *)(smem + L.off_bc);
    float *nrm = (float *)(smem + L.off_nrm);
    double *nrm64 = (double *)(smem + L.off_nrm64);
    const float *__restrict__ X = (const float *)P.X;
    const float *__restrict__ Y = (const float *)P.Y;

    const int64_t p = (a < k) ? (int64_t)P.N[i * k + a] : i;
    float y[ELLMAX];
#pragma unroll
    for (int c = 0; c < ELLMAX; ++c) y[c] = (a < k && c < ell) ? Y[p * ell + c] : 0.0f;

    // 1. Gram matrix of the centred rows on FP32 MFMA.
    stage_rows(X, d, k, i, p, xs, L.xs_ld, a);
    lds_sync();
    constexpr int NT = KMAX / 16;
    f32x4 acc[NT][NT];
#pragma unroll
    for (int r = 0; r < NT; ++r)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int fr = a & 15, fk = a >> 4;
    for (int s = 0; s < d; s += 4) {
        float f[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int row = t * 16 + fr;
            f[t] = (row < k) ? xs[row * L.xs_ld + s + fk] : 0.0f;
        }
#pragma unroll
        for (int r = 0; r < NT; ++r)
#pragma unroll
            for (int c = 0; c < NT; ++c)
                acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[r], f[c], acc[r][c], 0, 0, 0);
    }
    // Transpose through LDS, 32 columns at a time: tile (r, c), lane l holds
    // rows r*16 + 4*(l/16) + 0..3 of column c*16 + l%16; lane a then reads
    // column a, which is its row (G is symmetric).
    float K[KMAX];
#pragma unroll
    for (int h = 0; h < NT; h += 2) {
        lds_sync();  // previous readers (fragments or the other half) are done
#pragma unroll
        for (int r = 0; r < NT; ++r)
#pragma unroll
            for (int c = h; c < h + 2 && c < NT; ++c)
                *(f32x4 *)(G + ((c - h) * 16 + fr) * L.g_ld + r * 16 + 4 * fk) = acc[r][c];
        lds_sync();
        const bool mine = a >= h * 16 && a < (h + 2) * 16 && a < KMAX;
        const float *col = G + (a - h * 16) * L.g_ld;
#pragma unroll
        for (int b = 0; b < KMAX; b += 4) {
            if (mine) {
                const f32x4 v = *(const f32x4 *)(col + b);
                K[b] = v[0];
                K[b + 1] = v[1];
                K[b + 2] = v[2];
                K[b + 3] = v[3];
            }
        }
        if (mine) nrm[a] = col[a];
    }
    if (a >= KMAX) {
#pragma unroll
        for (int b = 0; b < KMAX; ++b) K[b] = 0.0f;
        nrm[a] = 0.0f;
    }
    lds_sync();
    const float na = nrm[a];
    const PhiForm<float> pf = phi_form<float>(P.kc, P.inv_rho, P.amp);
    const float diag = (float)(P.amp + P.noise);
#pragma unroll
    for (int b = 0; b < KMAX; ++b) {
        float v = 0.0f;
        if (b < k) {
            const float D = fmaxf(na + nrm[b] - 2.0f * K[b], 0.0f);
            v = (a == b) ? diag : phi_eval(pf, D);
        }
        K[b] = (a < k) ? v : ((a == b) ? 1.0f : 0.0f);
    }

    // 2. Right-looking Cholesky with the forward solve folded in.  Register
    // K[b] of lane a holds entry (a, j + b) at step j: after each step the
    // window moves one column, so the loop over j stays rolled and the code
    // small.  Column j of L is broadcast through LDS, stored shifted so that
    // entry b of the broadcast pairs with register b; the tail of the buffer
    // is zero.  L is kept packed by rows with 1/L_jj on the diagonal.
    bool bad = false;
    const int arow = a * (a + 1) / 2;
    for (int j = 0; j < k; ++j) {
        float piv = readlane_f32(K[0], j);
        if (!(piv > 0.0f) || !isfinite(piv)) {
            bad = true;
            piv = 1.0f;
        }
        const float ljj = sqrtf(piv);
        const float rjj = 1.0f / ljj;
        const float lj = (a == j) ? ljj : ((a > j && a < k) ? K[0] * rjj : 0.0f);
        if (a == j) Lm[arow + j] = rjj;
        if (a > j && a < k) Lm[arow + j] = lj;
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) {
            if (c >= ell) break;
            const float zj = readlane_f32(y[c], j) * rjj;
            y[c] = (a == j) ? zj : fmaf(-lj, zj, y[c]);  // lj = 0 above row j
        }
        bc[(a - j - 1) & 63] = (a > j) ? lj : 0.0f;
        lds_sync();
#pragma unroll
        for (int b = 0; b + 1 < KMAX; ++b) K[b] = fmaf(-lj, bc[b], K[b + 1]);
        K[KMAX - 1] = 0.0f;
        lds_sync();
    }

    // 3. Back substitution for all right-hand sides.
    solve_backward<ELLMAX>(Lm, k, ell, a, y);

    if constexpr (REFINE) {
        // 4. One refinement step, r = Y_N - (K64 + sigma^2 I) C, in FP64 on
        // FP64 MFMA.  The centred rows are exact in FP64 (a difference of two
        // FP32 values); their Gram matrix gives D_ab = |c_a|^2 + |c_b|^2 -
        // 2 <c_a, c_b>, and K64 C is a second FP64 MFMA product.  Both are
        // taken one 16-column tile of K at a time: in the 16x16x4 FP64 layout
        // lane l holds entries (4g + l/16, l%16), g = 0..3, of a tile, which
        // (K being symmetric) is exactly the A operand of the product for
        // the transposed tile, so K never leaves registers.
        double *KC = (double *)(smem + L.off_kc);  // [64][ELLMAX]
        const int ld = L.x64_ld, d4 = (d + 3) & ~3;
        double n64 = 0.0;
        if (a < k) {
            const float *__restrict__ xi = X + i * d;
            const float *__restrict__ xa = X + p * d;
            double *row = x64 + a * ld;
            for (int c = 0; c < d; ++c) {
                const double v = (double)xa[c] - (double)xi[c];
                row[c] = v;
                n64 = fma(v, v, n64);
            }
            for (int c = d; c < d4; ++c) row[c] = 0.0;
        }
        nrm64[a] = n64;
        float *cb = bc;  // [64][ELLMAX] current coefficients, zero past k / ell
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) cb[a * ELLMAX + c] = (a < k && c < ell) ? y[c] : 0.0f;
        lds_sync();
        const double diag64 = P.amp + P.noise;
        const PhiForm<double> pf64 = phi_form<double>(P.kc, P.inv_rho, P.amp);
        const int nt = (k + 15) >> 4;
        for (int ct = 0; ct < nt; ++ct) {
            f64x4 g[NT];
#pragma unroll
            for (int r = 0; r < NT; ++r) g[r] = f64x4{0.0, 0.0, 0.0, 0.0};
            const int rb = ct * 16 + fr;
            for (int s = 0; s < d4; s += 4) {
                const double fb = (rb < k) ? x64[rb * ld + s + fk] : 0.0;
#pragma unroll
                for (int r = 0; r < NT; ++r) {
                    const int row = r * 16 + fr;
                    const double fa = (row < k) ? x64[row * ld + s + fk] : 0.0;
                    g[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, fb, g[r], 0, 0, 0);
                }
            }
            const double ncol = nrm64[rb];
            f64x4 acc64 = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < NT; ++r) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = r * 16 + 4 * q + fk;
                    double kab = 0.0;
                    if (row < k && rb < k) {
                        if (row == rb) {
                            kab = diag64;
                        } else {
                            double D = nrm64[row] + ncol - 2.0 * g[r][q];
                            D = D > 0.0 ? D : 0.0;
                            kab = phi_eval(pf64, D);
                        }
                    }
                    const double cv = (fr < ell) ? (double)cb[row * ELLMAX + fr] : 0.0;
                    acc64 = __builtin_amdgcn_mfma_f64_16x16x4f64(kab, cv, acc64, 0, 0, 0);
                }
            }
            if (fr < ell) {
#pragma unroll
                for (int q = 0; q < 4; ++q) KC[(ct * 16 + 4 * q + fk) * ELLMAX + fr] = acc64[q];
            }
        }
        lds_sync();
        float dl[ELLMAX];
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c)
            dl[c] = (a < k && c < ell) ? (float)((double)Y[p * ell + c] - KC[a * ELLMAX + c])
                                       : 0.0f;
        solve_forward<ELLMAX>(Lm, k, ell, a, dl);
        solve_backward<ELLMAX>(Lm, k, ell, a, dl);
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) y[c] += dl[c];
    }

    if (a < k) {
        float *__restrict__ C = (float *)P.C + (i * k + a) * ell;
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c)
            if (c < ell) C[c] = bad ? NAN : y[c];
    }
    if (a == 0) P.status[i] = bad ? 1 : 0;
}

template <int KMAX, int ELLMAX, bool REFINE>
hipError_t launch_pc32(const PrecomputeArgs &a, hipStream_t s) {
    const PcLayout L = pc_layout(a.k, a.d, KMAX, ELLMAX, REFINE);
    hipLaunchKernelGGL((precompute32_kernel<KMAX, ELLMAX, REFINE>), dim3((unsigned)a.n), dim3(64),
                       (size_t)L.bytes, s, a);
    return hipGetLastError();
}

template <bool REFINE>
hipError_t launch_pc32_k(const PrecomputeArgs &a, hipStream_t s) {
    if (a.ell > 16 || a.d > 64) return hipErrorInvalidValue;
    if (a.k <= 32) {
        if (a.ell <= 1) return launch_pc32<32, 1, REFINE>(a, s);
        return launch_pc32<32, 16, REFINE>(a, s);
    }
    if (a.ell <= 1) return launch_pc32<64, 1, REFINE>(a, s);
    return launch_pc32<64, 16, REFINE>(a, s);
}

}  // namespace

hipError_t launch_precompute32(bool refine, const PrecomputeArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    return refine ? launch_pc32_k<true>(a, s) : launch_pc32_k<false>(a, s);
}

}  // namespace fmg
