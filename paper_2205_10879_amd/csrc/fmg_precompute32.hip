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
//   2. Cholesky in the form K = U D U^T (U unit lower triangular, D the
//      pivots), right-looking, with the forward substitution U w = y folded
//      into the same loop.  Register K[b] of lane a holds entry (a, j + b) at
//      step j; the window slides one column per step, and shrinks in steps
//      of 16 columns as the trailing matrix does, so the loops stay rolled.
//   3. v = D^{-1} w, then back substitution U^T x = v.  Every solve step is
//      one v_readlane and one FMA per right-hand side: the unit diagonal
//      leaves nothing to scale inside the loop.
//   4. MIXED only: one refinement step.  The rows, centred on x_i, are exact
//      in FP64 (each operand is formed as (double) x_b - (double) x_i from the
//      raw FP32 rows staged in LDS); their Gram matrix on FP64 MFMA
//      (v_mfma_f64_16x16x4f64) gives FP64 distances and kernel values, a
//      second FP64 MFMA product gives r = Y_N - (K64 + sigma^2 I) C, and
//      C += solve(U D U^T, r).
// U is kept in LDS packed by rows.  LDS per wavefront is about 14 KB (FP32)
// or 17 KB (MIXED) for d = 40, k = 50, ell = 10, so eight wavefronts fit a CU.
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

// Rows are staged a chunk of coordinates at a time (the Gram products
// accumulate in registers across chunks, so LDS holds one chunk): d rounded
// up to the MFMA k-step of 4 when that is at most 24, else chunks of 20.
// The row stride is the chunk plus one (odd, so that lanes reading different
// rows spread over the LDS banks).
__host__ __device__ __forceinline__ int stage_chunk(int d) {
    const int d4 = (d + 3) & ~3;
    return d4 <= 24 ? d4 : 20;
}
__host__ __device__ __forceinline__ int xs_stride(int d) { return stage_chunk(d) + 1; }

// LDS layout (bytes), one wavefront per block.
struct PcLayout {
    int xs_ld;      // floats per staged FP32 row
    int g_ld;       // floats per Gram column (column-major, 32 columns at a time)
    int off_r1;     // staged rows, then Gram halves, then the refinement's raw rows
    int off_l;      // U, strictly lower part packed by rows (row a at a(a-1)/2)
    int off_bc;     // column broadcast [64] floats; with refinement the
                    // coefficients [64][ELLMAX] floats
    int off_nrm;    // [64] floats
    int off_nrm64;  // [64] doubles
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
    L.g_ld = kmax + 4;
    // One region serves in turn: a chunk of the staged rows, the Gram
    // matrix's transpose 16 columns at a time, a chunk of the refinement's
    // raw rows and centre, one transposed FP64 tile, the residual.
    const int r64 = refine ? imax3(k * L.xs_ld * 4 + 32 * 4, 256 * 8, 64 * ellmax * 4) : 0;
    const int r1 = imax3(k * L.xs_ld * 4, 16 * L.g_ld * 4, r64);
    L.off_r1 = 0;
    L.off_l = (r1 + 15) & ~15;
    L.off_bc = (L.off_l + (k * (k - 1) / 2) * 4 + 15) & ~15;
    // two buffers of 64 float4 for the blocked Cholesky steps
    L.off_nrm = L.off_bc + (refine && ellmax >= 8 ? 64 * ellmax * 4 : 2048);
    L.off_nrm64 = L.off_nrm + 64 * 4;
    L.bytes = L.off_nrm64 + 64 * 8;
    return L;
}

// Stage coordinates c0 .. c0 + cw - 1 (cw a multiple of 4) of rows N(i)_b
// (b < k) centred on x_i (difference in FP64, rounded to FP32) into
// xs[b][0..cw), zero past d; lane b loads row b, four coordinates per load
// when rows are 16-byte aligned.  xi is the centre (the training point
// itself, or a query for per-query solves).
__device__ __forceinline__ void stage_rows(const float *__restrict__ X, int d, int k,
                                           const float *__restrict__ xi, int64_t p,
                                           float *__restrict__ xs, int ld, int a, int c0,
                                           int cw) {
    const float *__restrict__ xp = X + p * d;
    if (a >= k) return;
    float *row = xs + a * ld - c0;
    if ((d & 3) == 0 && (((uintptr_t)X | (uintptr_t)xi) & 15) == 0) {
        for (int c = c0; c < c0 + cw; c += 4) {
            const float4 u = *(const float4 *)(xp + c);
            const float4 v = *(const float4 *)(xi + c);
            row[c] = (float)((double)u.x - (double)v.x);
            row[c + 1] = (float)((double)u.y - (double)v.y);
            row[c + 2] = (float)((double)u.z - (double)v.z);
            row[c + 3] = (float)((double)u.w - (double)v.w);
        }
    } else {
        for (int c = c0; c < c0 + cw; ++c)
            row[c] = c < d ? (float)((double)xp[c] - (double)xi[c]) : 0.0f;
    }
}

// The refinement's rows: coordinates c0 .. c0 + cw - 1 of rows N(i)_b, raw
// FP32, staged in xr[b][0..cw) (zero past d) and of the centre in xc[0..cw),
// so that every FP64 MFMA operand is formed as the exact difference
// (double) x_b - (double) x_i when it is loaded.  Adds the chunk's part of
// |x_a - x_i|^2 (FP64, coordinates in order) to n64 for lane a's row.
__device__ __forceinline__ void stage_rows_raw(const float *__restrict__ X, int d, int k,
                                               const float *__restrict__ xi, int64_t p,
                                               float *__restrict__ xr, int ld,
                                               float *__restrict__ xc, int a, int c0, int cw,
                                               double &n64) {
    if (a < cw) xc[a] = c0 + a < d ? xi[c0 + a] : 0.0f;
    const float *__restrict__ xp = X + p * d;
    if (a >= k) return;
    float *row = xr + a * ld - c0;
    if ((d & 3) == 0 && (((uintptr_t)X | (uintptr_t)xi) & 15) == 0) {
        for (int c = c0; c < c0 + cw; c += 4) {
            const float4 u = *(const float4 *)(xp + c);
            const float4 v = *(const float4 *)(xi + c);
            const double e0 = (double)u.x - (double)v.x, e1 = (double)u.y - (double)v.y;
            const double e2 = (double)u.z - (double)v.z, e3 = (double)u.w - (double)v.w;
            row[c] = u.x;
            row[c + 1] = u.y;
            row[c + 2] = u.z;
            row[c + 3] = u.w;
            n64 = fma(e0, e0, n64);
            n64 = fma(e1, e1, n64);
            n64 = fma(e2, e2, n64);
            n64 = fma(e3, e3, n64);
        }
    } else {
        for (int c = c0; c < c0 + cw; ++c) {
            if (c < d) {
                const double e = (double)xp[c] - (double)xi[c];
                row[c] = xp[c];
                n64 = fma(e, e, n64);
            } else {
                row[c] = 0.0f;
            }
        }
    }
}

// exp(x) for x <= 0 in FP32: x log2(e) = n + f with n an integer and
// |f| <= 1/2 + 2^-24, the product carried in two parts (its rounded value
// and, from FMAs, its rounding error plus the tail of log2(e)), so that f is
// accurate to a few units of 2^-48; then 2^f from the hardware base-2
// exponential (about 1 ulp on that range) scaled by 2^n.  Results below the
// smallest normal float may round differently from a correctly rounded exp;
// the kernel values they stand for are negligible next to the diagonal.
__device__ __forceinline__ float exp_nonpos32(float x) {
    // th must be the rounded product: contracting it into th - n would count
    // its rounding error twice (once there, once in tl)
#pragma clang fp contract(off)
    const float kL2e = 1.44269502f;          // log2(e) rounded to FP32
    const float kL2eLo = 1.92596299e-8f;     // log2(e) - kL2e
    const float th = x * kL2e;
    const float tl = fmaf(x, kL2eLo, fmaf(x, kL2e, -th));
    const float n = rintf(th);
    const float f = (th - n) + tl;
    return ldexpf(__builtin_amdgcn_exp2f(f), (int)n);
}

// exp(x) for x <= 0 in FP64: additive range reduction x = n ln2 + r,
// |r| <= ln2/2 (Cody and Waite, with the product n ln2 taken in two FMAs),
// then the Taylor series of exp(r) to degree 12 (truncation below 1e-15
// relative) and a final scaling by 2^n.  Underflows to 0 below about -745.
__device__ __forceinline__ double exp_nonpos64(double x) {
    const double kLn2 = 0.6931471805599453;       // ln 2 rounded to FP64
    const double kLn2Lo = 2.3190468138462996e-17;  // ln 2 - kLn2
    const double n = rint(x * 1.4426950408889634);  // x / ln 2
    double r = fma(-n, kLn2, x);
    r = fma(-n, kLn2Lo, r);
    double q = 1.0 / 479001600.0;  // 1/12!
    q = fma(q, r, 1.0 / 39916800.0);
    q = fma(q, r, 1.0 / 3628800.0);
    q = fma(q, r, 1.0 / 362880.0);
    q = fma(q, r, 1.0 / 40320.0);
    q = fma(q, r, 1.0 / 5040.0);
    q = fma(q, r, 1.0 / 720.0);
    q = fma(q, r, 1.0 / 120.0);
    q = fma(q, r, 1.0 / 24.0);
    q = fma(q, r, 1.0 / 6.0);
    q = fma(q, r, 0.5);
    q = fma(q, r, 1.0);
    q = fma(q, r, 1.0);
    const int e = n < -1100.0 ? -1100 : (int)n;
    return ldexp(q, e);
}

// phi from its argument t (the distance for the Matern forms, the squared
// distance for RBF: the caller takes the square root under a uniform branch,
// so that RBF runs no square roots), in FP32 and in FP64 through
// exp_nonpos64 for the refinement residual.
__device__ __forceinline__ float phi_arg32(const PhiForm<float> &f, float t) {
    const float s = f.scale * t;
    return f.amp * fmaf(fmaf(f.c2, s, f.c1), s, 1.0f) * exp_nonpos32(-s);
}

__device__ __forceinline__ double phi_arg64(const PhiForm<double> &f, double t) {
    const double s = f.scale * t;
    return f.amp * fma(fma(f.c2, s, f.c1), s, 1.0) * exp_nonpos64(-s);
}

// Solves with U (unit lower, strictly lower part packed by rows in LDS, row
// a at a(a-1)/2).  Lane a holds row a of the ELLMAX right-hand sides; the
// value final at step j is read from lane j with v_readlane.  Columns past
// ell hold zeros and stay zero, so every loop over them has a fixed trip
// count and unrolls (no dynamic register indexing).
template <int ELLMAX>
__device__ __forceinline__ void solve_unit_forward(const float *__restrict__ U, int k, int ell,
                                                   int a, float (&y)[ELLMAX]) {
    const int arow = a * (a - 1) / 2;
    for (int j = 0; j < k - 1; ++j) {
        const float u = (a > j && a < k) ? U[arow + j] : 0.0f;
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) y[c] = fmaf(-u, readlane_f32(y[c], j), y[c]);
    }
}

template <int ELLMAX>
__device__ __forceinline__ void solve_unit_backward(const float *__restrict__ U, int k, int ell,
                                                    int a, float (&y)[ELLMAX]) {
    for (int j = k - 1; j > 0; --j) {
        const float u = (a < j) ? U[j * (j - 1) / 2 + a] : 0.0f;
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) y[c] = fmaf(-u, readlane_f32(y[c], j), y[c]);
    }
}

// A pivot is usable when it is positive and finite: its bits, as an
// unsigned integer, lie in [1, 0x7f7fffff] (a test on the scalar unit, the
// pivot being uniform).
__device__ __forceinline__ bool pivot_ok(float piv) {
    return __builtin_bit_cast(uint32_t, piv) - 1u < 0x7f7fffffu;
}

// 1/p for a usable pivot: the hardware reciprocal (about 1 ulp) refined by
// one Newton step whose residual 1 - p r comes from an FMA, which leaves it
// within an ulp of the quotient (the division sequence that correct
// rounding takes is seven times as long and runs once per step).
__device__ __forceinline__ float recip_pivot(float p) {
    const float r = __builtin_amdgcn_rcpf(p);
    return fmaf(fmaf(-p, r, 1.0f), r, r);
}

// Four Cholesky steps j .. j + 3 at once (register window of W columns);
// the first NY right-hand sides in y take the forward solve along.
// The panel, columns j .. j + 3 held in K[0..3], is factored with values
// read across lanes (the entry of row j + t2 in column j + t comes from lane
// j + t2); every lane then publishes its four panel entries in LDS, and the
// trailing columns take the four rank-one updates in step order, so each
// entry sees exactly the operations of four single steps, with one LDS
// round trip instead of four.  bc holds two buffers of 64 float4, used
// alternately.
template <int KMAX, int ELLMAX, int NY, int W>
__device__ __forceinline__ void chol_block4(float (&K)[KMAX], float (&y)[ELLMAX], int j, int k,
                                            int a, float *__restrict__ U,
                                            float *__restrict__ bc, float &dinv, bool &bad) {
    const int arow = a * (a - 1) / 2;
    float u[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float piv = readlane_f32(K[t], j + t);
        if (!pivot_ok(piv)) {
            bad = true;
            piv = 1.0f;
        }
        const float rp = recip_pivot(piv);
        const bool below = a > j + t && a < k;
        u[t] = below ? K[t] * rp : 0.0f;
        if (a == j + t) dinv = rp;
        if (below) U[arow + j + t] = u[t];
#pragma unroll
        for (int c = 0; c < NY; ++c) y[c] = fmaf(-u[t], readlane_f32(y[c], j + t), y[c]);
#pragma unroll
        for (int t2 = t + 1; t2 < 4; ++t2)
            K[t2] = fmaf(-u[t], readlane_f32(K[t], j + t2), K[t2]);
    }
    // Entry b of the buffer: the panel row of lane j + 4 + b; positions past
    // the last row are zero.
    float4 *buf = (float4 *)bc + ((j >> 2) & 1) * 64;
    buf[(a - j - 4) & 63] =
        (a >= j + 4) ? make_float4(K[0], K[1], K[2], K[3]) : make_float4(0.f, 0.f, 0.f, 0.f);
    lds_sync();
#pragma unroll
    for (int b = 4; b < W; ++b) {
        const float4 v = buf[b - 4];
        float x = fmaf(-u[0], v.x, K[b]);
        x = fmaf(-u[1], v.y, x);
        x = fmaf(-u[2], v.z, x);
        K[b - 4] = fmaf(-u[3], v.w, x);
    }
#pragma unroll
    for (int b = W - 4; b < W; ++b) K[b] = 0.0f;
}

// Eight Cholesky steps j .. j + 7 at once, as chol_block4 with a panel of
// eight columns (K[0..7]): each entry sees exactly the operations of eight
// single steps in step order, with one LDS round trip and one register shift
// per eight steps.  bc holds one buffer of 64 rows of two float4 (the space
// of chol_block4's two buffers), so it is written only after the previous
// block's readers are done.
template <int KMAX, int ELLMAX, int NY, int W>
__device__ __forceinline__ void chol_block8(float (&K)[KMAX], float (&y)[ELLMAX], int j, int k,
                                            int a, float *__restrict__ U,
                                            float *__restrict__ bc, float &dinv, bool &bad) {
    const int arow = a * (a - 1) / 2;
    float u[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        float piv = readlane_f32(K[t], j + t);
        if (!pivot_ok(piv)) {
            bad = true;
            piv = 1.0f;
        }
        const float rp = recip_pivot(piv);
        const bool below = a > j + t && a < k;
        u[t] = below ? K[t] * rp : 0.0f;
        if (a == j + t) dinv = rp;
        if (below) U[arow + j + t] = u[t];
#pragma unroll
        for (int c = 0; c < NY; ++c) y[c] = fmaf(-u[t], readlane_f32(y[c], j + t), y[c]);
#pragma unroll
        for (int t2 = t + 1; t2 < 8; ++t2)
            K[t2] = fmaf(-u[t], readlane_f32(K[t], j + t2), K[t2]);
    }
    // Entry b of the buffer (two float4): the panel row of lane j + 8 + b;
    // positions past the last row are zero.
    float4 *buf = (float4 *)bc;
    const int slot = 2 * ((a - j - 8) & 63);
    const bool pub = a >= j + 8;
    lds_sync();  // the previous block's readers are done
    buf[slot] = pub ? make_float4(K[0], K[1], K[2], K[3]) : make_float4(0.f, 0.f, 0.f, 0.f);
    buf[slot + 1] = pub ? make_float4(K[4], K[5], K[6], K[7]) : make_float4(0.f, 0.f, 0.f, 0.f);
    lds_sync();
#pragma unroll
    for (int b = 8; b < W; ++b) {
        const float4 v0 = buf[2 * (b - 8)];
        const float4 v1 = buf[2 * (b - 8) + 1];
        float x = fmaf(-u[0], v0.x, K[b]);
        x = fmaf(-u[1], v0.y, x);
        x = fmaf(-u[2], v0.z, x);
        x = fmaf(-u[3], v0.w, x);
        x = fmaf(-u[4], v1.x, x);
        x = fmaf(-u[5], v1.y, x);
        x = fmaf(-u[6], v1.z, x);
        K[b - 8] = fmaf(-u[7], v1.w, x);
    }
#pragma unroll
    for (int b = W - 8; b < W; ++b) K[b] = 0.0f;
}

// Cholesky steps j in [j0, j1) with a register window of W columns: blocks
// of eight steps, then of four, then single steps.
template <int KMAX, int ELLMAX, int NY, int W>
__device__ __forceinline__ void chol_steps(float (&K)[KMAX], float (&y)[ELLMAX], int j0, int j1,
                                           int k, int ell, int a, float *__restrict__ U,
                                           float *__restrict__ bc, float &dinv, bool &bad) {
    const int arow = a * (a - 1) / 2;
    int j = j0;
    if constexpr (W >= 16) {
        if (j + 8 <= j1) {
            for (; j + 8 <= j1; j += 8)
                chol_block8<KMAX, ELLMAX, NY, W>(K, y, j, k, a, U, bc, dinv, bad);
            lds_sync();  // the last block's readers are done before bc is written again
        }
    }
    if (j + 4 <= j1) {
        for (; j + 4 <= j1; j += 4) chol_block4<KMAX, ELLMAX, NY, W>(K, y, j, k, a, U, bc, dinv, bad);
        lds_sync();  // the last block's readers are done before bc is written again
    }
    for (; j < j1; ++j) {
        float piv = readlane_f32(K[0], j);
        if (!pivot_ok(piv)) {
            bad = true;
            piv = 1.0f;
        }
        const float rp = recip_pivot(piv);
        const bool below = a > j && a < k;
        const float u = below ? K[0] * rp : 0.0f;
        if (a == j) dinv = rp;
        if (below) U[arow + j] = u;
#pragma unroll
        for (int c = 0; c < NY; ++c) y[c] = fmaf(-u, readlane_f32(y[c], j), y[c]);
        // Entry b of the broadcast is column j of the trailing matrix at row
        // j + 1 + b; the positions past the last row are zero.
        bc[(a - j - 1) & 63] = (a > j) ? K[0] : 0.0f;
        lds_sync();
#pragma unroll
        for (int b = 0; b + 1 < W; ++b) K[b] = fmaf(-u, bc[b], K[b + 1]);
        K[W - 1] = 0.0f;
        lds_sync();
    }
}

// Blocked solves on FP32 MFMA (the mixed path).  The right-hand sides are
// held in the 16x16x4 output layout: per 16-row block J a lane holds rows
// 16 J + 4 (l / 16) + q (q < 4) of column l % 16 (columns past ell are zero).
// A product M W of a 16x16 block M and such a block W takes four k-steps, the
// k-index of step q on lane l being 4 (l / 16) + q, so that the B operand of
// step q is the lane's own element q and the A operand is
// M[l % 16][4 (l / 16) + q].  The unit diagonal blocks of U are replaced in
// LDS by their inverses (same packed places, unit diagonal implicit), so
// that a block solve is one product:
//   U w = r:      w_J = inv(U_JJ) (r_J - sum_{I<J} U_JI w_I),   J ascending;
//   U^T x = v:    x_J = inv(U_JJ)^T (v_J - sum_{I>J} U_IJ^T x_I), J descending.
// Entries of rows at or past k are zero (their right-hand sides are zero).

// The A operands of each 16x16 block product are read first, four at a time
// (branch free: addresses clamped to a valid entry and the value selected),
// so that the reads are in flight together and the four MFMAs follow
// without a wait each.
template <int NT>
__device__ __forceinline__ void mfma_forward(const float *__restrict__ U, int k, int fr, int fk,
                                             f32x4 (&r)[NT]) {
    // opaque copies: the addresses are formed afresh in every solve instead
    // of being shared (and kept live) across the kernel
    asm volatile("" : "+v"(fr), "+v"(fk));
#pragma unroll
    for (int J = 0; J < NT; ++J) {
        __builtin_amdgcn_sched_barrier(0);  // one block's reads at a time (register pressure)
        // row 16 J + fr of U: entries (row, 16 I + 4 fk + q), I < J, then
        // the inverted diagonal block's (row, 16 J + 4 fk + q)
        const int row = 16 * J + fr;
        const bool rv = row < k;
        const int rb = row * (row - 1) / 2 + 4 * fk;
        f32x4 acc = r[J];
#pragma unroll
        for (int I = 0; I < J; ++I) {
            float aop[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float v = U[rv ? rb + 16 * I + q : 0];
                aop[q] = rv ? -v : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (16 * I + q < k)  // else every k-index of the step is a zero row
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[q], r[I][q], acc, 0, 0, 0);
        }
        float aop[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = 4 * fk + q;  // column within the block
            const bool lower = rv && c < fr;
            const float v = U[lower ? rb + 16 * J + q : 0];
            aop[q] = lower ? v : ((rv && c == fr) ? 1.0f : 0.0f);
        }
        f32x4 w = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (16 * J + q < k) w = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[q], acc[q], w, 0, 0, 0);
        r[J] = w;
    }
}

template <int NT>
__device__ __forceinline__ void mfma_backward(const float *__restrict__ U, int k, int fr, int fk,
                                              f32x4 (&r)[NT]) {
    asm volatile("" : "+v"(fr), "+v"(fk));  // as in mfma_forward
#pragma unroll
    for (int J = NT - 1; J >= 0; --J) {
        __builtin_amdgcn_sched_barrier(0);  // one block's reads at a time (register pressure)
        // column 16 J + fr of U: entries (16 I + 4 fk + q, col), I > J, then
        // the inverted diagonal block's (16 J + 4 fk + q, col)
        f32x4 acc = r[J];
#pragma unroll
        for (int I = J + 1; I < NT; ++I) {
            float aop[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * I + 4 * fk + q;
                const bool rv = row < k;
                const float v = U[rv ? row * (row - 1) / 2 + 16 * J + fr : 0];
                aop[q] = rv ? -v : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (16 * I + q < k)  // else every k-index of the step is a zero row
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[q], r[I][q], acc, 0, 0, 0);
        }
        float aop[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = 4 * fk + q;  // row within the block
            const int row = 16 * J + c;
            const bool lower = row < k && fr < c;
            const float v = U[lower ? row * (row - 1) / 2 + 16 * J + fr : 0];
            aop[q] = lower ? v : ((row < k && c == fr) ? 1.0f : 0.0f);
        }
        f32x4 x = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (16 * J + q < k) x = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[q], acc[q], x, 0, 0, 0);
        r[J] = x;
    }
}

// The inverses of U's unit lower diagonal blocks, in place: lane a = 16 J + r
// holds row r of block J and forward-substitutes the identity, row m of its
// block coming from lane 16 J + m by a DPP row broadcast (row_newbcast).
template <int M>
__device__ __forceinline__ float bcast16(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 0x150 + M, 0xf, 0xf, false));
}
template <int M>
__device__ __forceinline__ void inv_step(float (&X)[16], const float (&um)[16]) {
#pragma unroll
    for (int c = 0; c <= M; ++c) X[c] = fmaf(-um[M], bcast16<M>(X[c]), X[c]);
}
template <int M>
__device__ __forceinline__ void inv_steps(float (&X)[16], const float (&um)[16]) {
    if constexpr (M < 15) {
        inv_step<M>(X, um);
        inv_steps<M + 1>(X, um);
    }
}
__device__ __forceinline__ void invert_diag_blocks(float *__restrict__ U, int k, int a) {
    const int J = a >> 4, r = a & 15;
    const int arow = a * (a - 1) / 2;
    float um[16], X[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        um[m] = (m < r && a < k) ? U[arow + 16 * J + m] : 0.0f;
        X[m] = (m == r) ? 1.0f : 0.0f;
    }
    inv_steps<0>(X, um);
    lds_sync();  // every lane has read its block row before any is overwritten
#pragma unroll
    for (int c = 0; c < 15; ++c)
        if (c < r && a < k) U[arow + 16 * J + c] = X[c];
    lds_sync();
}

template <int KMAX, int ELLMAX, bool REFINE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void precompute32_kernel(PrecomputeArgs P) {
    extern __shared__ __align__(16) char smem[];
    if ((int64_t)blockIdx.x >= P.n) return;
    const int64_t i = P.order ? (int64_t)P.order[blockIdx.x] : (int64_t)blockIdx.x;
    const int a = threadIdx.x;
    const int k = P.k, d = P.d, ell = P.ell;
    const PcLayout L = pc_layout(k, d, KMAX, ELLMAX, REFINE);
    float *xs = (float *)(smem + L.off_r1);
    float *G = (float *)(smem + L.off_r1);
    float *U = (float *)(smem + L.off_l);
    float *bc = (float *)(smem + L.off_bc);
    float *nrm = (float *)(smem + L.off_nrm);
    double *nrm64 = (double *)(smem + L.off_nrm64);
    const float *__restrict__ X = (const float *)P.X;
    const float *__restrict__ Y = (const float *)P.Y;

    const int64_t p = (a < k) ? (int64_t)P.N[i * k + a] : (int64_t)P.N[i * k];
    const float *__restrict__ xi = (P.Ctr ? (const float *)P.Ctr : X) + i * d;
    float y[ELLMAX];
#pragma unroll
    for (int c = 0; c < ELLMAX; ++c) y[c] = (a < k && c < ell) ? Y[p * ell + c] : 0.0f;

    // 1. Gram matrix of the centred rows on FP32 MFMA, a chunk of
    // coordinates at a time.
    constexpr int NT = KMAX / 16;
    f32x4 acc[NT][NT];
#pragma unroll
    for (int r = 0; r < NT; ++r)
#pragma unroll
        for (int c = 0; c < NT; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int fr = a & 15, fk = a >> 4;
    const int d4 = (d + 3) & ~3, cwmax = stage_chunk(d);
    for (int c0 = 0; c0 < d4; c0 += cwmax) {
        const int cw = d4 - c0 < cwmax ? d4 - c0 : cwmax;
        lds_sync();  // the previous chunk's readers are done
        stage_rows(X, d, k, xi, p, xs, L.xs_ld, a, c0, cw);
        lds_sync();
        for (int s = 0; s < cw; s += 4) {
            float f[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int row = t * 16 + fr;
                f[t] = (row < k) ? xs[row * L.xs_ld + s + fk] : 0.0f;
            }
            // tiles on and below the diagonal only: G is symmetric
#pragma unroll
            for (int r = 0; r < NT; ++r)
#pragma unroll
                for (int c = 0; c <= r; ++c)
                    acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[r], f[c], acc[r][c], 0, 0, 0);
        }
    }
    // Transpose through LDS, 16 columns at a time: tile (r, c), lane l holds
    // rows r*16 + 4*(l/16) + 0..3 of column c*16 + l%16; lane a then reads
    // column a, which is its row.  A tile above the diagonal is the transpose
    // of tile (c, r): its lane l holds column c*16 + 4*(l/16) + 0..3 at row
    // r*16 + l%16 (the same products summed in the same order, so G stays
    // exactly symmetric).
    float K[KMAX];
#pragma unroll
    for (int h = 0; h < NT; ++h) {
        lds_sync();  // previous readers (fragments or the previous columns) are done
#pragma unroll
        for (int r = 0; r < NT; ++r)
#pragma unroll
            for (int c = h; c < h + 1; ++c) {
                if (r >= c) {
                    *(f32x4 *)(G + ((c - h) * 16 + fr) * L.g_ld + r * 16 + 4 * fk) = acc[r][c];
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        G[((c - h) * 16 + 4 * fk + q) * L.g_ld + r * 16 + fr] = acc[c][r][q];
                }
            }
        lds_sync();
        const bool mine = a >= h * 16 && a < (h + 1) * 16 && a < KMAX;
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
    for (int b = 0; b < KMAX; ++b) K[b] = fmaxf(na + nrm[b] - 2.0f * K[b], 0.0f);
    if (pf.root) {
#pragma unroll
        for (int b = 0; b < KMAX; ++b) K[b] = sqrtf(K[b]);
    }
#pragma unroll
    for (int b = 0; b < KMAX; ++b) {
        float v = 0.0f;
        if (b < k) v = (a == b) ? diag : phi_arg32(pf, K[b]);
        K[b] = (a < k) ? v : ((a == b) ? 1.0f : 0.0f);
    }

    // 2. K = U D U^T with U w = y folded in (plain FP32; the mixed path
    // solves on MFMA afterwards); the window narrows by 16 columns whenever
    // the trailing matrix fits a narrower one.
    constexpr int NY = REFINE ? 0 : ELLMAX;
    bool bad = false;
    float dinv = 0.0f;
    // The factorisation and the first solves are one serial chain: at a
    // raised issue priority the SIMD serves it before the other wavefronts'
    // Gram and refinement work, which has more independent instructions to
    // fill the gaps (26.6 -> 26.2 ms at 1M points, mixed precision; the
    // priority is dropped again for the refinement, and the plain FP32 path
    // keeps it to its end, the back substitution being part of the chain).
    __builtin_amdgcn_s_setprio(3);
    {
        int j = 0;
        if constexpr (KMAX > 48) {
            const int e = k - 48 > 0 ? k - 48 : 0;
            chol_steps<KMAX, ELLMAX, NY, 64>(K, y, j, e, k, ell, a, U, bc, dinv, bad);
            j = e;
        }
        if constexpr (KMAX > 32) {
            const int e = k - 32 > j ? k - 32 : j;
            chol_steps<KMAX, ELLMAX, NY, 48>(K, y, j, e, k, ell, a, U, bc, dinv, bad);
            j = e;
        }
        {
            const int e = k - 16 > j ? k - 16 : j;
            chol_steps<KMAX, ELLMAX, NY, 32>(K, y, j, e, k, ell, a, U, bc, dinv, bad);
            j = e;
        }
        chol_steps<KMAX, ELLMAX, NY, 16>(K, y, j, k, k, ell, a, U, bc, dinv, bad);
    }

    // 3. v = D^{-1} w, then U^T x = v.
    if constexpr (!REFINE) {
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) y[c] *= dinv;
        solve_unit_backward<ELLMAX>(U, k, ell, a, y);
        if (a < k) {
            float *__restrict__ C = (float *)P.C + (i * k + a) * ell;
#pragma unroll
            for (int c = 0; c < ELLMAX; ++c)
                if (c < ell) C[c] = bad ? NAN : y[c];
        }
        if (a == 0) P.status[i] = bad ? 1 : 0;
    } else {
        // Mixed: the solves go through FP32 MFMA in 16-row blocks (see
        // mfma_forward / mfma_backward), with the diagonal blocks of U
        // inverted in place first.
        const int fr = a & 15, fk = a >> 4;
        invert_diag_blocks(U, k, a);
        float *dv = nrm;  // [64] D^{-1} (the norms are dead)
        dv[a] = a < k ? dinv : 0.0f;
        // Y in the MFMA layout, the neighbour of a row taken from its lane
        f32x4 Xs[NT];
#pragma unroll
        for (int J = 0; J < NT; ++J)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = 16 * J + 4 * fk + q;
                const int prow = __shfl((int)p, row);
                Xs[J][q] = (row < k && fr < ell) ? Y[(int64_t)prow * ell + fr] : 0.0f;
            }
        lds_sync();
        mfma_forward<NT>(U, k, fr, fk, Xs);
#pragma unroll
        for (int J = 0; J < NT; ++J)
#pragma unroll
            for (int q = 0; q < 4; ++q) Xs[J][q] *= dv[16 * J + 4 * fk + q];
        mfma_backward<NT>(U, k, fr, fk, Xs);
        __builtin_amdgcn_s_setprio(0);

        // 4. One refinement step, r = Y_N - (K64 + sigma^2 I) C, in FP64 on
        // FP64 MFMA.  The centred rows are exact in FP64 (a difference of two
        // FP32 values); their Gram matrix gives D_ab = |c_a|^2 + |c_b|^2 -
        // 2 <c_a, c_b>, and K64 C is a second FP64 MFMA product.  Both are
        // taken one 16-column tile of K at a time: in the 16x16x4 FP64 layout
        // lane l holds entries (4g + l/16, l%16), g = 0..3, of a tile, which
        // (K being symmetric) is exactly the A operand of the product for
        // the transposed tile, so K never leaves registers.
        const int ld = L.xs_ld;
        float *cb = bc;  // [64][ELLMAX] current coefficients, zero past k / ell
        if (fr < ELLMAX) {
#pragma unroll
            for (int J = 0; J < NT; ++J)
#pragma unroll
                for (int q = 0; q < 4; ++q) cb[(16 * J + 4 * fk + q) * ELLMAX + fr] = Xs[J][q];
        }
        float *xr = (float *)(smem + L.off_r1);
        float *xc = xr + k * ld;
        const double diag64 = P.amp + P.noise;
        const PhiForm<double> pf64 = phi_form<double>(P.kc, P.inv_rho, P.amp);
        // The Gram matrix is symmetric: only its tiles on and below the
        // diagonal, (r, c) with r >= c, go through the MFMA (each operand
        // formed from the raw rows serves every tile of its k-step), and
        // kernel values are evaluated once per such tile.  A tile above the
        // diagonal is the transpose of its mirror: the same products summed in
        // the same order and the two norms added the other way round, so its
        // entries are exactly the mirror's, read back transposed through LDS.
        constexpr int NL = NT * (NT + 1) / 2;
        f64x4 G[NL];  // tile (r, c), r >= c, at r (r + 1) / 2 + c
#pragma unroll
        for (int t = 0; t < NL; ++t) G[t] = f64x4{0.0, 0.0, 0.0, 0.0};
        double n64 = 0.0;  // |x_a - x_i|^2 in FP64, summed over the chunks in order
        for (int c0 = 0; c0 < d4; c0 += cwmax) {
            const int cw = d4 - c0 < cwmax ? d4 - c0 : cwmax;
            lds_sync();  // the previous chunk's readers are done
            stage_rows_raw(X, d, k, xi, p, xr, ld, xc, a, c0, cw, n64);
            lds_sync();
            for (int s = 0; s < cw; s += 4) {
                double f[NT];
                const double cc = (double)xc[s + fk];
#pragma unroll
                for (int r = 0; r < NT; ++r) {
                    const int row = r * 16 + fr;
                    f[r] = (row < k) ? (double)xr[row * ld + s + fk] - cc : 0.0;
                }
#pragma unroll
                for (int r = 0; r < NT; ++r)
#pragma unroll
                    for (int c = 0; c <= r; ++c)
                        if (r * 16 < k)
                            G[r * (r + 1) / 2 + c] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                f[r], f[c], G[r * (r + 1) / 2 + c], 0, 0, 0);
            }
        }
        nrm64[a] = n64;
        lds_sync();
        // kernel values of the lower tiles, in place: lane l holds entries
        // (r * 16 + 4 q + l / 16, c * 16 + l % 16)
#pragma unroll
        for (int r = 0; r < NT; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) {
                f64x4 &T = G[r * (r + 1) / 2 + c];
                const int col = c * 16 + fr;
                const double ncol = nrm64[col];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (r * 16 + 4 * q >= k) {  // rows past k (uniform skip)
                        T[q] = 0.0;
                        continue;
                    }
                    const int row = r * 16 + 4 * q + fk;
                    double D = nrm64[row] + ncol - 2.0 * T[q];
                    D = D > 0.0 ? D : 0.0;
                    if (pf64.root) D = sqrt(D);
                    double kab = 0.0;
                    if (row < k && col < k) kab = (row == col) ? diag64 : phi_arg64(pf64, D);
                    T[q] = kab;
                }
            }
        double *tr = (double *)(smem + L.off_r1);  // one transposed tile [16 x 16]
        f64x4 R[NT];
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
            f64x4 acc64 = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int r = 0; r < NT; ++r) {
                // tile (r, ct) with r < ct: the transpose of the lower tile
                // (ct, r), through LDS one tile at a time
                if (r < ct) {
                    lds_sync();  // the raw rows, or the previous transpose, are read
#pragma unroll
                    for (int q = 0; q < 4; ++q) tr[(4 * q + fk) * 16 + fr] = G[ct * (ct + 1) / 2 + r][q];
                    lds_sync();
                }
                if (ct * 16 < k) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        // k-step (r, q) covers rows r*16 + 4q .. + 3 of C:
                        // past k they are zero (uniform skip)
                        if (r * 16 + 4 * q >= k) continue;
                        const int row = r * 16 + 4 * q + fk;
                        const double kab =
                            (r >= ct) ? G[r * (r + 1) / 2 + ct][q] : tr[fr * 16 + 4 * q + fk];
                        const double cv = (fr < ell) ? (double)cb[row * ELLMAX + fr] : 0.0;
                        acc64 = __builtin_amdgcn_mfma_f64_16x16x4f64(kab, cv, acc64, 0, 0, 0);
                    }
                }
            }
            R[ct] = acc64;
        }
        // The residual, in FP64 and rounded to FP32, in the FP64 output
        // layout (rows 16 ct + 4 q + l / 16; the neighbour of a row taken from
        // that row's lane), moves through LDS to the FP32 layout of the
        // solves (rows 16 J + 4 (l / 16) + q).
        lds_sync();  // the last transpose is read; its space takes the residual
        float *res = (float *)(smem + L.off_r1);  // [64][ELLMAX]
#pragma unroll
        for (int ct = 0; ct < NT; ++ct)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = ct * 16 + 4 * q + fk;
                const int prow = __shfl((int)p, row);
                if (fr < ELLMAX)
                    res[row * ELLMAX + fr] =
                        (row < k && fr < ell)
                            ? (float)((double)Y[(int64_t)prow * ell + fr] - R[ct][q])
                            : 0.0f;
            }
        lds_sync();
        f32x4 Rs[NT];
#pragma unroll
        for (int J = 0; J < NT; ++J)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                Rs[J][q] = fr < ELLMAX ? res[(16 * J + 4 * fk + q) * ELLMAX + fr] : 0.0f;
        mfma_forward<NT>(U, k, fr, fk, Rs);
#pragma unroll
        for (int J = 0; J < NT; ++J)
#pragma unroll
            for (int q = 0; q < 4; ++q) Rs[J][q] *= dv[16 * J + 4 * fk + q];
        mfma_backward<NT>(U, k, fr, fk, Rs);
        if (fr < ell) {
#pragma unroll
            for (int J = 0; J < NT; ++J)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = 16 * J + 4 * fk + q;
                    if (row < k) {
                        const float cnew = cb[row * ELLMAX + fr] + Rs[J][q];
                        ((float *)P.C)[(i * k + row) * ell + fr] = bad ? NAN : cnew;
                    }
                }
        }
        if (a == 0) P.status[i] = bad ? 1 : 0;
    }
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
    // Right-hand-side columns are processed up to ELLMAX (zeros past ell).
    if (a.k <= 32) {
        if (a.ell <= 1) return launch_pc32<32, 1, REFINE>(a, s);
        if (a.ell <= 4) return launch_pc32<32, 4, REFINE>(a, s);
        if (a.ell <= 8) return launch_pc32<32, 8, REFINE>(a, s);
        if (a.ell <= 12) return launch_pc32<32, 12, REFINE>(a, s);
        return launch_pc32<32, 16, REFINE>(a, s);
    }
    if (a.ell <= 1) return launch_pc32<64, 1, REFINE>(a, s);
    if (a.ell <= 4) return launch_pc32<64, 4, REFINE>(a, s);
    if (a.ell <= 8) return launch_pc32<64, 8, REFINE>(a, s);
    if (a.ell <= 10) return launch_pc32<64, 10, REFINE>(a, s);
    if (a.ell <= 12) return launch_pc32<64, 12, REFINE>(a, s);
    return launch_pc32<64, 16, REFINE>(a, s);
}

__global__ __launch_bounds__(256) void exp_nonpos64_kernel(const double *__restrict__ x,
                                                          double *__restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = exp_nonpos64(x[i]);
}

__global__ __launch_bounds__(256) void exp_nonpos32_kernel(const float *__restrict__ x,
                                                           float *__restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = exp_nonpos32(x[i]);
}

}  // namespace

hipError_t launch_exp_nonpos64(const double *x, double *y, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(exp_nonpos64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       x, y, n);
    return hipGetLastError();
}

hipError_t launch_exp_nonpos32(const float *x, float *y, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(exp_nonpos32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       x, y, n);
    return hipGetLastError();
}

hipError_t launch_precompute32(bool refine, const PrecomputeArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    return refine ? launch_pc32_k<true>(a, s) : launch_pc32_k<false>(a, s);
}

}  // namespace fmg
