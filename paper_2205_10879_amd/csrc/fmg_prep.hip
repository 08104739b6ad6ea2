// Ingest kernels: input checks, the centring vector, and the screening rows.
//
// Screening rows let one MFMA product return the screened squared distance
// minus the query norm:
//   candidate row  P_p = [-2 x~_p , ||x~_p||^2 split into parts , 0 ...]
//   query row      Q_q = [   z~_q , 1 for every part          , 0 ...]
//   <P_p, Q_q> = ||x~_p||^2 - 2 <x~_p, z~_q> = ||x~_p - z~_q||^2 - ||z~_q||^2
// where x~ is x - mu rounded to the screening type.  BF16 carries the norm
// as three BF16 parts (hi + mid + lo, 24 significant bits together); FP32
// carries it as one FP32 value.  For every row the kernels also record the
// exact ||x~||^2 (FP64) and the rounding radius e = ||(x - mu) - x~||_2,
// which the exactness certificate of the re-rank uses.
#include "fmg_device.h"
#include "fmg_kernels.h"

namespace fmg {

namespace {

// Column mean in two deterministic passes.  Pass 1: block b sums a fixed
// chunk of rows; thread (rl, c) of the block adds rows rl, rl + RL, ... of
// column c (RL = 256 / d row lanes, so a wavefront reads whole rows), and
// the row lanes are combined in a fixed order.  Pass 2: one block per column
// sums the chunk partials in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void col_partial_kernel(const T *__restrict__ X, int64_t n, int d,
                                                          int64_t rows_per_block,
                                                          double *__restrict__ part) {
    __shared__ double sh[256];
    const int t = threadIdx.x;
    const int rlanes = 256 / d;
    const int c = t % d, rl = t / d;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = (r0 + rows_per_block < n) ? r0 + rows_per_block : n;
    double s = 0.0;
    if (rl < rlanes)
        for (int64_t r = r0 + rl; r < r1; r += rlanes) s += (double)X[r * d + c];
    sh[t] = s;
    __syncthreads();
    if (t < d) {
        double acc = 0.0;
        for (int k = 0; k < rlanes; ++k) acc += sh[k * d + t];
        part[(int64_t)blockIdx.x * d + t] = acc;
    }
}

__global__ __launch_bounds__(256) void col_final_kernel(const double *__restrict__ part, int nb,
                                                        int d, int64_t n, float *__restrict__ mu) {
    __shared__ double sh[256];
    const int c = blockIdx.x, t = threadIdx.x;
    double s = 0.0;
    for (int b = t; b < nb; b += 256) s += part[(int64_t)b * d + c];
    sh[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) mu[c] = (float)(sh[0] / (double)n);
}

template <typename T>
__global__ __launch_bounds__(256) void finite_kernel(const T *__restrict__ A, int64_t count,
                                                     int *__restrict__ flag) {
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * 256) {
        double v = (double)A[i];
        bad |= !isfinite(v);
    }
    if (__ballot(bad) != 0 && lane_id() == 0) atomicOr(flag, 1);
}

// Running maxima of non-negative doubles as their bit patterns (which order
// like the values): one atomic per wavefront, after a wave-wide maximum.
__device__ __forceinline__ void wave_atomic_max_bits(unsigned long long *dst, double v) {
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const unsigned long long o =
            ((unsigned long long)(uint32_t)__shfl_xor((int)(b >> 32), w) << 32) |
            (uint32_t)__shfl_xor((int)(uint32_t)b, w);
        b = o > b ? o : b;
    }
    if (lane_id() == 0) atomicMax(dst, b);
}

// One thread per row; the row (kp = 64 BF16 values, 128 bytes) is assembled
// in registers and written with 16-byte stores.
__global__ __launch_bounds__(256) void prep_bf16_kernel(
    const float *__restrict__ X, int64_t n, int64_t n_pad, int d, const float *__restrict__ mu,
    uint16_t *__restrict__ Q, uint16_t *__restrict__ P, double *__restrict__ e_out,
    double *__restrict__ nz_out, unsigned long long *emax_bits,
    unsigned long long *nxmax_bits) {
    constexpr int KP = 64;
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t qw[KP / 2], pw[KP / 2];  // pairs of BF16 values
#pragma unroll
    for (int w = 0; w < KP / 2; ++w) {
        qw[w] = 0u;
        pw[w] = 0u;
    }
    // lanes past n_pad write nothing but still take part in the wave maxima
    double e = 0.0, nz = 0.0;
    if (r < n) {
        const float *__restrict__ xr = X + r * d;
        double e2 = 0.0;
#pragma unroll
        for (int c = 0; c < KP; ++c) {
            if (c < d) {
                const double xc = (double)xr[c] - (double)mu[c];
                const uint16_t h = f32_to_bf16_rn((float)xc);
                const double xt = (double)bf16_to_f32(h);
                const double diff = xc - xt;
                e2 += diff * diff;
                nz += xt * xt;
                // -2 x~ is exact: a power-of-two scale
                const uint16_t ph = f32_to_bf16_rn(-2.0f * bf16_to_f32(h));
                qw[c >> 1] |= (uint32_t)h << (16 * (c & 1));
                pw[c >> 1] |= (uint32_t)ph << (16 * (c & 1));
            }
        }
        // norm split: nz = hi + mid + lo (+ a remainder below 2^-26 nz)
        const uint16_t hi = f32_to_bf16_rn((float)nz);
        const double r1 = nz - (double)bf16_to_f32(hi);
        const uint16_t mid = f32_to_bf16_rn((float)r1);
        const double r2 = r1 - (double)bf16_to_f32(mid);
        const uint16_t lo = f32_to_bf16_rn((float)r2);
        const uint16_t one = f32_to_bf16_rn(1.0f);
#pragma unroll
        for (int c = 0; c < KP; ++c) {
            const int sh = 16 * (c & 1);
            if (c >= d && c < d + 3) qw[c >> 1] |= (uint32_t)one << sh;
            const uint16_t pv = (c == d) ? hi : (c == d + 1) ? mid : (c == d + 2) ? lo : 0;
            pw[c >> 1] |= (uint32_t)pv << sh;
        }
        e = sqrt(e2) * (1.0 + 1.0e-12);
        if (e_out) e_out[r] = e;
        if (nz_out) nz_out[r] = nz;
    } else if (r < n_pad) {
        // Padding candidate: a huge norm part keeps it out of every selection.
        const uint16_t big = f32_to_bf16_rn(1.0e30f);
#pragma unroll
        for (int c = 0; c < KP; ++c)
            if (c == d) pw[c >> 1] |= (uint32_t)big << (16 * (c & 1));
    }
    if (r < n_pad) {
        if (Q) {
            uint4 *dst = (uint4 *)(Q + r * KP);
#pragma unroll
            for (int w = 0; w < KP / 8; ++w)
                dst[w] = make_uint4(qw[4 * w], qw[4 * w + 1], qw[4 * w + 2], qw[4 * w + 3]);
        }
        if (P) {
            uint4 *dst = (uint4 *)(P + r * KP);
#pragma unroll
            for (int w = 0; w < KP / 8; ++w)
                dst[w] = make_uint4(pw[4 * w], pw[4 * w + 1], pw[4 * w + 2], pw[4 * w + 3]);
        }
    }
    if (emax_bits) wave_atomic_max_bits(emax_bits, e);
    if (nxmax_bits) wave_atomic_max_bits(nxmax_bits, nz);
}

__global__ __launch_bounds__(256) void prep_f32_kernel(
    const float *__restrict__ X, int64_t n, int64_t n_pad, int d, const float *__restrict__ mu,
    int kp, float *__restrict__ Q, float *__restrict__ P, double *__restrict__ e_out,
    double *__restrict__ nz_out, unsigned long long *emax_bits,
    unsigned long long *nxmax_bits) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    // lanes past n_pad write nothing but still take part in the wave maxima
    float *q = (Q && r < n_pad) ? Q + r * kp : nullptr;
    float *p = (P && r < n_pad) ? P + r * kp : nullptr;
    double e = 0.0, nz = 0.0;
    if (r >= n_pad) {
    } else if (r >= n) {
        for (int c = 0; c < kp; ++c) {
            if (q) q[c] = 0.0f;
            if (p) p[c] = 0.0f;
        }
        if (p) p[d] = 1.0e30f;
    } else {
    double e2 = 0.0;
    for (int c = 0; c < d; ++c) {
        const double xc = (double)X[r * d + c] - (double)mu[c];
        const float xt = (float)xc;
        const double diff = xc - (double)xt;
        e2 += diff * diff;
        nz += (double)xt * (double)xt;
        if (q) q[c] = xt;
        if (p) p[c] = -2.0f * xt;
    }
    for (int c = d; c < kp; ++c) {
        if (q) q[c] = (c == d) ? 1.0f : 0.0f;
        if (p) p[c] = (c == d) ? (float)nz : 0.0f;
    }
    e = (e2 > 0.0) ? sqrt(e2) * (1.0 + 1.0e-12) : 0.0;
    if (e_out) e_out[r] = e;
    if (nz_out) nz_out[r] = nz;
    }
    if (emax_bits) wave_atomic_max_bits(emax_bits, e);
    if (nxmax_bits) wave_atomic_max_bits(nxmax_bits, nz);
}

__global__ __launch_bounds__(256) void count_nonzero_kernel(const int32_t *__restrict__ a,
                                                            int64_t n,
                                                            unsigned long long *out) {
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
        c += (a[i] != 0);
    for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m);
    if (lane_id() == 0 && c) atomicAdd(out, c);
}

__global__ __launch_bounds__(256) void self_rows_kernel(int32_t *N, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) N[i] = (int32_t)i;
}

__global__ __launch_bounds__(256) void zero_kernel(uint32_t *p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * 256)
        p[i] = 0u;
}

__global__ void accum_kernel(const int32_t *src, unsigned long long *dst) {
    if (threadIdx.x == 0) atomicAdd(dst, (unsigned long long)(*src));
}

}  // namespace

hipError_t launch_self_rows(int32_t *N, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(self_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, n);
    return hipGetLastError();
}

hipError_t launch_zero_u32(void *ptr, int64_t count, hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)ptr, count);
    return hipGetLastError();
}

hipError_t launch_accum(const int32_t *src, unsigned long long *dst, hipStream_t s) {
    hipLaunchKernelGGL(accum_kernel, dim3(1), dim3(64), 0, s, src, dst);
    return hipGetLastError();
}

int col_mean_blocks(int64_t n) {
    int64_t nb = (n + 255) / 256;
    return (int)(nb > 1024 ? 1024 : (nb < 1 ? 1 : nb));
}

hipError_t launch_col_mean(const void *X, bool f64, int64_t n, int d, float *mu, double *part,
                           hipStream_t s) {
    if (d < 1 || d > 256) return hipErrorInvalidValue;
    const int nb = col_mean_blocks(n);
    const int64_t rpb = (n + nb - 1) / nb;
    if (f64)
        hipLaunchKernelGGL(col_partial_kernel<double>, dim3(nb), dim3(256), 0, s,
                           (const double *)X, n, d, rpb, part);
    else
        hipLaunchKernelGGL(col_partial_kernel<float>, dim3(nb), dim3(256), 0, s,
                           (const float *)X, n, d, rpb, part);
    hipLaunchKernelGGL(col_final_kernel, dim3(d), dim3(256), 0, s, (const double *)part, nb, d, n,
                       mu);
    return hipGetLastError();
}

hipError_t launch_finite_check(const void *A, bool f64, int64_t count, int *flag,
                               hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    if (f64)
        hipLaunchKernelGGL(finite_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const double *)A, count, flag);
    else
        hipLaunchKernelGGL(finite_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (const float *)A, count, flag);
    return hipGetLastError();
}

hipError_t launch_prep_rows(const ScreenGeom &g, const float *X, int64_t n, int64_t n_pad, int d,
                            const float *mu, void *Qrows, void *Prows, double *e_out,
                            double *nz_out, unsigned long long *emax_bits,
                            unsigned long long *nxmax_bits, hipStream_t s) {
    const unsigned blocks = (unsigned)((n_pad + 255) / 256);
    if (g.mode == SCREEN_BF16) {
        if (g.kp != 64 || d + 3 > 64) return hipErrorInvalidValue;
        hipLaunchKernelGGL(prep_bf16_kernel, dim3(blocks), dim3(256), 0, s, X, n, n_pad, d, mu,
                           (uint16_t *)Qrows, (uint16_t *)Prows, e_out, nz_out, emax_bits,
                           nxmax_bits);
    } else {
        hipLaunchKernelGGL(prep_f32_kernel, dim3(blocks), dim3(256), 0, s, X, n, n_pad, d, mu,
                           g.kp, (float *)Qrows, (float *)Prows, e_out, nz_out, emax_bits,
                           nxmax_bits);
    }
    return hipGetLastError();
}

hipError_t launch_count_nonzero(const int32_t *a, int64_t n, unsigned long long *out,
                                hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(count_nonzero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, n, out);
    return hipGetLastError();
}

}  // namespace fmg
