// Attainable rates of the units the apply passes are bound by, measured on
// the device the library runs on: an HBM copy, FP32 FMA chains, v_rsq_f32
// chains, and the inner loop of the FP32 symmetric transverse pass (Sec. 4)
// with its operands in registers, once with the squared distances on the
// vector ALUs and once with one matrix-core product per 16 x 16 pair tile.
// The loops' results are stored so that nothing is optimised away.
#include <chrono>

#include "nnca_internal.h"

namespace nnca {

namespace {

typedef float pr_floatx4 __attribute__((ext_vector_type(4)));
constexpr int PR_NT = 256;
constexpr int PR_BLOCKS = 4 * 4096;   // 64 workgroups per CU
constexpr int PR_ITERS = 2000;

__global__ void k_pr_copy(int64_t n4, const float4 *a, float4 *b)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// eight independent FMA chains per lane
__global__ __launch_bounds__(PR_NT) void k_pr_fma(const float *in, float *out, int iters)
{
    const int l = threadIdx.x & 63;
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; q++) v[q] = in[l + q];
    const float m = in[l + 9] + 0.999f, a = in[l + 10] + 1e-3f;
    for (int it = 0; it < iters; it++)
#pragma unroll
        for (int q = 0; q < 8; q++) v[q] = fmaf(v[q], m, a);
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < 8; q++) s += v[q];
    out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = s;
}

// eight independent reciprocal-square-root chains per lane
__global__ __launch_bounds__(PR_NT) void k_pr_rsq(const float *in, float *out, int iters)
{
    const int l = threadIdx.x & 63;
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; q++) v[q] = in[l + q] + 1.5f;
    for (int it = 0; it < iters; it++)
#pragma unroll
        for (int q = 0; q < 8; q++) v[q] = __builtin_amdgcn_rsqf(v[q]);
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < 8; q++) s += v[q];
    out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = s;
}

// four targets per lane, one source per step: r^2 = |t|^2 + |s|^2 - 2 t.s
// (one addition, three FMAs), v_rsq_f32, a row and a column FMA
__global__ __launch_bounds__(PR_NT) void k_pr_pairs_valu(const float *in, float *out, int iters)
{
    constexpr int R = 4;
    const int l = threadIdx.x & 63;
    float tx[R], ty[R], tz[R], tn[R], tw[R], acc[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        tx[r] = in[l + r];
        ty[r] = in[l + r + 1];
        tz[r] = in[l + r + 2];
        tn[r] = 3.f + in[l + r];
        tw[r] = in[l + r + 4];
        acc[r] = 0.f;
    }
    float qx = in[l + 7];
    const float qy = in[l + 8], qz = in[l + 9], qn = in[l + 10], qw = in[l + 11];
    float col = 0.f;
    for (int it = 0; it < iters; it++) {
        qx += 1e-7f;
        float cp = 0.f;
#pragma unroll
        for (int r = 0; r < R; r++) {
            float r2 = tn[r] + qn;
            r2 = fmaf(tz[r], qz, r2);
            r2 = fmaf(ty[r], qy, r2);
            r2 = fmaf(tx[r], qx, r2);
            const float k = __builtin_amdgcn_rsqf(r2);
            acc[r] = fmaf(k, qw, acc[r]);
            cp = fmaf(k, tw[r], cp);
        }
        col += cp;
    }
    float s = col;
#pragma unroll
    for (int r = 0; r < R; r++) s += acc[r];
    out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = s;
}

// one 16 x 16 tile per step: r^2 from v_mfma_f32_16x16x4f32 (A = (t, 1),
// B = (-2 s, |s|^2), C = |t|^2), then per lane four v_rsq_f32 and eight FMAs
__global__ __launch_bounds__(PR_NT) void k_pr_pairs_mfma(const float *in, float *out, int iters)
{
    const int l = threadIdx.x & 63;
    const float a = in[l];
    pr_floatx4 c;
    float tw[4], racc[4];
#pragma unroll
    for (int r = 0; r < 4; r++) {
        c[r] = 1.f + in[l + r];
        tw[r] = in[l + 8 + r];
        racc[r] = 0.f;
    }
    float b = in[l + 3];
    const float w = in[l + 5];
    float cp = 0.f;
    for (int it = 0; it < iters; it++) {
        b += 1e-7f;
        const pr_floatx4 r2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const float k = __builtin_amdgcn_rsqf(r2[r]);
            racc[r] = fmaf(k, w, racc[r]);
            cp = fmaf(k, tw[r], cp);
        }
    }
    float s = cp;
#pragma unroll
    for (int r = 0; r < 4; r++) s += racc[r];
    out[blockIdx.x * (int64_t)blockDim.x + threadIdx.x] = s;
}

// milliseconds of the second of two launches
template <typename F>
double time_ms(F launch, hipStream_t s)
{
    hipEvent_t a, b;
    HIPCHECK(hipEventCreate(&a));
    HIPCHECK(hipEventCreate(&b));
    float ms = 0.f;
    try {
        launch();
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipEventRecord(a, s));
        launch();
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipEventRecord(b, s));
        HIPCHECK(hipEventSynchronize(b));
        HIPCHECK(hipEventElapsedTime(&ms, a, b));
    } catch (...) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        throw;
    }
    HIPCHECK(hipEventDestroy(a));
    HIPCHECK(hipEventDestroy(b));
    return ms;
}

}  // namespace

void probe_rates(double *out, int32_t count, hipStream_t s)
{
    const int64_t copy_floats = (int64_t)64 << 20;   // 256 MiB each way
    const int64_t nout = (int64_t)PR_BLOCKS * PR_NT;
    float *buf = dalloc<float>(2 * copy_floats);
    float *res = dalloc<float>(nout + 4096);
    try {
        float *in = res + nout;   // 4096 zeros: the loops' operands
        HIPCHECK(hipMemsetAsync(in, 0, 4096 * sizeof(float), s));
        HIPCHECK(hipMemsetAsync(buf, 0, copy_floats * sizeof(float), s));
        double r[5] = {0, 0, 0, 0, 0};
        {
            const int64_t n4 = copy_floats / 4;
            const double ms = time_ms([&] {
                k_pr_copy<<<4096, 256, 0, s>>>(n4, reinterpret_cast<const float4 *>(buf),
                                               reinterpret_cast<float4 *>(buf + copy_floats));
            }, s);
            r[0] = 2.0 * copy_floats * sizeof(float) / (ms * 1e-3);
        }
        const double lanes = (double)PR_BLOCKS * PR_NT * PR_ITERS;
        r[1] = lanes * 8 / (time_ms([&] { k_pr_fma<<<PR_BLOCKS, PR_NT, 0, s>>>(in, res, PR_ITERS); }, s) * 1e-3);
        r[2] = lanes * 8 / (time_ms([&] { k_pr_rsq<<<PR_BLOCKS, PR_NT, 0, s>>>(in, res, PR_ITERS); }, s) * 1e-3);
        r[3] = lanes * 4 /
               (time_ms([&] { k_pr_pairs_valu<<<PR_BLOCKS, PR_NT, 0, s>>>(in, res, PR_ITERS); }, s) * 1e-3);
        r[4] = lanes * 4 /   // 256 pairs per wave and step: 4 per lane
               (time_ms([&] { k_pr_pairs_mfma<<<PR_BLOCKS, PR_NT, 0, s>>>(in, res, PR_ITERS); }, s) * 1e-3);
        for (int32_t q = 0; q < count && q < 5; q++) out[q] = r[q];
    } catch (...) {
        dfree(buf);
        dfree(res);
        throw;
    }
    dfree(buf);
    dfree(res);
}

}  // namespace nnca
