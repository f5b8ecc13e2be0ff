// Kernel SVM by gradient ascent with the H2 matvec (Exp. 6 of Sec. 5).  The
// dual objective with the equality constraint as a penalty,
//   L(a) = sum_i a_i - 1/2 sum_ij K_ij y_i y_j a_i a_j - 1/2 beta (sum_j a_j y_j)^2,
// has the gradient 1 - y .* (K v) - beta (sum v) y with v = y .* a.  Each
// step adds eta times the gradient and projects onto the box 0 <= a <= lambda.
// Every reduction has a fixed shape (run-to-run deterministic).  The decision
// function at new points is f(x) = sum_i a_i y_i K(x_i, x) + b, the product
// of a general (targets = new points, sources = training points) handle with
// v = y .* a.
#include <cmath>
#include <vector>

#include "nnca_internal.h"

namespace nnca {

namespace {

constexpr int SV_NT = 256;
constexpr int SV_BLK = 512;   // partial sums per reduction
static_assert(SV_BLK == 2 * SV_NT, "k_sv_step folds the partials two per thread");

// elementwise kernels: grid-stride loops (the grid is capped by grid_for)
__global__ void k_sv_mul(int64_t n, const double *a, const double *b, double *c)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c[i] = a[i] * b[i];
}

// part[b] = the sum of v over block b's fixed slice of [0, n)
__global__ __launch_bounds__(SV_NT) void k_sv_sum(int64_t n, const double *v, double *part)
{
    __shared__ double red[SV_NT];
    const int b = blockIdx.x, t = threadIdx.x;
    const int64_t per = (n + SV_BLK - 1) / SV_BLK;
    const int64_t i0 = (int64_t)b * per, i1 = i0 + per < n ? i0 + per : n;
    double s = 0.0;
    for (int64_t i = i0 + t; i < i1; i += SV_NT) s += v[i];
    red[t] = s;
    __syncthreads();
    for (int h = SV_NT / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) part[b] = red[0];
}

// One step, for every block: s = sum v from the previous step's SV_BLK
// partials (svin, the same fixed-shape fold in every block), then
// a_new = clip(a + eta (1 - y Kv - beta s y), 0, lambda), v_new = y a_new, and
// per block the sums of (a_new - a)^2, a_new^2 (part, part + SV_BLK) and
// v_new (svout).  Nothing is written once the stopping rule has fired
// (*state: [0] done flag, [1] steps taken).
__global__ __launch_bounds__(SV_NT) void k_sv_step(int64_t n, const double *y, const double *kv, const double *svin,
                                                   double eta, double beta, double lambda, double *a, double *v,
                                                   double *part, double *svout, const int32_t *state)
{
    __shared__ double rd[SV_NT], ra[SV_NT], rv[SV_NT];
    if (state[0]) return;   // uniform for the grid
    const int b = blockIdx.x, t = threadIdx.x;
    rd[t] = svin[t] + svin[t + SV_NT];   // SV_BLK = 2 SV_NT partials
    __syncthreads();
    for (int h = SV_NT / 2; h > 0; h >>= 1) {
        if (t < h) rd[t] += rd[t + h];
        __syncthreads();
    }
    const double s = rd[0];
    __syncthreads();
    const int64_t per = (n + SV_BLK - 1) / SV_BLK;
    const int64_t i0 = (int64_t)b * per, i1 = i0 + per < n ? i0 + per : n;
    double d2 = 0.0, a2 = 0.0, vs = 0.0;
    for (int64_t i = i0 + t; i < i1; i += SV_NT) {
        const double g = (1.0 - y[i] * kv[i]) - beta * s * y[i];
        double an = a[i] + eta * g;
        an = an < 0.0 ? 0.0 : (an > lambda ? lambda : an);
        const double dd = an - a[i];
        d2 += dd * dd;
        a2 += an * an;
        a[i] = an;
        const double vn = y[i] * an;
        v[i] = vn;
        vs += vn;
    }
    rd[t] = d2;
    ra[t] = a2;
    rv[t] = vs;
    __syncthreads();
    for (int h = SV_NT / 2; h > 0; h >>= 1) {
        if (t < h) {
            rd[t] += rd[t + h];
            ra[t] += ra[t + h];
            rv[t] += rv[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        part[b] = rd[0];
        part[SV_BLK + b] = ra[0];
        svout[b] = rv[0];
    }
}

// the stopping rule after a step: ||a_new - a|| <= tol ||a_new|| (||a_new||
// read as 1 when it is 0); counts the step and sets the done flag
__global__ void k_sv_check(const double *part, double tol, int32_t *state)
{
    if (threadIdx.x != 0 || state[0]) return;
    double d2 = 0.0, a2 = 0.0;
    for (int b = 0; b < SV_BLK; b++) {
        d2 += part[b];
        a2 += part[SV_BLK + b];
    }
    const double dn = sqrt(d2), an = sqrt(a2);
    state[1] += 1;
    if (dn <= tol * (an > 0.0 ? an : 1.0)) state[0] = 1;
}

// the bias terms: per block the sum of y_i - (K v)_i over the free support
// vectors (0 < a_i < lambda) and their count
__global__ __launch_bounds__(SV_NT) void k_sv_bias(int64_t n, const double *y, const double *kv, const double *a,
                                                   double lambda, double *part)
{
    __shared__ double rs[SV_NT], rc[SV_NT];
    const int b = blockIdx.x, t = threadIdx.x;
    const int64_t per = (n + SV_BLK - 1) / SV_BLK;
    const int64_t i0 = (int64_t)b * per, i1 = i0 + per < n ? i0 + per : n;
    double s = 0.0, c = 0.0;
    for (int64_t i = i0 + t; i < i1; i += SV_NT)
        if (a[i] > 0.0 && a[i] < lambda) {
            s += y[i] - kv[i];
            c += 1.0;
        }
    rs[t] = s;
    rc[t] = c;
    __syncthreads();
    for (int h = SV_NT / 2; h > 0; h >>= 1) {
        if (t < h) {
            rs[t] += rs[t + h];
            rc[t] += rc[t + h];
        }
        __syncthreads();
    }
    if (t == 0) {
        part[b] = rs[0];
        part[SV_BLK + b] = rc[0];
    }
}

// out[q] = sum of the SV_BLK partials of quantity q, in order
__global__ void k_sv_fold(int nq, const double *part, double *out)
{
    const int q = threadIdx.x;
    if (q >= nq) return;
    double s = 0.0;
    for (int b = 0; b < SV_BLK; b++) s += part[q * SV_BLK + b];
    out[q] = s;
}

__global__ void k_sv_addc(int64_t n, double c, double *y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += c;
}

__global__ void k_sv_scale(int64_t n, double c, const double *x, double *y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = c * x[i];
}

__global__ void k_sv_fill(int64_t n, double c, double *y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = c;
}

}  // namespace

void run_svm_train(nnca_h2 *H, const double *y, double *alpha, double lambda, double beta, double eta, double tol,
                   int32_t max_iter, int precision, int32_t *iters, double *bias, double *eta_used,
                   hipStream_t s)
{
    const int64_t n = H->n;
    double *v = dalloc<double>(n), *kv = dalloc<double>(n);
    double *part = dalloc<double>(4 * SV_BLK), *red = dalloc<double>(2);
    double *svp[2] = {part + 2 * SV_BLK, part + 3 * SV_BLK};   // sum-v partials, by step parity
    int32_t *state = dalloc<int32_t>(2);
    auto release = [&] {
        dfree(v);
        dfree(kv);
        dfree(part);
        dfree(red);
        dfree(state);
    };
    try {
        const int g = grid_for(n, 256);
        double hr[2] = {0.0, 0.0};
        auto fold = [&](int nq) {
            k_sv_fold<<<1, 64, 0, s>>>(nq, part, red);
            HIPCHECK(hipGetLastError());
            HIPCHECK(hipMemcpyAsync(hr, red, sizeof(double) * nq, hipMemcpyDeviceToHost, s));
            HIPCHECK(hipStreamSynchronize(s));
        };
        if (!(eta > 0.0)) {
            // eta = 1 / (|K~|_2 + beta n): |K~|_2 by 30 steps of the power
            // method from the all-ones vector (K is symmetric positive
            // definite for the kernels of Exp. 6)
            k_sv_fill<<<g, 256, 0, s>>>(n, 1.0 / std::sqrt((double)n), v);
            HIPCHECK(hipGetLastError());
            double lam = 0.0;
            for (int it = 0; it < 30; it++) {
                run_matvec(H, v, kv, 1, n, n, NNCA_F64, precision, s);
                k_sv_mul<<<g, 256, 0, s>>>(n, kv, kv, v);
                HIPCHECK(hipGetLastError());
                k_sv_sum<<<SV_BLK, SV_NT, 0, s>>>(n, v, part);
                HIPCHECK(hipGetLastError());
                fold(1);
                lam = std::sqrt(hr[0]);
                if (!(lam > 0.0)) break;
                k_sv_scale<<<g, 256, 0, s>>>(n, 1.0 / lam, kv, v);
                HIPCHECK(hipGetLastError());
            }
            if (!(lam > 0.0)) fail(NNCA_ERR_NUMERICAL, "the kernel matrix has no positive norm");
            eta = 1.0 / (lam + beta * (double)n);
        }
        if (eta_used) *eta_used = eta;
        // v = y a and its block partials; state = {done, steps}
        k_sv_mul<<<g, 256, 0, s>>>(n, y, alpha, v);
        HIPCHECK(hipGetLastError());
        k_sv_sum<<<SV_BLK, SV_NT, 0, s>>>(n, v, svp[0]);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipMemsetAsync(state, 0, 2 * sizeof(int32_t), s));
        int32_t hs[2] = {0, 0};
        // the host reads the state every SV_POLL steps: steps launched after
        // the rule has fired change nothing (the step kernel returns at once)
        constexpr int SV_POLL = 16;
        for (int32_t it = 0; it < max_iter; it++) {
            run_matvec(H, v, kv, 1, n, n, NNCA_F64, precision, s);
            k_sv_step<<<SV_BLK, SV_NT, 0, s>>>(n, y, kv, svp[it & 1], eta, beta, lambda, alpha, v, part,
                                               svp[(it + 1) & 1], state);
            HIPCHECK(hipGetLastError());
            k_sv_check<<<1, 64, 0, s>>>(part, tol, state);
            HIPCHECK(hipGetLastError());
            if ((it + 1) % SV_POLL == 0 || it + 1 == max_iter) {
                HIPCHECK(hipMemcpyAsync(hs, state, sizeof(hs), hipMemcpyDeviceToHost, s));
                HIPCHECK(hipStreamSynchronize(s));
                if (hs[0]) break;
            }
        }
        if (iters) *iters = hs[1];
        if (bias) {
            k_sv_mul<<<g, 256, 0, s>>>(n, y, alpha, v);
            HIPCHECK(hipGetLastError());
            run_matvec(H, v, kv, 1, n, n, NNCA_F64, precision, s);
            k_sv_bias<<<SV_BLK, SV_NT, 0, s>>>(n, y, kv, alpha, lambda, part);
            HIPCHECK(hipGetLastError());
            fold(2);
            *bias = hr[1] > 0.0 ? hr[0] / hr[1] : 0.0;
        }
    } catch (...) {
        (void)hipStreamSynchronize(s);
        release();
        throw;
    }
    HIPCHECK(hipStreamSynchronize(s));
    release();
}

void run_svm_decision(nnca_h2 *H, const double *y, const double *alpha, double bias, double *f, int precision,
                      hipStream_t s)
{
    const int64_t nq = H->general ? H->nq : H->n, np = H->n;
    double *v = dalloc<double>(nq);
    try {
        k_sv_mul<<<grid_for(nq, 256), 256, 0, s>>>(nq, y, alpha, v);
        HIPCHECK(hipGetLastError());
        if (H->general) run_matvec_general(H, v, f, 1, nq, np, NNCA_F64, precision, false, s);
        else run_matvec(H, v, f, 1, nq, np, NNCA_F64, precision, s);
        k_sv_addc<<<grid_for(np, 256), 256, 0, s>>>(np, bias, f);
        HIPCHECK(hipGetLastError());
    } catch (...) {
        (void)hipStreamSynchronize(s);
        dfree(v);
        throw;
    }
    HIPCHECK(hipStreamSynchronize(s));
    dfree(v);
}

}  // namespace nnca
