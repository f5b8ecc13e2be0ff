// Restarted GMRES for (alpha I + beta A~) x = f with the H2 matvec (the
// integral-equation solve of Exp. 5 of Sec. 5: a Nystrom discretisation of a
// second-kind Fredholm equation gives alpha = 1 and beta = the quadrature
// weight).  Arnoldi with classical Gram-Schmidt applied twice; the small
// Hessenberg least-squares problem is solved on the host by Givens rotations.
// Every inner product is a fixed-shape device reduction, so the iteration is
// run-to-run deterministic.
#include <cmath>
#include <vector>

#include "nnca_internal.h"

namespace nnca {

namespace {

constexpr int GM_NT = 256;
constexpr int GM_BLK = 512;   // partial sums per inner product

// part[c * GM_BLK + b] = sum over block b's fixed slice of V[:, c] . w
// (c < ncols; columns of V at stride ld)
__global__ __launch_bounds__(GM_NT) void k_gm_dots(int64_t n, const double *V, int64_t ld, int ncols,
                                                   const double *w, double *part)
{
    __shared__ double red[GM_NT];
    const int c = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
    const int64_t per = (n + GM_BLK - 1) / GM_BLK;
    const int64_t i0 = (int64_t)b * per, i1 = i0 + per < n ? i0 + per : n;
    const double *v = V + (int64_t)c * ld;
    double s = 0.0;
    for (int64_t i = i0 + t; i < i1; i += GM_NT) s += v[i] * w[i];
    red[t] = s;
    __syncthreads();
    for (int h = GM_NT / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) part[(int64_t)c * GM_BLK + b] = red[0];
}

// out[c] = sum of the GM_BLK partials of column c, in order
__global__ void k_gm_sum(int ncols, const double *part, double *out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    double s = 0.0;
    for (int b = 0; b < GM_BLK; b++) s += part[(int64_t)c * GM_BLK + b];
    out[c] = s;
}

// w -= sum_c V[:, c] h[c]
__global__ void k_gm_sub(int64_t n, const double *V, int64_t ld, int ncols, const double *h, double *w)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = w[i];
    for (int c = 0; c < ncols; c++) s -= V[(int64_t)c * ld + i] * h[c];
    w[i] = s;
}

// y = a x + b y
__global__ void k_gm_axpby(int64_t n, double a, const double *x, double b, double *y)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + b * y[i];
}

// y = a x
__global__ void k_gm_scale(int64_t n, double a, const double *x, double *y)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}

// x += sum_c V[:, c] y[c]
__global__ void k_gm_add(int64_t n, const double *V, int64_t ld, int ncols, const double *y, double *x)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = x[i];
    for (int c = 0; c < ncols; c++) s += V[(int64_t)c * ld + i] * y[c];
    x[i] = s;
}

struct Gm {
    nnca_h2 *H;
    hipStream_t s;
    int64_t n;
    double alpha, beta;
    int prec;
    double *part, *dh, *tmp;

    // out = (alpha I + beta A~) x
    void op(const double *x, double *out)
    {
        run_matvec(H, x, tmp, 1, n, n, NNCA_F64, prec, s);
        k_gm_axpby<<<grid_for(n, 256), 256, 0, s>>>(n, alpha, x, beta, tmp);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipMemcpyAsync(out, tmp, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    // host h[0..nc) = V[:, 0..nc)^T w
    void dots(const double *V, int nc, const double *w, double *h)
    {
        k_gm_dots<<<dim3(GM_BLK, nc), GM_NT, 0, s>>>(n, V, n, nc, w, part);
        HIPCHECK(hipGetLastError());
        k_gm_sum<<<(nc + 63) / 64, 64, 0, s>>>(nc, part, dh);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipMemcpyAsync(h, dh, sizeof(double) * nc, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
    }
    double norm(const double *w)
    {
        double v = 0.0;
        dots(w, 1, w, &v);
        return std::sqrt(v);
    }
};

}  // namespace

void run_gmres(nnca_h2 *H, double alpha, double beta, const double *F, double *X, double tol, int32_t max_iter,
               int32_t restart, int precision, int32_t *iters, double *relres, hipStream_t s)
{
    const int64_t n = H->n;
    const int m = restart;
    double *V = dalloc<double>((size_t)n * (m + 1));
    double *w = dalloc<double>(n);
    Gm g{H, s, n, alpha, beta, precision, nullptr, nullptr, nullptr};
    try {
        g.part = dalloc<double>((size_t)GM_BLK * (m + 1));
        g.dh = dalloc<double>(m + 1);
        g.tmp = dalloc<double>(n);
        const double fn = g.norm(F);
        int it = 0;
        double rel = 0.0;
        std::vector<double> Hh((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), hc(m + 1), hc2(m + 1), y(m);
        if (fn == 0.0) {
            k_gm_scale<<<grid_for(n, 256), 256, 0, s>>>(n, 0.0, F, X);
            HIPCHECK(hipGetLastError());
        } else {
            for (;;) {
                // r = f - (alpha I + beta A~) x
                g.op(X, w);
                k_gm_axpby<<<grid_for(n, 256), 256, 0, s>>>(n, 1.0, F, -1.0, w);
                HIPCHECK(hipGetLastError());
                const double b0 = g.norm(w);
                rel = b0 / fn;
                if (rel <= tol || it >= max_iter) break;
                k_gm_scale<<<grid_for(n, 256), 256, 0, s>>>(n, 1.0 / b0, w, V);
                HIPCHECK(hipGetLastError());
                std::fill(gv.begin(), gv.end(), 0.0);
                gv[0] = b0;
                int j = 0;
                for (; j < m && it < max_iter; j++, it++) {
                    double *vj1 = V + (int64_t)(j + 1) * n;
                    g.op(V + (int64_t)j * n, vj1);
                    // classical Gram-Schmidt, twice
                    g.dots(V, j + 1, vj1, hc.data());
                    HIPCHECK(hipMemcpyAsync(g.dh, hc.data(), sizeof(double) * (j + 1), hipMemcpyHostToDevice, s));
                    k_gm_sub<<<grid_for(n, 256), 256, 0, s>>>(n, V, n, j + 1, g.dh, vj1);
                    HIPCHECK(hipGetLastError());
                    g.dots(V, j + 1, vj1, hc2.data());
                    HIPCHECK(hipMemcpyAsync(g.dh, hc2.data(), sizeof(double) * (j + 1), hipMemcpyHostToDevice, s));
                    k_gm_sub<<<grid_for(n, 256), 256, 0, s>>>(n, V, n, j + 1, g.dh, vj1);
                    HIPCHECK(hipGetLastError());
                    for (int i = 0; i <= j; i++) hc[i] += hc2[i];
                    const double hn = g.norm(vj1);
                    if (hn > 0.0) {
                        k_gm_scale<<<grid_for(n, 256), 256, 0, s>>>(n, 1.0 / hn, vj1, vj1);
                        HIPCHECK(hipGetLastError());
                    }
                    // the new column of the Hessenberg matrix through the
                    // previous rotations, then its own rotation
                    for (int i = 0; i < j; i++) {
                        const double a = cs[i] * hc[i] + sn[i] * hc[i + 1];
                        hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
                        hc[i] = a;
                    }
                    const double rr = std::hypot(hc[j], hn);
                    cs[j] = rr > 0.0 ? hc[j] / rr : 1.0;
                    sn[j] = rr > 0.0 ? hn / rr : 0.0;
                    hc[j] = rr;
                    for (int i = 0; i <= j; i++) Hh[(size_t)i * m + j] = hc[i];
                    gv[j + 1] = -sn[j] * gv[j];
                    gv[j] = cs[j] * gv[j];
                    rel = std::fabs(gv[j + 1]) / fn;
                    if (rel <= tol || hn == 0.0) {
                        j++;
                        it++;
                        break;
                    }
                }
                // y = R^{-1} g, x += V y
                for (int i = j - 1; i >= 0; i--) {
                    double a = gv[i];
                    for (int q = i + 1; q < j; q++) a -= Hh[(size_t)i * m + q] * y[q];
                    y[i] = a / Hh[(size_t)i * m + i];
                }
                HIPCHECK(hipMemcpyAsync(g.dh, y.data(), sizeof(double) * j, hipMemcpyHostToDevice, s));
                k_gm_add<<<grid_for(n, 256), 256, 0, s>>>(n, V, n, j, g.dh, X);
                HIPCHECK(hipGetLastError());
                HIPCHECK(hipStreamSynchronize(s));
                if (rel <= tol || it >= max_iter) {
                    // the true residual of the final iterate
                    g.op(X, w);
                    k_gm_axpby<<<grid_for(n, 256), 256, 0, s>>>(n, 1.0, F, -1.0, w);
                    HIPCHECK(hipGetLastError());
                    rel = g.norm(w) / fn;
                    break;
                }
            }
        }
        if (iters) *iters = it;
        if (relres) *relres = rel;
    } catch (...) {
        (void)hipStreamSynchronize(s);
        dfree(V);
        dfree(w);
        dfree(g.part);
        dfree(g.dh);
        dfree(g.tmp);
        throw;
    }
    HIPCHECK(hipStreamSynchronize(s));
    dfree(V);
    dfree(w);
    dfree(g.part);
    dfree(g.dh);
    dfree(g.tmp);
}

}  // namespace nnca
