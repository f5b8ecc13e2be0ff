// Backward of y = A~ x for the Gaussian kernel K(r) = exp(-r^2/h^2):
// the gradient with respect to x (the transposed passes, which the symmetric
// case of Sec. 5 makes equal to the forward ones) and the derivative of
// L = g^T A~ x with respect to the length scale h with the pivot sets frozen.
//
// With the pivots fixed, every piece of the H2 form of Sec. 3 is a function
// of h: the near-field blocks K(t^B, t^B'), the M2L blocks K(t^{B,i},
// t^{B',i}) and the transfer operators of the ACA cells,
//   C_B = K(t~, J) K(I, J)^{-1}       (I = t^{B,i} inside t~, J = s^{B,i};
//                                      Remark in Sec. 2.3.2),
// whose derivative is dC_B = (dK(t~, J) - C_B dK(I, J)) K(I, J)^{-1}.
// Reverse mode through the passes of Sec. 4 gives
//   dL/dh = g^T A~_D x + sum_B [ a_B(x)^T D(t~, J) z_B(g) + a_B(g)^T D(t~, J) z_B(x) ] (times 2/h)
// where D(r) = (r^2/h^2) exp(-r^2/h^2) = (h/2) dK/dh, A~_D is the H2 form
// with D in place of K in the M2L and near-field blocks (transfers
// unchanged), z_B(v) = K(I, J)^{-1} u_B(v) with u_B the local vector of cell
// B after the downward pass has added every coarser contribution, and
// a_B(v) = the cell's upward input over t~ (the points' values at a leaf, the
// children's multipole vectors otherwise) minus, on the pivot rows, the
// cell's own multipole vector (that is a^T dC u with C's identity rows).
//
// K(I, J) is factored once per handle in FP64 without row exchanges, in the
// ACA selection order: the ACA of Sec. 2.2.1 is exactly Gaussian elimination
// of that block with those pivots, each the largest entry of its residual
// row.
#include <algorithm>
#include <cstring>

#include "nnca_internal.h"
#include "kernel_values.h"

namespace nnca {

namespace {

constexpr int NT = 256;
constexpr int KMAX = 1024;   // largest rank the derivative kernels accept

// L U = K(I, J) for every ACA cell of a level, column-major k x k at
// lu + lu_off[c]: A(a, b) = K(t^{B,i}_a, s^{B,i}_b).
__global__ __launch_bounds__(NT) void k_lu(const int32_t *piv_ptr, const int32_t *jid, const double *ipc,
                                           int64_t npiv, const double *pts, int64_t n, int d, double prm,
                                           const int64_t *lu_off, double *lu, int32_t *flag)
{
    const int64_t c = blockIdx.x;
    const int32_t po = piv_ptr[c], k = piv_ptr[c + 1] - po;
    if (k == 0 || jid[po] < 0) return;
    double *A = lu + lu_off[c];
    for (int32_t e = threadIdx.x; e < k * k; e += NT) {
        const int32_t a = e % k, b = e / k;
        const int32_t j = jid[po + b];
        const double dx = ipc[po + a] - pts[j];
        const double dy = ipc[npiv + po + a] - pts[n + j];
        const double dz = d == 3 ? ipc[2 * npiv + po + a] - pts[2 * n + j] : 0.0;
        A[e] = kv64<NNCA_K_GAUSS>(dx * dx + dy * dy + dz * dz, prm);
    }
    for (int32_t p = 0; p < k; p++) {
        __syncthreads();
        const double piv = A[p + (int64_t)p * k];
        if (piv == 0.0) {   // the same value in every thread: a uniform exit
            if (threadIdx.x == 0) *flag = 1;
            return;
        }
        for (int32_t i = p + 1 + threadIdx.x; i < k; i += NT) A[i + (int64_t)p * k] /= piv;
        __syncthreads();
        const int32_t r = k - p - 1;
        for (int32_t e = threadIdx.x; e < r * r; e += NT) {
            const int32_t i = p + 1 + e % r, j = p + 1 + e / r;
            A[i + (int64_t)j * k] -= A[i + (int64_t)p * k] * A[p + (int64_t)j * k];
        }
    }
}

// z = K(I, J)^{-1} u for the local vectors of x and of the cotangent, one
// workgroup per ACA cell of a level (z of other cells is not used).
__global__ __launch_bounds__(NT) void k_tsolve(const int32_t *piv_ptr, const int32_t *jid, const int64_t *lu_off,
                                               const double *lu, const double *ux, const double *ug, double *zx,
                                               double *zg)
{
    __shared__ double bg[KMAX], bx[KMAX];
    const int t = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int32_t po = piv_ptr[c], k = piv_ptr[c + 1] - po;
    if (k == 0 || jid[po] < 0) return;   // uniform for the workgroup
    const double *A = lu + lu_off[c];
    for (int32_t i = t; i < k; i += NT) {
        bg[i] = ug[po + i];
        bx[i] = ux[po + i];
    }
    // forward substitution with the unit lower factor; step p only changes
    // entries other than p, so one barrier per step suffices
    for (int32_t p = 0; p < k; p++) {
        __syncthreads();
        const double vg = bg[p], vx = bx[p];
        for (int32_t i = p + 1 + t; i < k; i += NT) {
            const double l = A[i + (int64_t)p * k];
            bg[i] -= l * vg;
            bx[i] -= l * vx;
        }
    }
    // back substitution with the upper factor
    for (int32_t p = k - 1; p >= 0; p--) {
        __syncthreads();
        const double upp = A[p + (int64_t)p * k];
        const double vg = bg[p] / upp, vx = bx[p] / upp;
        if (t == 0) {
            zg[po + p] = vg;
            zx[po + p] = vx;
        }
        for (int32_t i = t; i < p; i += NT) {
            const double uu = A[i + (int64_t)p * k];
            bg[i] -= uu * vg;
            bx[i] -= uu * vx;
        }
    }
}

// Transfer-operator term of one row block of an ACA cell:
//   out[item] = sum over the block's rows r of
//               al_r * (D(r, J) z(g)) + be_r * (D(r, J) z(x)).
// Rows 0..m-1 are t~ (coordinates tpc with leading dimension tld, weights
// the upward inputs inx / ing), rows m..m+k-1 the pivots I (coordinates ipc,
// weights minus the multipole vectors wx / wg).  Item = (cell, first row);
// a block has at most NT rows.
__global__ __launch_bounds__(NT) void k_tgrad(const int32_t *items, const int32_t *piv_ptr, const int32_t *jid,
                                              const int32_t *mm, const int32_t *tt_off, const double *zx,
                                              const double *zg, const double *wx, const double *wg,
                                              const double *inx, const double *ing, const double *tpc, int64_t tld,
                                              const double *ipc, int64_t npiv, const double *pts, int64_t n, int d,
                                              double prm, double *out)
{
    __shared__ double szg[KMAX], szx[KMAX];
    __shared__ double jx[KMAX], jy[KMAX], jz[KMAX];
    __shared__ double red[NT];
    const int t = threadIdx.x;
    const int64_t it = blockIdx.x;
    const int32_t c = items[2 * it], r0 = items[2 * it + 1];
    const int32_t po = piv_ptr[c], k = piv_ptr[c + 1] - po;
    for (int32_t i = t; i < k; i += NT) {
        szg[i] = zg[po + i];
        szx[i] = zx[po + i];
        const int32_t j = jid[po + i];
        jx[i] = pts[j];
        jy[i] = pts[n + j];
        jz[i] = d == 3 ? pts[2 * n + j] : 0.0;
    }
    __syncthreads();
    const int32_t m = mm[c], to = tt_off[c];
    double acc = 0.0;
    const int32_t r = r0 + t;
    if (r < m + k) {
        double px, py, pz, al, be;
        if (r < m) {
            const int64_t q = to + r;
            px = tpc[q];
            py = tpc[tld + q];
            pz = d == 3 ? tpc[2 * tld + q] : 0.0;
            al = inx[q];
            be = ing[q];
        } else {
            const int64_t q = po + (r - m);
            px = ipc[q];
            py = ipc[npiv + q];
            pz = d == 3 ? ipc[2 * npiv + q] : 0.0;
            al = -wx[q];
            be = -wg[q];
        }
        double sg = 0.0, sx = 0.0;
        for (int32_t j = 0; j < k; j++) {
            const double dx = px - jx[j], dy = py - jy[j], dz = pz - jz[j];
            const double v = kv64<K_GAUSS_DH>(dx * dx + dy * dy + dz * dz, prm);
            sg += v * szg[j];
            sx += v * szx[j];
        }
        acc = al * sg + be * sx;
    }
    red[t] = acc;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    if (t == 0) out[it] = red[0];
}

// partial dot products a . b, one per workgroup (fixed shape)
constexpr int DOT_PARTS = 256;
__global__ __launch_bounds__(NT) void k_dot_parts(int64_t n, const double *a, const double *b, double *out)
{
    __shared__ double red[NT];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)NT + t; i < n; i += (int64_t)gridDim.x * NT) s += a[i] * b[i];
    red[t] = s;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) out[blockIdx.x] = red[0];
}

// *res = (accumulate ? *res : 0) + scale * sum(terms), in a fixed order
__global__ __launch_bounds__(NT) void k_final(int64_t cnt, const double *terms, double scale, double *res,
                                              int accumulate)
{
    __shared__ double red[NT];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int64_t i = t; i < cnt; i += NT) s += terms[i];
    red[t] = s;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) *res = (accumulate ? *res : 0.0) + scale * red[0];
}

void prepare_grad(nnca_h2 *H)
{
    auto &G = H->grad;
    if (G.ready) return;
    hipStream_t s = H->stream;
    const int kap = H->kappa, lmin = H->lmin;
    const int nl = kap + 1;
    G.lu_off.assign(nl, nullptr);
    G.lu.assign(nl, nullptr);
    G.gw.assign(nl, nullptr);
    G.gu.assign(nl, nullptr);
    G.zx.assign(nl, nullptr);
    G.zg.assign(nl, nullptr);
    G.items.assign(nl, nullptr);
    G.nitems.assign(nl, 0);
    G.term_off.assign(nl + 1, 0);
    G.gs = dalloc<double>(H->n);
    G.yd = dalloc<double>(H->n);
    G.flag = dalloc<int32_t>(1);
    HIPCHECK(hipMemsetAsync(G.flag, 0, sizeof(int32_t), s));
    const double prm = 1.0 / (H->hparam * H->hparam);
    G.lu_entries = 0;
    for (int l = lmin; l <= kap; l++) {
        Level &L = H->lev[l];
        const int64_t nc = L.ncell;
        std::vector<int32_t> jid(L.npiv > 0 ? L.npiv : 1);
        if (L.npiv) HIPCHECK(hipMemcpy(jid.data(), L.jid, sizeof(int32_t) * L.npiv, hipMemcpyDeviceToHost));
        std::vector<int64_t> off(nc + 1, 0);
        int64_t po = 0;
        for (int64_t c = 0; c < nc; c++) {
            const int64_t k = L.h_k[c];
            const bool aca = k > 0 && jid[po] >= 0;
            if (aca && k > KMAX)
                fail(NNCA_ERR_NOT_SUPPORTED, "length-scale derivative supports ranks up to " + std::to_string(KMAX));
            off[c + 1] = off[c] + (aca ? k * k : 0);
            po += k;
        }
        // row blocks of NT rows over t~ and the pivots of every ACA cell
        std::vector<int32_t> items;
        po = 0;
        for (int64_t c = 0; c < nc; c++) {
            const int32_t k = L.h_k[c];
            if (k > 0 && jid[po] >= 0)
                for (int32_t r0 = 0; r0 < L.h_m[c] + k; r0 += NT) {
                    items.push_back((int32_t)c);
                    items.push_back(r0);
                }
            po += k;
        }
        G.nitems[l] = (int64_t)items.size() / 2;
        G.items[l] = dalloc<int32_t>(items.size());
        if (!items.empty())
            HIPCHECK(hipMemcpy(G.items[l], items.data(), sizeof(int32_t) * items.size(), hipMemcpyHostToDevice));
        G.zx[l] = dalloc<double>(L.npiv);
        G.zg[l] = dalloc<double>(L.npiv);
        G.lu_off[l] = dalloc<int64_t>(nc + 1);
        G.lu[l] = dalloc<double>(off[nc]);
        G.gw[l] = dalloc<double>(L.npiv);
        G.gu[l] = dalloc<double>(L.npiv);
        G.lu_entries += off[nc];
        HIPCHECK(hipMemcpyAsync(G.lu_off[l], off.data(), sizeof(int64_t) * (nc + 1), hipMemcpyHostToDevice, s));
        if (off[nc] > 0)
            k_lu<<<(int)nc, NT, 0, s>>>(L.piv_ptr, L.jid, L.pc64, L.npiv, H->pts64, H->n, H->dim, prm, G.lu_off[l],
                                        G.lu[l], G.flag);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(s));   // `off` leaves scope
    }
    int64_t nterm = 0;
    for (int l = lmin; l <= kap; l++) {
        G.term_off[l] = nterm;
        nterm += G.nitems[l];
    }
    G.term_off[nl] = nterm;
    G.nterms = nterm + DOT_PARTS;
    G.terms = dalloc<double>(G.nterms);
    int32_t bad = 0;
    HIPCHECK(hipMemcpy(&bad, G.flag, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (bad) fail(NNCA_ERR_NUMERICAL, "zero pivot in K(I, J) of the length-scale derivative");
    G.ready = true;
}

}  // namespace

void free_grad(nnca_h2 *H)
{
    auto &G = H->grad;
    for (auto p : G.lu_off) dfree(p);
    for (auto p : G.lu) dfree(p);
    for (auto p : G.gw) dfree(p);
    for (auto p : G.gu) dfree(p);
    for (auto p : G.zx) dfree(p);
    for (auto p : G.zg) dfree(p);
    for (auto p : G.items) dfree(p);
    dfree(G.gs);
    dfree(G.yd);
    dfree(G.terms);
    dfree(G.flag);
    G = nnca_h2::Grad{};
}

void run_backward(nnca_h2 *H, const double *X, const double *Gv, int64_t nrhs, int64_t ldx, int64_t ldg,
                  int precision, double *DX, int64_t lddx, double *dldh, hipStream_t s)
{
    if (!dldh) {   // the gradient with respect to x alone: A~^T G = A~ G
        run_matvec(H, Gv, DX, nrhs, ldg, lddx, NNCA_F64, precision, s);
        return;
    }
    if (H->kind != NNCA_K_GAUSS) fail(NNCA_ERR_NOT_SUPPORTED, "length-scale derivative needs the Gaussian kernel");
    if (!H->grad.ready) {
        try {
            prepare_grad(H);
        } catch (...) {
            (void)hipStreamSynchronize(H->stream);
            free_grad(H);
            throw;
        }
        HIPCHECK(hipStreamSynchronize(H->stream));
    }
    auto &G = H->grad;
    const int kap = H->kappa, lmin = H->lmin;
    const int64_t n = H->n;
    const double prm = 1.0 / (H->hparam * H->hparam);
    for (int64_t col = 0; col < nrhs; col++) {
        const double *x = X + col * ldx, *g = Gv + col * ldg;
        // 1. passes on g: A~ g (the x-gradient) and g's nested vectors
        gather_input(H, g, precision, s);
        column_passes(H, precision, H->kind, true, true, DX ? DX + col * lddx : G.yd, s);
        for (int l = lmin; l <= kap; l++) {
            const Level &L = H->lev[l];
            HIPCHECK(hipMemcpyAsync(G.gw[l], L.w64, sizeof(double) * L.npiv, hipMemcpyDeviceToDevice, s));
            HIPCHECK(hipMemcpyAsync(G.gu[l], L.u64, sizeof(double) * L.npiv, hipMemcpyDeviceToDevice, s));
        }
        HIPCHECK(hipMemcpyAsync(G.gs, H->xs64, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        // 2. upward, transverse and downward passes on x
        gather_input(H, x, precision, s);
        column_passes(H, precision, H->kind, true, false, nullptr, s);
        // 3. transfer-operator terms, level by level
        for (int l = lmin; l <= kap; l++) {
            const Level &L = H->lev[l];
            const bool leaf = l == kap;
            const double *inx = leaf ? H->xs64 : H->lev[l + 1].w64;
            const double *ing = leaf ? G.gs : G.gw[l + 1];
            const double *tpc = leaf ? H->pts64 : H->lev[l + 1].pc64;
            const int64_t tld = leaf ? n : H->lev[l + 1].npiv;
            k_tsolve<<<(int)L.ncell, NT, 0, s>>>(L.piv_ptr, L.jid, G.lu_off[l], G.lu[l], L.u64, G.gu[l], G.zx[l],
                                                 G.zg[l]);
            HIPCHECK(hipGetLastError());
            if (G.nitems[l] > 0)
                k_tgrad<<<(int)G.nitems[l], NT, 0, s>>>(G.items[l], L.piv_ptr, L.jid, L.m, L.tt_off, G.zx[l], G.zg[l],
                                                        L.w64, G.gw[l], inx, ing, tpc, tld, L.pc64, L.npiv, H->pts64,
                                                        n, H->dim, prm, G.terms + G.term_off[l]);
            HIPCHECK(hipGetLastError());
        }
        // 4. the derivative kernel in the M2L and near-field blocks on x
        //    (the multipole vectors of x are still in the levels)
        column_passes(H, precision, K_GAUSS_DH, false, true, G.yd, s);
        k_dot_parts<<<DOT_PARTS, NT, 0, s>>>(n, g, G.yd, G.terms + G.term_off[kap + 1]);
        HIPCHECK(hipGetLastError());
        k_final<<<1, NT, 0, s>>>(G.nterms, G.terms, 2.0 / H->hparam, dldh, col > 0 ? 1 : 0);
        HIPCHECK(hipGetLastError());
    }
}

}  // namespace nnca
