// NNCA pivots and transfer operators on the GPU: the single bottom-up
// traversal of Sec. 2.3.2 with one partially pivoted ACA (Sec. 2.2.1) per
// cell, symmetric case of Sec. 5, and the transfer operators from the ACA
// by-products (Remark in Sec. 2.3.2).
//
// The whole file is FP64 with contraction off: every rounding happens in the
// order written, which is the order the method is specified in, so that the
// pivot sets agree bit for bit with any other implementation of the same
// specification.  Reductions use one fixed shape: 256 partial sums (element e
// to partial e mod 256, ascending e) and the pairwise tree
// p[t] += p[t + s], s = 128, ..., 1 -- one workgroup of 256 threads per cell.
//
// Candidate sets (symmetric case): t~^{B,i} is the cell's points at a leaf and
// the concatenation of the children's t^{B_c,i} above; s~^{B,i} is the
// concatenation over B' in IL(B) (ascending) of t~^{B',i}, which equals the
// union over IL(B) of the cells' points (leaf) or of the children's pivots
// s^{B'',o} = t^{B'',i} (non-leaf).
#include <cstring>
#include <algorithm>

#include "nnca_internal.h"

#pragma clang fp contract(off)

namespace nnca {

void scan_i32(const int32_t *in, int32_t *out, int64_t n, bool inclusive, hipStream_t s);
void scan_i64(const int64_t *in, int64_t *out, int64_t n, bool inclusive, hipStream_t s);

namespace {

constexpr int NT = 256;      // threads per cell
constexpr int DOTB = 8;      // cross products reduced per pass
constexpr int COEF = 2048;   // coefficients staged in LDS
constexpr int RW = 2;        // residual columns per thread and pass
constexpr int LA = 4;        // panel rows loaded ahead in the row residual
constexpr int LU = 8;        // panel columns loaded ahead in the column residual

// log x from IEEE operations: x = m 2^e, m in (sqrt(1/2), sqrt(2)],
// log m = 2 atanh(s) with s = (m-1)/(m+1) and the series of atanh(s)/s in s^2
// up to s^24 in Horner form; log x = e ln2 + 2 s P(s^2).
__device__ double dlog(double x)
{
    int e;
    double m = frexp(x, &e);
    m = m * 2.0;
    e = e - 1;
    if (m > 0x1.6a09e667f3bcdp+0) {
        m = m * 0.5;
        e = e + 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    double p = 1.0 / 25.0;
    p = p * z + 1.0 / 23.0;
    p = p * z + 1.0 / 21.0;
    p = p * z + 1.0 / 19.0;
    p = p * z + 1.0 / 17.0;
    p = p * z + 1.0 / 15.0;
    p = p * z + 1.0 / 13.0;
    p = p * z + 1.0 / 11.0;
    p = p * z + 1.0 / 9.0;
    p = p * z + 1.0 / 7.0;
    p = p * z + 1.0 / 5.0;
    p = p * z + 1.0 / 3.0;
    p = p * z + 1.0;
    return (double)e * 0x1.62e42fefa39efp-1 + (2.0 * s) * p;
}

// exp x (x <= 0) from IEEE operations: x = n ln2 + r with ln2 as a 32-bit head
// plus a tail, Taylor polynomial of degree 13 in Horner form, times 2^n.
__device__ double dexp(double x)
{
    if (x < -745.5) return 0.0;
    if (x > 709.0) return INFINITY;
    double nn = floor(x * 0x1.71547652b82fep+0 + 0.5);
    double r = (x - nn * 0x1.62e42fee00000p-1) - nn * 0x1.a39ef35793c76p-33;
    double p = 1.0 / 6227020800.0;
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 1.0 / 2.0;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)nn);
}

// K(a, b) in FP64 as the method specifies it: squared distance accumulated
// axis by axis, 1/sqrt and log r = log(r^2)/2 set to zero at r = 0.
__device__ inline double kval(int kind, double hh, int d, double ax, double ay, double az, double bx,
                              double by, double bz)
{
    double dx = ax - bx;
    double s = dx * dx;
    double dy = ay - by;
    s = s + dy * dy;
    if (d == 3) {
        double dz = az - bz;
        s = s + dz * dz;
    }
    if (kind == NNCA_K_INV_R) return s == 0.0 ? 0.0 : 1.0 / sqrt(s);
    if (kind == NNCA_K_LOG_R) return s == 0.0 ? 0.0 : 0.5 * dlog(s);
    if (kind == NNCA_K_INV_REG) {   // hh = a
        if (s == 0.0) return 0.0;
        return s >= hh * hh ? hh / sqrt(s) : sqrt(s) / hh;
    }
    if (kind == NNCA_K_LOG_REG) {   // hh = a
        if (s == 0.0) return 0.0;
        const double la = dlog(hh);
        return s >= hh * hh ? (0.5 * dlog(s)) / la : (sqrt(s) * (0.5 * dlog(s) - 1.0)) / (hh * (la - 1.0));
    }
    if (kind == NNCA_K_EXP_R) return dexp(-(sqrt(s) / hh));   // hh = h
    return dexp(-(s / hh));
}

// the kernel parameter kval takes: the Gaussian h^2, the regularised
// kernels their a
inline double aca_param(int kind, double hparam) { return kind == NNCA_K_GAUSS ? hparam * hparam : hparam; }

__global__ void k_debug_kernel(int kind, double hh, int d, const double *a, const double *b, int64_t cnt,
                               double *out)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    out[i] = kval(kind, hh, d, a[i], a[cnt + i], d == 3 ? a[2 * cnt + i] : 0.0, b[i], b[cnt + i],
                  d == 3 ? b[2 * cnt + i] : 0.0);
}

// ----------------------------------------------------------------------------
// candidate sizes

// m_B and the start of t~ (tree order at a leaf, else inside piv_id of l+1)
__global__ void k_level_m(int64_t nc, int leaf, const int32_t *first, const int32_t *count,
                          const int32_t *child_first, const int32_t *child_count, const int32_t *cpiv_ptr,
                          int32_t *m, int32_t *tt_off)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    if (leaf) {
        m[c] = count[c];
        tt_off[c] = first[c];
    } else {
        int32_t f = child_first[c], e = f + child_count[c];
        tt_off[c] = cpiv_ptr[f];
        m[c] = cpiv_ptr[e] - cpiv_ptr[f];
    }
}

// n_B = sum over IL(B) of m_B'
__global__ void k_level_n(int64_t nc, const int32_t *il_ptr, const int32_t *il, const int32_t *m, int64_t *n)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int64_t s = 0;
    for (int32_t e = il_ptr[c]; e < il_ptr[c + 1]; e++) s += m[il[e]];
    n[c] = s;
}

}  // namespace

// per-cell work description of one ACA chunk
struct AcaCell {
    int64_t s_off;    // candidate columns (sid, sc)
    int64_t u_off;    // U panel, m x kcap, column l at u_off + l m
    int64_t v_off;    // V panel, kcap x n, row l at v_off + l n
    int64_t f_off;    // row flags (m bytes) then column flags (n bytes)
    int64_t r_off;    // row map (m int32) for the transfer solve
    int64_t cap_off;  // pivot slots (kcap, or m for a cell kept whole)
    int32_t m, n, kcap, whole;
    int32_t tt_off;
    int32_t kfull;    // min(m, n): the largest rank the cell can reach
};

namespace {

// s~ of every cell of the chunk: ids and FP64 coordinates, in candidate order
__global__ void k_gather_cand(const AcaCell *cells, int32_t cell0, const int32_t *il_ptr, const int32_t *il,
                              const int32_t *m, const int32_t *tt_off, const int32_t *tsrc,
                              const double *P, int64_t np, int d, int32_t *sid, double *sc, int64_t ntot)
{
    const AcaCell C = cells[blockIdx.x];
    if (C.whole) return;
    int32_t c = cell0 + blockIdx.x;
    int64_t pos = C.s_off;
    for (int32_t e = il_ptr[c]; e < il_ptr[c + 1]; e++) {
        int32_t b = il[e];
        int32_t mb = m[b], to = tt_off[b];
        for (int32_t i = threadIdx.x; i < mb; i += blockDim.x) {
            int32_t id = tsrc ? tsrc[to + i] : to + i;
            sid[pos + i] = id;
            sc[pos + i] = P[id];
            sc[ntot + pos + i] = P[np + id];
            sc[2 * ntot + pos + i] = d == 3 ? P[2 * np + id] : 0.0;
        }
        pos += mb;
    }
}

__device__ inline void tree_sum(double *a, int t)
{
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s) a[t] = a[t] + a[t + s];
        __syncthreads();
    }
}

// argmax of (value, index): larger value wins, equal values go to the
// smaller index
__device__ inline void tree_argmax(double *v, int32_t *ix, int t)
{
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (t < s) {
            double a = v[t], b = v[t + s];
            int32_t ia = ix[t], ib = ix[t + s];
            if (b > a || (b == a && ib < ia)) { v[t] = b; ix[t] = ib; }
        }
        __syncthreads();
    }
}

// One partially pivoted ACA per workgroup (Sec. 2.2.1).  Step k:
//  1. residual of row i_k:  R(c) = K(i_k, c) - sum_{l<k} u_l(i_k) v_l(c)
//  2. j_k = argmax over unused columns of |R|; if the maximum is zero the row
//     is marked used and the smallest unused row is tried instead
//  3. v_k = R / R(j_k), zero at used columns
//  4. u_k(r) = K(r, j_k) - sum_{l<k} v_l(j_k) u_l(r), zero at used rows
//  5. ||A^(k)||^2 = (||A^(k-1)||^2 + 2 sum_{l<k} (u_k.u_l)(v_l.v_k)) + |u_k|^2 |v_k|^2
//  6. stop when |u_k| |v_k| <= tol ||A^(k)|| (the cross is kept) or k = min(m, n)
//  7. i_{k+1} = argmax over unused rows of |u_k|
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_aca(const AcaCell *cells, int32_t cell0, const double *P, int64_t np,
                                             int d, const int32_t *tsrc, const int32_t *sid,
                                             const double *sc, int64_t ntot, double *U, double *V,
                                             uint8_t *flags, int kind, double hh, double tol, int32_t *k_out,
                                             int32_t *ipos_cap, int32_t *jid_cap)
{
    const AcaCell C = cells[blockIdx.x];
    const int t = threadIdx.x;
    const int32_t cell = cell0 + blockIdx.x;
    if (C.whole) {
        for (int32_t q = t; q < C.m; q += NT) {
            ipos_cap[C.cap_off + q] = q;
            jid_cap[C.cap_off + q] = -1;
        }
        if (t == 0) k_out[cell] = C.m;
        return;
    }
    __shared__ double sv[NT];
    __shared__ int32_t si[NT];
    __shared__ double su2[NT], sv2[NT];
    __shared__ double red[DOTB][NT];   // cross-term partials: the u side, then the v side
    __shared__ double ured[DOTB];
    __shared__ double coef[COEF];
    __shared__ int32_t s_row, s_k, s_stop, s_jk, s_over;

    const int32_t m = C.m, n = C.n, kcap = C.kcap;
    if (kcap == 0) {
        if (t == 0) k_out[cell] = 0;
        return;
    }
    double *Uc = U + C.u_off;
    double *Vc = V + C.v_off;
    uint8_t *rf = flags + C.f_off;
    uint8_t *cf = rf + m;
    const double *sx = sc + C.s_off, *sy = sc + ntot + C.s_off, *sz = sc + 2 * ntot + C.s_off;
    for (int32_t r = t; r < m; r += NT) rf[r] = 0;
    for (int32_t j = t; j < n; j += NT) cf[j] = 0;
    if (t == 0) { s_row = 0; s_k = 0; s_stop = 0; s_over = 0; }
    double nrm2 = 0.0;   // meaningful in thread 0
    __syncthreads();
    int32_t k = 0;
    for (;;) {
        const int32_t i = s_row;
        const int32_t pid = tsrc ? tsrc[C.tt_off + i] : C.tt_off + i;
        const double ax = P[pid], ay = P[np + pid], az = d == 3 ? P[2 * np + pid] : 0.0;
        for (int32_t l = t; l < k && l < COEF; l += NT) coef[l] = Uc[(int64_t)l * m + i];
        __syncthreads();
        // 1-2: row residual and its argmax over unused columns.  Each thread
        // runs RW columns side by side (independent chains, every column
        // still accumulated in ascending l) and scans them in ascending j.
        double best = 0.0;
        int32_t bj = INT32_MAX;
        double *Rk = Vc + (int64_t)k * n;
        for (int32_t j0 = t; j0 < n; j0 += RW * NT) {
            double r[RW];
#pragma unroll
            for (int c = 0; c < RW; c++) {
                int32_t j = j0 + c * NT;
                r[c] = j < n ? kval(kind, hh, d, ax, ay, az, sx[j], sy[j], sz[j]) : 0.0;
            }
            const int nv = (n - j0 + NT - 1) / NT < RW ? (n - j0 + NT - 1) / NT : RW;
            if (nv == RW) {
                // LA rows of the panel in flight: their loads are issued
                // before the updates, which still run in ascending l for
                // every column
                int32_t l = 0;
                for (; l + LA - 1 < k; l += LA) {
                    double ul[LA], a[LA][RW];
#pragma unroll
                    for (int q = 0; q < LA; q++) {
                        ul[q] = l + q < COEF ? coef[l + q] : Uc[(int64_t)(l + q) * m + i];
                        const double *Vl = Vc + (int64_t)(l + q) * n + j0;
#pragma unroll
                        for (int c = 0; c < RW; c++) a[q][c] = Vl[c * NT];
                    }
#pragma unroll
                    for (int q = 0; q < LA; q++)
#pragma unroll
                        for (int c = 0; c < RW; c++) r[c] = r[c] - ul[q] * a[q][c];
                }
                for (; l < k; l++) {
                    double ul = l < COEF ? coef[l] : Uc[(int64_t)l * m + i];
                    const double *Vl = Vc + (int64_t)l * n + j0;
#pragma unroll
                    for (int c = 0; c < RW; c++) r[c] = r[c] - ul * Vl[c * NT];
                }
            } else {
                for (int32_t l = 0; l < k; l++) {
                    double ul = l < COEF ? coef[l] : Uc[(int64_t)l * m + i];
                    const double *Vl = Vc + (int64_t)l * n + j0;
                    for (int c = 0; c < nv; c++) r[c] = r[c] - ul * Vl[c * NT];
                }
            }
            for (int c = 0; c < nv; c++) {
                int32_t j = j0 + c * NT;
                Rk[j] = r[c];
                if (!cf[j]) {
                    double a = fabs(r[c]);
                    if (a > best) { best = a; bj = j; }
                }
            }
        }
        sv[t] = best;
        si[t] = bj;
        __syncthreads();
        tree_argmax(sv, si, t);
        const int32_t jk = si[0];
        if (jk == INT32_MAX) {
            // zero residual row: mark it and continue with the smallest unused row
            if (t == 0) rf[i] = 1;
            __syncthreads();
            int32_t cand = INT32_MAX;
            for (int32_t r = t; r < m; r += NT)
                if (!rf[r] && r < cand) cand = r;
            sv[t] = 0.0;
            si[t] = cand;
            __syncthreads();
            tree_argmax(sv, si, t);
            if (si[0] == INT32_MAX) break;
            if (t == 0) s_row = si[0];
            __syncthreads();
            continue;
        }
        const double piv = Rk[jk];
        __syncthreads();
        // 3: v_k
        double pv = 0.0;
        for (int32_t j = t; j < n; j += NT) {
            double v = cf[j] ? 0.0 : Rk[j] / piv;
            Rk[j] = v;
            pv = pv + v * v;
        }
        for (int32_t l = t; l < k && l < COEF; l += NT) coef[l] = Vc[(int64_t)l * n + jk];
        __syncthreads();
        // 4: u_k and the argmax for the next row
        const double bx = sx[jk], by = sy[jk], bz = sz[jk];
        double *uk = Uc + (int64_t)k * m;
        double pu = 0.0;
        double ub = -1.0;
        int32_t bi = INT32_MAX;
        for (int32_t r = t; r < m; r += NT) {
            double u = 0.0;
            if (!rf[r]) {
                int32_t rid = tsrc ? tsrc[C.tt_off + r] : C.tt_off + r;
                u = kval(kind, hh, d, P[rid], P[np + rid], d == 3 ? P[2 * np + rid] : 0.0, bx, by, bz);
                int32_t l = 0;
                for (; l + LU - 1 < k; l += LU) {   // LU loads in flight, updates in ascending l
                    double vl[LU], a[LU];
#pragma unroll
                    for (int q = 0; q < LU; q++) {
                        vl[q] = l + q < COEF ? coef[l + q] : Vc[(int64_t)(l + q) * n + jk];
                        a[q] = Uc[(int64_t)(l + q) * m + r];
                    }
#pragma unroll
                    for (int q = 0; q < LU; q++) u = u - vl[q] * a[q];
                }
                for (; l < k; l++) {
                    double vl = l < COEF ? coef[l] : Vc[(int64_t)l * n + jk];
                    u = u - vl * Uc[(int64_t)l * m + r];
                }
            }
            uk[r] = u;
            pu = pu + u * u;
            if (!rf[r] && r != i) {
                double a = fabs(u);
                if (a > ub) { ub = a; bi = r; }
            }
        }
        su2[t] = pu;
        sv2[t] = pv;
        sv[t] = ub;
        si[t] = bi;
        __syncthreads();
        for (int s = NT / 2; s > 0; s >>= 1) {
            if (t < s) {
                su2[t] = su2[t] + su2[t + s];
                sv2[t] = sv2[t] + sv2[t + s];
                double a = sv[t], b = sv[t + s];
                int32_t ia = si[t], ib = si[t + s];
                if (b > a || (b == a && ib < ia)) { sv[t] = b; si[t] = ib; }
            }
            __syncthreads();
        }
        const double ukk = su2[0], vkk = sv2[0];
        const int32_t next = si[0];
        // 5: cross terms, DOTB at a time
        double s = 0.0;
        for (int32_t lb = 0; lb < k; lb += DOTB) {
            int nbat = k - lb < DOTB ? k - lb : DOTB;
            double au[DOTB], av[DOTB];
#pragma unroll
            for (int q = 0; q < DOTB; q++) { au[q] = 0.0; av[q] = 0.0; }
            for (int32_t r = t; r < m; r += NT) {
                double x = uk[r];
#pragma unroll
                for (int q = 0; q < DOTB; q++)
                    if (q < nbat) au[q] = au[q] + x * Uc[(int64_t)(lb + q) * m + r];
            }
            int32_t j = t;
            for (; j < n; j += NT) {
                double x = Rk[j];
#pragma unroll
                for (int q = 0; q < DOTB; q++)
                    if (q < nbat) av[q] = av[q] + Vc[(int64_t)(lb + q) * n + j] * x;
            }
            // the pairwise trees of the u partials, then of the v partials,
            // in one LDS buffer
#pragma unroll
            for (int q = 0; q < DOTB; q++) red[q][t] = au[q];
            __syncthreads();
            for (int st = NT / 2; st > 0; st >>= 1) {
                if (t < st)
                    for (int q = 0; q < nbat; q++) red[q][t] = red[q][t] + red[q][t + st];
                __syncthreads();
            }
            if (t < DOTB) ured[t] = red[t][0];
            __syncthreads();
#pragma unroll
            for (int q = 0; q < DOTB; q++) red[q][t] = av[q];
            __syncthreads();
            for (int st = NT / 2; st > 0; st >>= 1) {
                if (t < st)
                    for (int q = 0; q < nbat; q++) red[q][t] = red[q][t] + red[q][t + st];
                __syncthreads();
            }
            if (t == 0)
                for (int q = 0; q < nbat; q++) s = s + ured[q] * red[q][0];
            __syncthreads();
        }
        // 6: bookkeeping and the stopping rule (thread 0)
        if (t == 0) {
            nrm2 = (nrm2 + 2.0 * s) + ukk * vkk;
            if (nrm2 < 0.0) nrm2 = 0.0;
            ipos_cap[C.cap_off + k] = i;
            jid_cap[C.cap_off + k] = sid[C.s_off + jk];
            rf[i] = 1;
            cf[jk] = 1;
            int32_t kn = k + 1;
            bool conv = sqrt(ukk) * sqrt(vkk) <= tol * sqrt(nrm2);
            int stop = conv || kn >= kcap || next == INT32_MAX;
            // the panel was sized below min(m, n): the cell is run again with room for it
            if (!conv && next != INT32_MAX && kn >= kcap && kcap < C.kfull) s_over = 1;
            s_k = kn;
            s_stop = stop;
            s_row = next;
        }
        __syncthreads();
        k = s_k;
        if (s_stop) break;
    }
    if (t == 0) k_out[cell] = s_over ? -1 : k;
}

// ----------------------------------------------------------------------------
// The same ACA spread over many workgroups per cell, for levels whose cells
// are few and long (the coarse levels: hundreds of cells with 10^4-10^5
// candidate columns, where one workgroup per cell leaves the chip idle).
// The cells of a chunk advance in lockstep; each step is five launches:
//   row    (column segments x cells)  1-2: the residual of row i_k on a
//          segment of columns, and the segment's argmax over unused columns;
//   pivot  (cells)  the argmax over the segments; a zero row is marked used
//          and the smallest unused row taken instead (the step is redone);
//          else 4: u_k, |u_k|^2, the next row, and u_k . u_l for l < k;
//   scale  (column segments x cells)  3: v_k = R / R(j_k), zero at used columns;
//   cross  (groups x cells)  |v_k|^2 and v_l . v_k for l < k;
//   finish (cells)  5-7: the norm update and the stopping rule.
// Every column's residual is formed by one thread, every dot product by one
// workgroup in the fixed shape, and every argmax keeps the larger value and
// then the smaller index, exactly as in k_aca: the pivots are the same bit
// for bit.

struct AcaState {
    int32_t i, k, stop, over, jk, next, retry, pad;
    double nrm2, piv, ukk, vkk;
};

constexpr int MSEG = 1024;   // columns per row / scale workgroup (four per thread)
constexpr int MRW = MSEG / NT;

__global__ __launch_bounds__(NT) void k_acm_init(const AcaCell *cells, int32_t cell0, AcaState *st, uint8_t *flags,
                                                 int32_t *k_out, int32_t *ipos_cap, int32_t *jid_cap)
{
    const AcaCell C = cells[blockIdx.x];
    const int t = threadIdx.x;
    const int32_t cell = cell0 + blockIdx.x;
    AcaState *S = st + blockIdx.x;
    if (C.whole) {
        for (int32_t q = t; q < C.m; q += NT) {
            ipos_cap[C.cap_off + q] = q;
            jid_cap[C.cap_off + q] = -1;
        }
        if (t == 0) {
            k_out[cell] = C.m;
            S->stop = 1;
        }
        return;
    }
    if (C.kcap == 0) {
        if (t == 0) {
            k_out[cell] = 0;
            S->stop = 1;
        }
        return;
    }
    uint8_t *rf = flags + C.f_off;
    uint8_t *cf = rf + C.m;
    for (int32_t r = t; r < C.m; r += NT) rf[r] = 0;
    for (int32_t j = t; j < C.n; j += NT) cf[j] = 0;
    if (t == 0) {
        S->i = 0;
        S->k = 0;
        S->stop = 0;
        S->over = 0;
        S->jk = INT32_MAX;
        S->next = INT32_MAX;
        S->retry = 0;
        S->nrm2 = 0.0;
    }
}

// 1-2 on columns [blockIdx.x MSEG, (blockIdx.x + 1) MSEG) of cell blockIdx.y
__global__ __launch_bounds__(NT) void k_acm_row(const AcaCell *cells, const AcaState *st, const double *P,
                                                int64_t np, int d, const int32_t *tsrc, const double *sc,
                                                int64_t ntot, const double *U, double *V, const uint8_t *flags,
                                                int kind, double hh, double *segv, int32_t *segi, int32_t nsegmax)
{
    const AcaCell C = cells[blockIdx.y];
    const AcaState S = st[blockIdx.y];
    const int32_t j0 = blockIdx.x * MSEG;
    if (C.whole || S.stop || j0 >= C.n) return;   // uniform for the workgroup
    __shared__ double coef[COEF];
    __shared__ double sv[NT];
    __shared__ int32_t si[NT];
    const int t = threadIdx.x;
    const int32_t m = C.m, n = C.n, k = S.k, i = S.i;
    const double *Uc = U + C.u_off;
    double *Vc = V + C.v_off;
    const uint8_t *cf = flags + C.f_off + m;
    const double *sx = sc + C.s_off, *sy = sc + ntot + C.s_off, *sz = sc + 2 * ntot + C.s_off;
    const int32_t pid = tsrc ? tsrc[C.tt_off + i] : C.tt_off + i;
    const double ax = P[pid], ay = P[np + pid], az = d == 3 ? P[2 * np + pid] : 0.0;
    for (int32_t l = t; l < k && l < COEF; l += NT) coef[l] = Uc[(int64_t)l * m + i];
    __syncthreads();
    const int32_t j1 = n - j0 < MSEG ? n : j0 + MSEG;
    const int32_t jb = j0 + t;
    double r[MRW];
#pragma unroll
    for (int c = 0; c < MRW; c++) {
        const int32_t j = jb + c * NT;
        r[c] = j < j1 ? kval(kind, hh, d, ax, ay, az, sx[j], sy[j], sz[j]) : 0.0;
    }
    if (jb + (MRW - 1) * NT < j1) {
        int32_t l = 0;
        for (; l + LA - 1 < k; l += LA) {   // LA rows in flight, updates in ascending l
            double ul[LA], a[LA][MRW];
#pragma unroll
            for (int q = 0; q < LA; q++) {
                ul[q] = l + q < COEF ? coef[l + q] : Uc[(int64_t)(l + q) * m + i];
                const double *Vl = Vc + (int64_t)(l + q) * n + jb;
#pragma unroll
                for (int c = 0; c < MRW; c++) a[q][c] = Vl[c * NT];
            }
#pragma unroll
            for (int q = 0; q < LA; q++)
#pragma unroll
                for (int c = 0; c < MRW; c++) r[c] = r[c] - ul[q] * a[q][c];
        }
        for (; l < k; l++) {
            const double ul = l < COEF ? coef[l] : Uc[(int64_t)l * m + i];
            const double *Vl = Vc + (int64_t)l * n + jb;
#pragma unroll
            for (int c = 0; c < MRW; c++) r[c] = r[c] - ul * Vl[c * NT];
        }
    } else {
        for (int32_t l = 0; l < k; l++) {
            const double ul = l < COEF ? coef[l] : Uc[(int64_t)l * m + i];
            const double *Vl = Vc + (int64_t)l * n;
#pragma unroll
            for (int c = 0; c < MRW; c++) {
                const int32_t j = jb + c * NT;
                if (j < j1) r[c] = r[c] - ul * Vl[j];
            }
        }
    }
    double best = 0.0;
    int32_t bj = INT32_MAX;
    double *Rk = Vc + (int64_t)k * n;
#pragma unroll
    for (int c = 0; c < MRW; c++) {
        const int32_t j = jb + c * NT;
        if (j < j1) {
            Rk[j] = r[c];
            if (!cf[j]) {
                const double a = fabs(r[c]);
                if (a > best) { best = a; bj = j; }
            }
        }
    }
    sv[t] = best;
    si[t] = bj;
    __syncthreads();
    tree_argmax(sv, si, t);
    if (t == 0) {
        segv[(int64_t)blockIdx.y * nsegmax + blockIdx.x] = sv[0];
        segi[(int64_t)blockIdx.y * nsegmax + blockIdx.x] = si[0];
    }
}

// the pivot of the step, then 4 (u_k) and the u side of the cross terms
__global__ __launch_bounds__(NT) void k_acm_pivot(const AcaCell *cells, int32_t cell0, AcaState *st, const double *P,
                                                  int64_t np, int d, const int32_t *tsrc, const double *sc,
                                                  int64_t ntot, double *U, const double *V, uint8_t *flags, int kind,
                                                  double hh, const double *segv, const int32_t *segi,
                                                  int32_t nsegmax, double *uu, int32_t kcapmax, int32_t *k_out)
{
    const AcaCell C = cells[blockIdx.x];
    AcaState *S = st + blockIdx.x;
    if (C.whole || S->stop) return;   // uniform
    __shared__ double sv[NT];
    __shared__ int32_t si[NT];
    __shared__ double su2[NT];
    __shared__ double red[DOTB][NT];
    __shared__ double coef[COEF];
    const int t = threadIdx.x;
    const int32_t m = C.m, n = C.n, k = S->k, i = S->i;
    double *Uc = U + C.u_off;
    const double *Vc = V + C.v_off;
    uint8_t *rf = flags + C.f_off;
    const int32_t nseg = (n + MSEG - 1) / MSEG;
    double bv = 0.0;
    int32_t bi = INT32_MAX;
    for (int32_t q = t; q < nseg; q += NT) {
        const double v = segv[(int64_t)blockIdx.x * nsegmax + q];
        const int32_t ix = segi[(int64_t)blockIdx.x * nsegmax + q];
        if (v > bv || (v == bv && ix < bi)) { bv = v; bi = ix; }
    }
    sv[t] = bv;
    si[t] = bi;
    __syncthreads();
    tree_argmax(sv, si, t);
    const int32_t jk = si[0];
    __syncthreads();
    if (jk == INT32_MAX) {
        // zero residual row: mark it and continue with the smallest unused row
        if (t == 0) rf[i] = 1;
        __syncthreads();
        int32_t cand = INT32_MAX;
        for (int32_t r = t; r < m; r += NT)
            if (!rf[r] && r < cand) cand = r;
        sv[t] = 0.0;
        si[t] = cand;
        __syncthreads();
        tree_argmax(sv, si, t);
        if (t == 0) {
            if (si[0] == INT32_MAX) {
                S->stop = 1;
                k_out[cell0 + blockIdx.x] = S->over ? -1 : k;
            } else {
                S->i = si[0];
                S->retry = 1;
            }
        }
        return;
    }
    const double *Rk = Vc + (int64_t)k * n;
    const double piv = Rk[jk];
    for (int32_t l = t; l < k && l < COEF; l += NT) coef[l] = Vc[(int64_t)l * n + jk];
    __syncthreads();
    const double bx = sc[C.s_off + jk], by = sc[ntot + C.s_off + jk], bz = sc[2 * ntot + C.s_off + jk];
    double *uk = Uc + (int64_t)k * m;
    double pu = 0.0;
    double ub = -1.0;
    int32_t bu = INT32_MAX;
    for (int32_t r = t; r < m; r += NT) {
        double u = 0.0;
        if (!rf[r]) {
            const int32_t rid = tsrc ? tsrc[C.tt_off + r] : C.tt_off + r;
            u = kval(kind, hh, d, P[rid], P[np + rid], d == 3 ? P[2 * np + rid] : 0.0, bx, by, bz);
            int32_t l = 0;
            for (; l + LU - 1 < k; l += LU) {
                double vl[LU], a[LU];
#pragma unroll
                for (int q = 0; q < LU; q++) {
                    vl[q] = l + q < COEF ? coef[l + q] : Vc[(int64_t)(l + q) * n + jk];
                    a[q] = Uc[(int64_t)(l + q) * m + r];
                }
#pragma unroll
                for (int q = 0; q < LU; q++) u = u - vl[q] * a[q];
            }
            for (; l < k; l++) {
                const double vl = l < COEF ? coef[l] : Vc[(int64_t)l * n + jk];
                u = u - vl * Uc[(int64_t)l * m + r];
            }
        }
        uk[r] = u;
        pu = pu + u * u;
        if (!rf[r] && r != i) {
            const double a = fabs(u);
            if (a > ub) { ub = a; bu = r; }
        }
    }
    su2[t] = pu;
    sv[t] = ub;
    si[t] = bu;
    __syncthreads();
    for (int st2 = NT / 2; st2 > 0; st2 >>= 1) {
        if (t < st2) {
            su2[t] = su2[t] + su2[t + st2];
            const double a = sv[t], b = sv[t + st2];
            const int32_t ia = si[t], ib = si[t + st2];
            if (b > a || (b == a && ib < ia)) { sv[t] = b; si[t] = ib; }
        }
        __syncthreads();
    }
    if (t == 0) {
        S->jk = jk;
        S->piv = piv;
        S->ukk = su2[0];
        S->next = si[0];
    }
    // u_k . u_l for l < k, DOTB at a time
    double *uuc = uu + (int64_t)blockIdx.x * kcapmax;
    for (int32_t lb = 0; lb < k; lb += DOTB) {
        const int nbat = k - lb < DOTB ? k - lb : DOTB;
        double au[DOTB];
#pragma unroll
        for (int q = 0; q < DOTB; q++) au[q] = 0.0;
        for (int32_t r = t; r < m; r += NT) {
            const double x = uk[r];
#pragma unroll
            for (int q = 0; q < DOTB; q++)
                if (q < nbat) au[q] = au[q] + x * Uc[(int64_t)(lb + q) * m + r];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < DOTB; q++) red[q][t] = au[q];
        __syncthreads();
        for (int st2 = NT / 2; st2 > 0; st2 >>= 1) {
            if (t < st2)
                for (int q = 0; q < nbat; q++) red[q][t] = red[q][t] + red[q][t + st2];
            __syncthreads();
        }
        if (t < nbat) uuc[lb + t] = red[t][0];
    }
}

// 3: v_k on a segment of columns
__global__ __launch_bounds__(NT) void k_acm_scale(const AcaCell *cells, const AcaState *st, double *V,
                                                  const uint8_t *flags)
{
    const AcaCell C = cells[blockIdx.y];
    const AcaState S = st[blockIdx.y];
    const int32_t j0 = blockIdx.x * MSEG;
    if (C.whole || S.stop || S.retry || j0 >= C.n) return;
    const int32_t n = C.n;
    const uint8_t *cf = flags + C.f_off + C.m;
    double *Rk = V + C.v_off + (int64_t)S.k * n;
    const double piv = S.piv;
    const int32_t j1 = n - j0 < MSEG ? n : j0 + MSEG;
    for (int32_t j = j0 + threadIdx.x; j < j1; j += NT) Rk[j] = cf[j] ? 0.0 : Rk[j] / piv;
}

// group 0: |v_k|^2; group g > 0: v_l . v_k for l in [(g - 1) DOTB, g DOTB) below k
__global__ __launch_bounds__(NT) void k_acm_cross(const AcaCell *cells, AcaState *st, const double *V, double *vv,
                                                  int32_t kcapmax)
{
    const AcaCell C = cells[blockIdx.y];
    AcaState *S = st + blockIdx.y;
    const int32_t k = S->k;
    const int32_t lb = ((int32_t)blockIdx.x - 1) * DOTB;
    if (C.whole || S->stop || S->retry || (blockIdx.x > 0 && lb >= k)) return;
    __shared__ double red[DOTB][NT];
    const int t = threadIdx.x;
    const int32_t n = C.n;
    const double *Vc = V + C.v_off;
    const double *vk = Vc + (int64_t)k * n;
    if (blockIdx.x == 0) {
        double pv = 0.0;
        for (int32_t j = t; j < n; j += NT) {
            const double v = vk[j];
            pv = pv + v * v;
        }
        red[0][t] = pv;
        __syncthreads();
        for (int st2 = NT / 2; st2 > 0; st2 >>= 1) {
            if (t < st2) red[0][t] = red[0][t] + red[0][t + st2];
            __syncthreads();
        }
        if (t == 0) S->vkk = red[0][0];
        return;
    }
    const int nbat = k - lb < DOTB ? k - lb : DOTB;
    double av[DOTB];
#pragma unroll
    for (int q = 0; q < DOTB; q++) av[q] = 0.0;
    for (int32_t j = t; j < n; j += NT) {
        const double x = vk[j];
#pragma unroll
        for (int q = 0; q < DOTB; q++)
            if (q < nbat) av[q] = av[q] + Vc[(int64_t)(lb + q) * n + j] * x;
    }
#pragma unroll
    for (int q = 0; q < DOTB; q++) red[q][t] = av[q];
    __syncthreads();
    for (int st2 = NT / 2; st2 > 0; st2 >>= 1) {
        if (t < st2)
            for (int q = 0; q < nbat; q++) red[q][t] = red[q][t] + red[q][t + st2];
        __syncthreads();
    }
    if (t < nbat) vv[(int64_t)blockIdx.y * kcapmax + lb + t] = red[t][0];
}

// 5-7 (one thread per cell)
__global__ void k_acm_finish(int32_t cn, const AcaCell *cells, int32_t cell0, AcaState *st, const int32_t *sid,
                             uint8_t *flags, const double *uu, const double *vv, int32_t kcapmax, double tol,
                             int32_t *k_out, int32_t *ipos_cap, int32_t *jid_cap)
{
    const int32_t cb = blockIdx.x * blockDim.x + threadIdx.x;
    if (cb >= cn) return;
    const AcaCell C = cells[cb];
    AcaState *S = st + cb;
    if (C.whole || S->stop) return;
    if (S->retry) {
        S->retry = 0;
        return;
    }
    const int32_t k = S->k, i = S->i, jk = S->jk;
    const double *uuc = uu + (int64_t)cb * kcapmax, *vvc = vv + (int64_t)cb * kcapmax;
    double s = 0.0;
    for (int32_t l = 0; l < k; l++) s = s + uuc[l] * vvc[l];
    const double ukk = S->ukk, vkk = S->vkk;
    double nrm2 = (S->nrm2 + 2.0 * s) + ukk * vkk;
    if (nrm2 < 0.0) nrm2 = 0.0;
    S->nrm2 = nrm2;
    ipos_cap[C.cap_off + k] = i;
    jid_cap[C.cap_off + k] = sid[C.s_off + jk];
    uint8_t *rf = flags + C.f_off;
    rf[i] = 1;
    rf[C.m + jk] = 1;
    const int32_t kn = k + 1, next = S->next;
    const bool conv = sqrt(ukk) * sqrt(vkk) <= tol * sqrt(nrm2);
    const int stop = conv || kn >= C.kcap || next == INT32_MAX;
    if (!conv && next != INT32_MAX && kn >= C.kcap && C.kcap < C.kfull) S->over = 1;
    S->k = kn;
    S->i = next;
    S->stop = stop;
    if (stop) k_out[cell0 + cb] = S->over ? -1 : kn;
}

__global__ void k_acm_active(int32_t cn, const AcaState *st, int32_t *cnt)
{
    const int32_t cb = blockIdx.x * blockDim.x + threadIdx.x;
    if (cb < cn && !st[cb].stop) atomicAdd(cnt, 1);
}

// Transfer operator C_B = U L^{-1}, L = U(I, :) (Remark in Sec. 2.3.2).  The
// pivot rows of C_B are the identity and are not stored; every other row x
// solves x L = U(r, :) from the last column down:
//   x(c) = (U(r, c) - sum_{l=c+1}^{k-1} x(l) L(l, c)) / L(c, c).
__global__ __launch_bounds__(NT) void k_transfer(const AcaCell *cells, int32_t cell0, const int32_t *k_lvl,
                                                  const int32_t *ipos_cap, const double *U, int32_t *rowmap,
                                                  const int64_t *rem_base, const int64_t *crem_base,
                                                  int32_t *rem_pos, double *crem, int *zero_pivot)
{
    const AcaCell C = cells[blockIdx.x];
    if (C.whole) return;
    const int t = threadIdx.x;
    const int32_t m = C.m, k = k_lvl[cell0 + blockIdx.x];
    const int32_t *ip = ipos_cap + C.cap_off;
    int32_t *rm = rowmap + C.r_off;
    const double *Uc = U + C.u_off;
    int32_t *rp = rem_pos + rem_base[blockIdx.x];
    double *X = crem + crem_base[blockIdx.x];
    for (int32_t r = t; r < m; r += NT) rm[r] = -1;
    __syncthreads();
    for (int32_t q = t; q < k; q += NT) rm[ip[q]] = q;
    __syncthreads();
    __shared__ int32_t sc[NT];
    int32_t base = 0;
    for (int32_t r0 = 0; r0 < m; r0 += NT) {
        int32_t r = r0 + t;
        int32_t f = (r < m && rm[r] < 0) ? 1 : 0;
        sc[t] = f;
        __syncthreads();
        for (int s = 1; s < NT; s <<= 1) {
            int32_t v = t >= s ? sc[t - s] : 0;
            __syncthreads();
            sc[t] += v;
            __syncthreads();
        }
        if (f) rp[base + sc[t] - 1] = r;
        int32_t tot = sc[NT - 1];
        __syncthreads();
        base += tot;
    }
    __syncthreads();
    const int32_t nrem = m - k;
    for (int32_t q = t; q < nrem; q += NT) {
        int32_t r = rp[q];
        double *x = X + (int64_t)q * k;
        for (int32_t c = k - 1; c >= 0; c--) {
            const double *Ucol = Uc + (int64_t)c * m;
            double acc = Ucol[r];
            for (int32_t l = c + 1; l < k; l++) acc = acc - x[l] * Ucol[ip[l]];
            double dg = Ucol[ip[c]];
            if (dg == 0.0) *zero_pivot = 1;
            x[c] = acc / dg;
        }
    }
}

// compact the per-cell pivot slots into the level arrays
__global__ void k_compact_pivots(int64_t nc, const int64_t *cap_off, const int32_t *piv_ptr,
                                 const int32_t *tt_off, const int32_t *tsrc, const int32_t *ipos_cap,
                                 const int32_t *jid_cap, int32_t *ipos, int32_t *jid, int32_t *piv_id)
{
    int64_t c = blockIdx.x;
    if (c >= nc) return;
    int32_t b = piv_ptr[c], k = piv_ptr[c + 1] - b;
    int64_t co = cap_off[c];
    for (int32_t q = threadIdx.x; q < k; q += blockDim.x) {
        int32_t p = ipos_cap[co + q];
        ipos[b + q] = p;
        jid[b + q] = jid_cap[co + q];
        piv_id[b + q] = tsrc ? tsrc[tt_off[c] + p] : tt_off[c] + p;
    }
}

}  // namespace

void debug_kernel_eval(int kind, double hparam, int dim, const double *a, const double *b, int64_t count,
                       double *out, hipStream_t s)
{
    double *da = dalloc<double>(3 * count), *db = dalloc<double>(3 * count), *dout = dalloc<double>(count);
    HIPCHECK(hipMemsetAsync(da, 0, sizeof(double) * 3 * count, s));
    HIPCHECK(hipMemsetAsync(db, 0, sizeof(double) * 3 * count, s));
    HIPCHECK(hipMemcpyAsync(da, a, sizeof(double) * dim * count, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(db, b, sizeof(double) * dim * count, hipMemcpyHostToDevice, s));
    k_debug_kernel<<<grid_for(count, 256), 256, 0, s>>>(kind, aca_param(kind, hparam), dim, da, db, count, dout);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(out, dout, sizeof(double) * count, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    dfree(da);
    dfree(db);
    dfree(dout);
}

// One half of the cells' pivots.  The symmetric case has one: the rows are
// the cell's own points (or the children's pivots), the columns those of the
// interaction list.  The general case P != Q has two, whose candidate sets
// are crossed (Sec. 2.3.2): the incoming half's rows are targets (P) and its
// columns the IL region's rows of the outgoing half (sources: a leaf's Q
// points, else the IL children's s^{B'',o}); the outgoing half's rows are
// sources and its columns the IL region's rows of the incoming half (targets:
// a leaf's P points, else t^{B'',i}).  The outgoing ACA therefore runs on the
// transposed block, its first pivot among the cell's own sources, and its
// C = U~ L^{-1} is V_B (leaf) or the stacked T_{B B_c}^T.  Its entries are
// evaluated as K(q, p); for the radial kernels here that is K(p, q) bit for
// bit (the coordinate differences change sign exactly).
struct Half {
    std::vector<Level> *lv;
    const double *pts;   // 3 x n, this half's tree order
    int64_t n;
};

// Levels with fewer cells than this run the ACA spread over many workgroups
// per cell (k_acm_*): there one workgroup per cell would leave most of the
// chip idle while it waits on its panel loads.
constexpr int64_t ACA_SPREAD_BELOW = 8192;

// The steps of the spread ACA for the cells [c0, c1) of a chunk, in lockstep
// until every cell has stopped.
static void aca_spread(nnca_h2 *H, const AcaCell *dcells, const std::vector<AcaCell> &hc, int64_t c0, int64_t c1,
                       const Half &own, const int32_t *tsrc, const int32_t *sid, const double *sc,
                       int64_t ntot, double *U, double *V, uint8_t *fl, int32_t *k_out, int32_t *ipos_cap,
                       int32_t *jid_cap)
{
    hipStream_t s = H->stream;
    const int32_t cn = (int32_t)(c1 - c0);
    int32_t nsegmax = 1, kcapmax = 1, mmax = 1;
    for (int64_t c = c0; c < c1; c++) {
        if (hc[c].whole) continue;
        nsegmax = std::max(nsegmax, (hc[c].n + MSEG - 1) / MSEG);
        kcapmax = std::max(kcapmax, hc[c].kcap);
        mmax = std::max(mmax, hc[c].m);
    }
    AcaState *st = dalloc<AcaState>(cn);
    double *segv = dalloc<double>((size_t)cn * nsegmax);
    int32_t *segi = dalloc<int32_t>((size_t)cn * nsegmax);
    double *uu = dalloc<double>((size_t)cn * kcapmax);
    double *vv = dalloc<double>((size_t)cn * kcapmax);
    int32_t *cnt = dalloc<int32_t>(1);
    const double hh = aca_param(H->kind, H->hparam);
    try {
        k_acm_init<<<cn, NT, 0, s>>>(dcells, (int32_t)c0, st, fl, k_out, ipos_cap, jid_cap);
        HIPCHECK(hipGetLastError());
        // every step advances k or uses up a row of the cell: at most m + kcap steps
        const int64_t max_steps = (int64_t)mmax + kcapmax + 2;
        for (int64_t step = 0;; step++) {
            k_acm_row<<<dim3(nsegmax, cn), NT, 0, s>>>(dcells, st, own.pts, own.n, H->dim, tsrc, sc, ntot, U, V, fl,
                                                      H->kind, hh, segv, segi, nsegmax);
            k_acm_pivot<<<cn, NT, 0, s>>>(dcells, (int32_t)c0, st, own.pts, own.n, H->dim, tsrc, sc, ntot, U, V, fl,
                                          H->kind, hh, segv, segi, nsegmax, uu, kcapmax, k_out);
            k_acm_scale<<<dim3(nsegmax, cn), NT, 0, s>>>(dcells, st, V, fl);
            const int64_t kbound = std::min<int64_t>(step, kcapmax);   // k <= step
            const unsigned ngrp = (unsigned)(1 + (kbound + DOTB - 1) / DOTB);
            k_acm_cross<<<dim3(ngrp, cn), NT, 0, s>>>(dcells, st, V, vv, kcapmax);
            k_acm_finish<<<grid_for(cn, 64), 64, 0, s>>>(cn, dcells, (int32_t)c0, st, sid, fl, uu, vv, kcapmax,
                                                         H->tol, k_out, ipos_cap, jid_cap);
            HIPCHECK(hipGetLastError());
            if (step % 8 == 7 || step >= max_steps) {
                int32_t h = 0;
                HIPCHECK(hipMemsetAsync(cnt, 0, sizeof(int32_t), s));
                k_acm_active<<<grid_for(cn, 256), 256, 0, s>>>(cn, st, cnt);
                HIPCHECK(hipGetLastError());
                HIPCHECK(hipMemcpyAsync(&h, cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
                HIPCHECK(hipStreamSynchronize(s));
                if (h == 0) break;
                if (step >= max_steps) fail(NNCA_ERR_INTERNAL, "spread ACA did not stop");
            }
        }
    } catch (...) {
        (void)hipStreamSynchronize(s);
        dfree(st); dfree(segv); dfree(segi); dfree(uu); dfree(vv); dfree(cnt);
        throw;
    }
    HIPCHECK(hipStreamSynchronize(s));
    dfree(st); dfree(segv); dfree(segi); dfree(uu); dfree(vv); dfree(cnt);
}

// step 1 of Sec. 2.3.2 for one half: m_B and the start of t~
static void level_sizes(nnca_h2 *H, std::vector<Level> &lv, int l)
{
    hipStream_t s = H->stream;
    Level &L = lv[l];
    const int64_t nc = L.ncell;
    const bool leaf = (l == H->kappa);
    L.m = dalloc<int32_t>(nc);
    L.tt_off = dalloc<int32_t>(nc);
    k_level_m<<<grid_for(nc, 256), 256, 0, s>>>(nc, leaf, L.first, L.count, L.child_first, L.child_count,
                                               leaf ? nullptr : lv[l + 1].piv_ptr, L.m, L.tt_off);
    HIPCHECK(hipGetLastError());
}

// Step 2 of Sec. 2.3.2 for one half of a level (all of its cells): the rows
// of `own`, the columns gathered from the interaction lists' rows of `far`
// (the same half in the symmetric case).  level_sizes has run for both.
static void build_level(nnca_h2 *H, int l, const Half &own, const Half &far)
{
    hipStream_t s = H->stream;
    Level &L = (*own.lv)[l];
    const Level &Lf = (*far.lv)[l];
    const int64_t nc = L.ncell;
    const bool leaf = (l == H->kappa);
    const int32_t *tsrc = leaf ? nullptr : (*own.lv)[l + 1].piv_id;
    const int32_t *ftsrc = leaf ? nullptr : (*far.lv)[l + 1].piv_id;

    int64_t *nn = dalloc<int64_t>(nc);
    k_level_n<<<grid_for(nc, 256), 256, 0, s>>>(nc, L.il_ptr, L.il, Lf.m, nn);
    HIPCHECK(hipGetLastError());
    std::vector<int32_t> hm(nc), htt(nc);
    std::vector<int64_t> hn(nc);
    HIPCHECK(hipMemcpyAsync(hm.data(), L.m, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(htt.data(), L.tt_off, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(hn.data(), nn, sizeof(int64_t) * nc, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    dfree(nn);
    L.h_m = hm;

    // per-cell work and chunks bounded by the workspace budget
    std::vector<AcaCell> hc(nc);
    std::vector<int64_t> bytes(nc);
    int64_t sum_cap = 0;
    std::vector<int64_t> cap_off(nc + 1, 0);
    for (int64_t c = 0; c < nc; c++) {
        AcaCell &a = hc[c];
        std::memset(&a, 0, sizeof(a));
        a.m = hm[c];
        if (hn[c] > INT32_MAX) fail(NNCA_ERR_NOT_SUPPORTED, "candidate set larger than 2^31");
        a.n = (int32_t)hn[c];
        a.tt_off = htt[c];
        a.whole = (a.n == 0 || (H->policy == 1 && a.n < a.m)) ? 1 : 0;
        a.kfull = std::min(a.m, a.n);
        a.kcap = a.whole ? a.m : (leaf ? a.kfull : std::min(a.kfull, H->rank_reserve));
        cap_off[c] = sum_cap;
        a.cap_off = sum_cap;
        sum_cap += a.whole ? a.m : a.kfull;
    }
    auto cell_bytes = [&](const AcaCell &a) -> int64_t {
        return a.whole ? 64
                       : (int64_t)a.n * (4 + 24) + ((int64_t)a.m * a.kcap + (int64_t)a.kcap * a.n) * 8 +
                             (int64_t)a.m * 5 + a.n + 256;
    };
    for (int64_t c = 0; c < nc; c++) bytes[c] = cell_bytes(hc[c]);
    cap_off[nc] = sum_cap;
    int32_t *ipos_cap = dalloc<int32_t>(sum_cap);
    int32_t *jid_cap = dalloc<int32_t>(sum_cap);
    L.k = dalloc<int32_t>(nc);
    int64_t budget = H->ws_budget;
    if (budget <= 0) {
        size_t fr = 0, tot = 0;
        HIPCHECK(hipMemGetInfo(&fr, &tot));
        budget = (int64_t)(fr * 0.6);
        if (budget > ((int64_t)96 << 30)) budget = (int64_t)96 << 30;
    }

    std::vector<int32_t> hk(nc, 0);
    std::vector<int32_t *> rem_chunks;
    std::vector<double *> crem_chunks;
    std::vector<int64_t> rem_cnt, crem_cnt;
    AcaCell *dcells = nullptr;
    int zp_host = 0;
    int *zp = dalloc<int>(1);
    HIPCHECK(hipMemsetAsync(zp, 0, sizeof(int), s));

    int64_t c0 = 0;
    while (c0 < nc) {
        // chunk [c0, c1)
        int64_t c1 = c0, acc = 0;
        while (c1 < nc && (c1 == c0 || acc + bytes[c1] <= budget) && c1 - c0 < 65535) { acc += bytes[c1]; c1++; }
        int64_t cn = c1 - c0;
        int64_t so = 0, uo = 0, vo = 0, fo = 0, ro = 0;
        for (int64_t c = c0; c < c1; c++) {
            AcaCell &a = hc[c];
            if (a.whole) continue;
            a.s_off = so; so += a.n;
            a.u_off = uo; uo += (int64_t)a.m * a.kcap;
            a.v_off = vo; vo += (int64_t)a.kcap * a.n;
            a.f_off = fo; fo += a.m + a.n;
            a.r_off = ro; ro += a.m;
        }
        if (!dcells || true) {
            if (dcells) dfree(dcells);
            dcells = dalloc<AcaCell>(cn);
        }
        HIPCHECK(hipMemcpyAsync(dcells, hc.data() + c0, sizeof(AcaCell) * cn, hipMemcpyHostToDevice, s));
        int32_t *sid = dalloc<int32_t>(so);
        double *sc = dalloc<double>(3 * so);
        double *U = dalloc<double>(uo);
        double *V = dalloc<double>(vo);
        uint8_t *fl = dalloc<uint8_t>(fo);
        int32_t *rowmap = dalloc<int32_t>(ro);
        k_gather_cand<<<(int)cn, 256, 0, s>>>(dcells, (int32_t)c0, L.il_ptr, L.il, Lf.m, Lf.tt_off, ftsrc, far.pts,
                                              far.n, H->dim, sid, sc, so);
        HIPCHECK(hipGetLastError());
        if (nc < ACA_SPREAD_BELOW)
            aca_spread(H, dcells, hc, c0, c1, own, tsrc, sid, sc, so, U, V, fl, L.k, ipos_cap, jid_cap);
        else
            k_aca<<<(int)cn, NT, 0, s>>>(dcells, (int32_t)c0, own.pts, own.n, H->dim, tsrc, sid, sc, so, U, V, fl,
                                         H->kind, aca_param(H->kind, H->hparam), H->tol, L.k, ipos_cap, jid_cap);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipMemcpyAsync(hk.data() + c0, L.k + c0, sizeof(int32_t) * cn, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        // cells whose rank outgrew the reserved panel: widen them and redo the chunk
        bool again = false;
        for (int64_t c = c0; c < c1; c++)
            if (hk[c] < 0) {
                hc[c].kcap = hc[c].kfull;
                bytes[c] = cell_bytes(hc[c]);
                again = true;
            }
        if (again) {
            dfree(sid); dfree(sc); dfree(U); dfree(V); dfree(fl); dfree(rowmap);
            continue;
        }
        // remainder rows of this chunk
        std::vector<int64_t> rb(cn), cb(cn);
        int64_t rt = 0, ct = 0;
        for (int64_t c = c0; c < c1; c++) {
            rb[c - c0] = rt;
            cb[c - c0] = ct;
            if (!hc[c].whole) {
                rt += hc[c].m - hk[c];
                ct += (int64_t)(hc[c].m - hk[c]) * hk[c];
            }
        }
        int64_t *drb = dalloc<int64_t>(cn), *dcb = dalloc<int64_t>(cn);
        HIPCHECK(hipMemcpyAsync(drb, rb.data(), sizeof(int64_t) * cn, hipMemcpyHostToDevice, s));
        HIPCHECK(hipMemcpyAsync(dcb, cb.data(), sizeof(int64_t) * cn, hipMemcpyHostToDevice, s));
        int32_t *rp = dalloc<int32_t>(rt);
        double *cr = dalloc<double>(ct);
        k_transfer<<<(int)cn, NT, 0, s>>>(dcells, (int32_t)c0, L.k, ipos_cap, U, rowmap, drb, dcb, rp, cr, zp);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(s));
        rem_chunks.push_back(rp);
        crem_chunks.push_back(cr);
        rem_cnt.push_back(rt);
        crem_cnt.push_back(ct);
        dfree(drb); dfree(dcb);
        dfree(sid); dfree(sc); dfree(U); dfree(V); dfree(fl); dfree(rowmap);
        c0 = c1;
    }
    if (dcells) dfree(dcells);
    HIPCHECK(hipMemcpy(&zp_host, zp, sizeof(int), hipMemcpyDeviceToHost));
    dfree(zp);
    if (zp_host) fail(NNCA_ERR_NUMERICAL, "zero pivot in a transfer-operator solve");

    // level layout of pivots and operators
    std::vector<int32_t> pp(nc + 1, 0), rpp(nc + 1, 0);
    std::vector<int64_t> cpp(nc + 1, 0);
    int32_t kmx = 0;
    for (int64_t c = 0; c < nc; c++) {
        pp[c + 1] = pp[c] + hk[c];
        int32_t nr = hc[c].whole ? 0 : hc[c].m - hk[c];
        rpp[c + 1] = rpp[c] + nr;
        cpp[c + 1] = cpp[c] + (int64_t)nr * hk[c];
        kmx = std::max(kmx, hk[c]);
        L.max_nrem = std::max(L.max_nrem, nr);
    }
    L.h_k = hk;
    // algorithmic panel traffic: step k of a cell reads its k V rows of n
    // entries twice (row residual, cross terms)
    for (int64_t c = 0; c < nc; c++)
        if (!hc[c].whole) H->aca_panel_bytes += (double)hk[c] * (double)(hk[c] - 1) * (double)hc[c].n * 8.0;
    L.max_k = kmx;
    L.npiv = pp[nc];
    L.ncrem = cpp[nc];
    L.piv_ptr = dalloc<int32_t>(nc + 1);
    L.rem_ptr = dalloc<int32_t>(nc + 1);
    L.crem_off = dalloc<int64_t>(nc + 1);
    HIPCHECK(hipMemcpyAsync(L.piv_ptr, pp.data(), sizeof(int32_t) * (nc + 1), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(L.rem_ptr, rpp.data(), sizeof(int32_t) * (nc + 1), hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(L.crem_off, cpp.data(), sizeof(int64_t) * (nc + 1), hipMemcpyHostToDevice, s));
    L.rem_pos = dalloc<int32_t>(rpp[nc]);
    L.crem64 = dalloc<double>(cpp[nc]);
    int64_t ro = 0, co = 0;
    for (size_t q = 0; q < rem_chunks.size(); q++) {
        if (rem_cnt[q]) HIPCHECK(hipMemcpyAsync(L.rem_pos + ro, rem_chunks[q], sizeof(int32_t) * rem_cnt[q], hipMemcpyDeviceToDevice, s));
        if (crem_cnt[q]) HIPCHECK(hipMemcpyAsync(L.crem64 + co, crem_chunks[q], sizeof(double) * crem_cnt[q], hipMemcpyDeviceToDevice, s));
        ro += rem_cnt[q];
        co += crem_cnt[q];
    }
    HIPCHECK(hipStreamSynchronize(s));
    for (auto p : rem_chunks) dfree(p);
    for (auto p : crem_chunks) dfree(p);

    int64_t *dcap = dalloc<int64_t>(nc + 1);
    HIPCHECK(hipMemcpyAsync(dcap, cap_off.data(), sizeof(int64_t) * (nc + 1), hipMemcpyHostToDevice, s));
    L.ipos = dalloc<int32_t>(L.npiv);
    L.jid = dalloc<int32_t>(L.npiv);
    L.piv_id = dalloc<int32_t>(L.npiv);
    k_compact_pivots<<<(int)nc, 64, 0, s>>>(nc, dcap, L.piv_ptr, L.tt_off, tsrc, ipos_cap, jid_cap, L.ipos, L.jid,
                                          L.piv_id);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(s));
    dfree(dcap);
    dfree(ipos_cap);
    dfree(jid_cap);
    L.has_piv = true;
}

void build_pivots(nnca_h2 *H)
{
    if (!H->general) {
        const Half one{&H->lev, H->pts64, H->n};
        for (int l = H->kappa; l >= H->lmin; l--) {
            level_sizes(H, H->lev, l);
            build_level(H, l, one, one);
        }
        return;
    }
    const Half in{&H->lev, H->pts64, H->n}, out{&H->lev_o, H->qpts64, H->nq};
    for (int l = H->kappa; l >= H->lmin; l--) {
        level_sizes(H, H->lev, l);
        level_sizes(H, H->lev_o, l);
        build_level(H, l, in, out);
        build_level(H, l, out, in);
    }
}

}  // namespace nnca
