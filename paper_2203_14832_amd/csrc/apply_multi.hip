// H2 matrix-vector product for many right-hand sides (Sec. 4 passes applied
// to an N x R block).  Vectors are held in tree order with the R columns
// innermost and padded to RP = 16 * NCB columns, so one source row of weights
// is contiguous.
//
// Transverse pass, mixed precision, finest levels (two for 1/r, one for the
// other kernels, as for one column): the kernel tile
// K(t^{B,i}, sources) is generated in FP32 on the vector ALUs, one entry per
// lane in the A-operand layout of v_mfma_f32_16x16x4f32, and multiplied by the
// weight tile (4 sources x 16 columns) on the matrix cores, R/16 products per
// generated tile; FP32 accumulators are folded into FP64 every 4 steps
// (16 sources).
// FP64 and the coarse levels of the mixed form use v_mfma_f64_16x16x4f64 on an
// FP64 kernel tile; the near field uses the matrix cores as well.  Precision
// scheme as for one column.
#include <cstring>
#include <algorithm>
#include <type_traits>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>

#include "nnca_internal.h"
#include "kernel_values.h"

namespace nnca {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
constexpr int NT = 256;

// Input gather for RP columns: X (original order, column-major, leading
// dimension ldx) to row-major tree order, zero columns past R, and the
// x_hi / x_lo split of the mixed form.  A workgroup takes 64 consecutive
// original indices: it reads each column's 64 entries (contiguous) into LDS,
// then writes each point's row of RP values at its tree position.
template <typename TI>
__global__ __launch_bounds__(256) void k_gather_multi(int64_t n, int R, int RP, const int32_t *rank, const TI *X,
                                                      int64_t ldx, double *xs, float *hi, float *lo)
{
    __shared__ double tile[64 * 65];   // [point][column], rows padded against bank conflicts
    const int t = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    const int jn = n - j0 < 64 ? (int)(n - j0) : 64;
    {
        const int jj = t & 63;
        for (int c = t >> 6; c < RP; c += 4)
            tile[jj * 65 + c] = (c < R && jj < jn) ? (double)X[(int64_t)c * ldx + j0 + jj] : 0.0;
    }
    __syncthreads();
    const int ppr = 256 / RP;   // rows written per round
    if (t >= ppr * RP) return;
    const int c = t % RP;
    for (int jj = t / RP; jj < jn; jj += ppr) {
        const double v = tile[jj * 65 + c];
        const int64_t i = (int64_t)rank[j0 + jj] * RP + c;
        xs[i] = v;
        if (hi) {
            const float h = (float)v;
            hi[i] = h;
            lo[i] = (float)(v - (double)h);
        }
    }
}

// Output scatter for RP columns, the converse of the gather: the row-major
// tree-order result to Y (original order, column-major, leading dimension
// ldy), columns below R.  A workgroup reads the rows of 64 consecutive
// original indices (contiguous) into LDS and writes each column's 64 entries
// (contiguous).
template <typename TO>
__global__ __launch_bounds__(256) void k_scatter_multi(int64_t n, int R, int RP, const int32_t *rank, const double *yt,
                                                       TO *Y, int64_t ldy)
{
    __shared__ double tile[64 * 65];
    const int t = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    const int jn = n - j0 < 64 ? (int)(n - j0) : 64;
    const int ppr = 256 / RP;
    if (t < ppr * RP) {
        const int c = t % RP;
        for (int jj = t / RP; jj < jn; jj += ppr) tile[jj * 65 + c] = yt[(int64_t)rank[j0 + jj] * RP + c];
    }
    __syncthreads();
    const int jj = t & 63;
    if (jj < jn)
        for (int c = t >> 6; c < R; c += 4) Y[(int64_t)c * ldy + j0 + jj] = (TO)tile[jj * 65 + c];
}

// Transfer passes for RP columns (Sec. 4).  One wavefront per (cell, 64 rows,
// 16 columns): every lane keeps the 16 sums of its row in registers, the
// matrix entries of the wave's 64 rows are contiguous in memory, and the
// vector entry each step multiplies is the same for the whole wave (one
// address).  The flat grid numbers the items of a cell consecutively, so the
// column blocks of one cell re-read its matrix block from the cache.

// upward pass: w_q = x~(ipos_q) + sum_r C(r, q) x~(rem_pos_r) over the rows of
// t~ that are not pivots (C holds those rows of C_B, (m - k) x k row-major)
__global__ __launch_bounds__(64) void k_up_multi(int ipc, int RP, const int32_t *piv_ptr, const int32_t *tt_off,
                                                 const int32_t *ipos, const int32_t *rem_ptr, const int32_t *rem_pos,
                                                 const int64_t *crem_off, const double *__restrict__ crem,
                                                 const double *__restrict__ xin, double *__restrict__ w)
{
    const int64_t c = blockIdx.x / ipc;
    const int item = (int)(blockIdx.x % ipc), ncb = RP / 16;
    const int32_t qc = item / ncb, cb = item % ncb;
    const int32_t po = piv_ptr[c], kk = piv_ptr[c + 1] - po;
    if (qc * 64 >= kk) return;   // uniform for the wavefront
    const int32_t to = tt_off[c], ro = rem_ptr[c], nr = rem_ptr[c + 1] - ro;
    const int32_t q = qc * 64 + (int32_t)threadIdx.x, qs = q < kk ? q : kk - 1;
    const double *xb = xin + cb * 16;
    double acc[16];
    {
        const double2 *xp = reinterpret_cast<const double2 *>(xb + (int64_t)(to + ipos[po + qs]) * RP);
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const double2 v = xp[j];
            acc[2 * j] = v.x;
            acc[2 * j + 1] = v.y;
        }
    }
    const double *Cq = crem + crem_off[c] + qs;
#pragma unroll 2
    for (int32_t r = 0; r < nr; r++) {
        const double cv = Cq[(int64_t)r * kk];
        const double *xr = xb + (int64_t)(to + rem_pos[ro + r]) * RP;
#pragma unroll
        for (int j = 0; j < 16; j++) acc[j] = fma(cv, xr[j], acc[j]);
    }
    if (q < kk) {
        double2 *wp = reinterpret_cast<double2 *>(w + (int64_t)(po + q) * RP + cb * 16);
#pragma unroll
        for (int j = 0; j < 8; j++) wp[j] = make_double2(acc[2 * j], acc[2 * j + 1]);
    }
}

// downward pass: the stacked C_B u added to the children (L2L) or written as
// the far field of the leaf's points (L2P).  Items [0, nqc * ncb) of a cell
// copy u to the pivot rows of t~; the others form sum_q C(r, q) u_q for the
// other rows from the transposed blocks (crem_t, k x (m - k) row-major).
__global__ __launch_bounds__(64) void k_down_multi(int ipc, int nqc, int RP, const int32_t *piv_ptr,
                                                   const int32_t *tt_off, const int32_t *ipos, const int32_t *rem_ptr,
                                                   const int32_t *rem_pos, const int64_t *crem_off,
                                                   const double *__restrict__ crem_t, const double *__restrict__ u,
                                                   double *__restrict__ out, int accumulate)
{
    const int64_t c = blockIdx.x / ipc;
    int item = (int)(blockIdx.x % ipc);
    const int ncb = RP / 16, lane = threadIdx.x;
    const int32_t po = piv_ptr[c], kk = piv_ptr[c + 1] - po, to = tt_off[c];
    if (item < nqc * ncb) {
        const int32_t qc = item / ncb, cb = item % ncb, q = qc * 64 + lane;
        if (q >= kk) return;
        const double2 *up = reinterpret_cast<const double2 *>(u + (int64_t)(po + q) * RP + cb * 16);
        double2 *op = reinterpret_cast<double2 *>(out + (int64_t)(to + ipos[po + q]) * RP + cb * 16);
#pragma unroll
        for (int j = 0; j < 8; j++) {
            double2 v = up[j];
            if (accumulate) {
                const double2 o = op[j];
                v.x += o.x;
                v.y += o.y;
            }
            op[j] = v;
        }
        return;
    }
    item -= nqc * ncb;
    const int32_t rc = item / ncb, cb = item % ncb;
    const int32_t ro = rem_ptr[c], nr = rem_ptr[c + 1] - ro;
    if (rc * 64 >= nr) return;   // uniform for the wavefront
    const int32_t r = rc * 64 + lane, rs = r < nr ? r : nr - 1;
    const double *Ct = crem_t + crem_off[c] + rs;
    const double *ub = u + (int64_t)po * RP + cb * 16;
    double acc[16];
#pragma unroll
    for (int j = 0; j < 16; j++) acc[j] = 0.0;
#pragma unroll 2
    for (int32_t q = 0; q < kk; q++) {
        const double cv = Ct[(int64_t)q * nr];
        const double *uq = ub + (int64_t)q * RP;
#pragma unroll
        for (int j = 0; j < 16; j++) acc[j] = fma(cv, uq[j], acc[j]);
    }
    if (r < nr) {
        double2 *op = reinterpret_cast<double2 *>(out + (int64_t)(to + rem_pos[ro + r]) * RP + cb * 16);
#pragma unroll
        for (int j = 0; j < 8; j++) {
            double2 v = make_double2(acc[2 * j], acc[2 * j + 1]);
            if (accumulate) {
                const double2 o = op[j];
                v.x += o.x;
                v.y += o.y;
            }
            op[j] = v;
        }
    }
}

// The same passes for levels with few items: four wavefronts per item, each
// taking every fourth term of the sum; the partial sums are added in order
// through LDS.
constexpr int SPLIT_WAVES = 4;

__device__ inline void add_split_partials(double (&acc)[16], int wv, int lane, double *red)
{
    if (wv > 0)
#pragma unroll
        for (int j = 0; j < 16; j++) red[((wv - 1) * 16 + j) * 64 + lane] = acc[j];
    __syncthreads();
    if (wv == 0)
        for (int w2 = 1; w2 < SPLIT_WAVES; w2++)
#pragma unroll
            for (int j = 0; j < 16; j++) acc[j] += red[((w2 - 1) * 16 + j) * 64 + lane];
}

__global__ __launch_bounds__(64 * SPLIT_WAVES) void k_up_multi_split(
    int ipc, int RP, const int32_t *piv_ptr, const int32_t *tt_off, const int32_t *ipos, const int32_t *rem_ptr,
    const int32_t *rem_pos, const int64_t *crem_off, const double *__restrict__ crem,
    const double *__restrict__ xin, double *__restrict__ w)
{
    __shared__ double red[(SPLIT_WAVES - 1) * 16 * 64];
    const int64_t c = blockIdx.x / ipc;
    const int item = (int)(blockIdx.x % ipc), ncb = RP / 16;
    const int32_t qc = item / ncb, cb = item % ncb;
    const int32_t po = piv_ptr[c], kk = piv_ptr[c + 1] - po;
    if (qc * 64 >= kk) return;   // uniform for the workgroup
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int32_t to = tt_off[c], ro = rem_ptr[c], nr = rem_ptr[c + 1] - ro;
    const int32_t q = qc * 64 + lane, qs = q < kk ? q : kk - 1;
    const double *xb = xin + cb * 16;
    double acc[16];
#pragma unroll
    for (int j = 0; j < 16; j++) acc[j] = 0.0;
    const double *Cq = crem + crem_off[c] + qs;
#pragma unroll 2
    for (int32_t r = wv; r < nr; r += SPLIT_WAVES) {
        const double cv = Cq[(int64_t)r * kk];
        const double *xr = xb + (int64_t)(to + rem_pos[ro + r]) * RP;
#pragma unroll
        for (int j = 0; j < 16; j++) acc[j] = fma(cv, xr[j], acc[j]);
    }
    add_split_partials(acc, wv, lane, red);
    if (wv == 0 && q < kk) {
        const double2 *xp = reinterpret_cast<const double2 *>(xb + (int64_t)(to + ipos[po + q]) * RP);
        double2 *wp = reinterpret_cast<double2 *>(w + (int64_t)(po + q) * RP + cb * 16);
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const double2 v = xp[j];
            wp[j] = make_double2(v.x + acc[2 * j], v.y + acc[2 * j + 1]);
        }
    }
}

__global__ __launch_bounds__(64 * SPLIT_WAVES) void k_down_multi_split(
    int ipc, int nqc, int RP, const int32_t *piv_ptr, const int32_t *tt_off, const int32_t *ipos,
    const int32_t *rem_ptr, const int32_t *rem_pos, const int64_t *crem_off, const double *__restrict__ crem_t,
    const double *__restrict__ u, double *__restrict__ out, int accumulate)
{
    __shared__ double red[(SPLIT_WAVES - 1) * 16 * 64];
    const int64_t c = blockIdx.x / ipc;
    int item = (int)(blockIdx.x % ipc);
    const int ncb = RP / 16, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int32_t po = piv_ptr[c], kk = piv_ptr[c + 1] - po, to = tt_off[c];
    if (item < nqc * ncb) {
        const int32_t qc = item / ncb, cb = item % ncb, q = qc * 64 + lane;
        if (wv > 0 || q >= kk) return;
        const double2 *up = reinterpret_cast<const double2 *>(u + (int64_t)(po + q) * RP + cb * 16);
        double2 *op = reinterpret_cast<double2 *>(out + (int64_t)(to + ipos[po + q]) * RP + cb * 16);
#pragma unroll
        for (int j = 0; j < 8; j++) {
            double2 v = up[j];
            if (accumulate) {
                const double2 o = op[j];
                v.x += o.x;
                v.y += o.y;
            }
            op[j] = v;
        }
        return;
    }
    item -= nqc * ncb;
    const int32_t rc = item / ncb, cb = item % ncb;
    const int32_t ro = rem_ptr[c], nr = rem_ptr[c + 1] - ro;
    if (rc * 64 >= nr) return;   // uniform for the workgroup
    const int32_t r = rc * 64 + lane, rs = r < nr ? r : nr - 1;
    const double *Ct = crem_t + crem_off[c] + rs;
    const double *ub = u + (int64_t)po * RP + cb * 16;
    double acc[16];
#pragma unroll
    for (int j = 0; j < 16; j++) acc[j] = 0.0;
#pragma unroll 2
    for (int32_t q = wv; q < kk; q += SPLIT_WAVES) {
        const double cv = Ct[(int64_t)q * nr];
        const double *uq = ub + (int64_t)q * RP;
#pragma unroll
        for (int j = 0; j < 16; j++) acc[j] = fma(cv, uq[j], acc[j]);
    }
    add_split_partials(acc, wv, lane, red);
    if (wv == 0 && r < nr) {
        double2 *op = reinterpret_cast<double2 *>(out + (int64_t)(to + rem_pos[ro + r]) * RP + cb * 16);
#pragma unroll
        for (int j = 0; j < 8; j++) {
            double2 v = make_double2(acc[2 * j], acc[2 * j + 1]);
            if (accumulate) {
                const double2 o = op[j];
                v.x += o.x;
                v.y += o.y;
            }
            op[j] = v;
        }
    }
}

// index of the interaction-list entry holding source s of the cell (the
// largest e in [e0, e1) with pre[e] <= s)
__device__ inline int32_t list_entry(const int32_t *pre, int32_t e0, int32_t e1, int32_t s)
{
    int32_t lo = e0, hi = e1 - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= s) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// transfer-pass launches with fewer items than this take the four-wavefront
// kernels
constexpr unsigned SPLIT_BELOW = 2048;
// interaction-list entries staged in LDS at a time.  128 with the row stride
// RP + 4 below keeps the 64-column transverse kernel under 40 KB of LDS, so
// four workgroups (four waves per SIMD) fit on a CU: c3 (64 columns) 4.03
// against 4.21 ms per block matvec with 256 entries and stride RP + 16
// (48.6 KB, three workgroups); c5 unchanged
constexpr int MET = 128;

__global__ void k_to_f32(int64_t cnt, const double *a, float *b)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < cnt) b[i] = (float)a[i];
}

// M2L, FP32 on the matrix cores.  Four wavefronts; each takes a unit of TB
// blocks of 16 targets (TB = 2 for up to 32 columns: one source step then
// feeds two kernel values per lane into two matrix products that share the
// weight operand), or, with fewer than four units, a phase of the 4-source
// steps of one unit.  With one column block the kernel fits six waves per
// SIMD in 80 registers (the matrix products then accumulate in ordinary
// vector registers).  TSEL = 1 halves the sources per LDS tile (a tile
// shape the autotuner may pick per level).
template <int KIND, int NCB, int TSEL>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NCB == 1 ? 6 : 2))) void k_m2l_mfma(int64_t nc, int P, const int32_t *k, const int32_t *piv_ptr,
                                                 const int32_t *il_ptr, const int32_t *il, const int32_t *ilpre,
                                                 const int32_t *ilsum, const float *pc, int64_t npiv,
                                                 const int32_t *coord, const float *hc, float h0, int d,
                                                 const float *w32, int R, double *u, double *part_out, float prm)
{
    constexpr int RP = NCB * 16;
    constexpr int TB = NCB <= 2 ? 2 : 1;             // target blocks per wavefront
    constexpr int TS = (NCB == 1 ? 256 : 128) >> TSEL;   // sources per LDS tile
    static_assert(TS % 64 == 0 && TS <= NT, "the tile pads to a multiple of 64 sources, one per thread");
    constexpr int SW = (NCB & 1) ? RP : RP + 4;   // LDS row stride (even widths padded by four)
    constexpr int RED = NT * NCB * 4 * TB;           // doubles of the phase reduction
    __shared__ float4 sx[TS];
    __shared__ int32_t sidx[TS];
    __shared__ __align__(16) double swt_raw[TS * SW / 2 > RED ? TS * SW / 2 : RED];
    __shared__ int32_t est[MET + 1], ebase[MET];
    __shared__ float esh[3][MET];
    float *swt = reinterpret_cast<float *>(swt_raw);
    double *red = swt_raw;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int64_t c = blockIdx.x / P;
    const int pp = blockIdx.x % P;
    const int32_t kk = k[c], po = piv_ptr[c], S = ilsum[c];
    const int32_t sb = (int32_t)(((int64_t)S * pp) / P), se = (int32_t)(((int64_t)S * (pp + 1)) / P);
    const int32_t e0 = il_ptr[c], e1 = il_ptr[c + 1];
    const int32_t cc0 = coord[c], cc1 = coord[nc + c], cc2 = d == 3 ? coord[2 * nc + c] : 0;
    const float h = hc ? hc[c] : h0;   // cell side (per cell when the level mixes problems)
    double *dst = P > 1 ? part_out + (int64_t)pp * npiv * RP : u;
    const int32_t ntb = (kk + 15) / 16;
    const int32_t nun = (ntb + TB - 1) / TB;
    const int32_t efirst = sb < se ? list_entry(ilpre, e0, e1, sb) : e1;
    for (int32_t tu0 = 0; tu0 < nun; tu0 += 4) {
        const int nb = nun - tu0 < 4 ? nun - tu0 : 4;
        const int nph = 4 / nb;
        const int myb = wave % nb, ph = wave / nb;
        const bool wact = ph < nph;
        const int32_t tu = tu0 + myb;
        // r^2 = |t|^2 + |s|^2 - 2 t.s in the target cell's frame (one
        // addition and three FMAs): -2t and |t|^2 per target, |s|^2 per source
        float tx[TB], ty[TB], tz[TB], tn[TB];
#pragma unroll
        for (int j = 0; j < TB; j++) {
            const int32_t row = (tu * TB + j) * 16 + (lane & 15);
            const int32_t rc = row < kk ? row : kk - 1;
            tx[j] = pc[po + rc];
            ty[j] = pc[npiv + po + rc];
            tz[j] = d == 3 ? pc[2 * npiv + po + rc] : 0.f;
            tn[j] = tx[j] * tx[j] + ty[j] * ty[j] + tz[j] * tz[j];
            tx[j] *= -2.f;
            ty[j] *= -2.f;
            tz[j] *= -2.f;
        }
        floatx4 accf[TB][NCB];
        double accd[TB][NCB][4];
#pragma unroll
        for (int j = 0; j < TB; j++)
#pragma unroll
            for (int b = 0; b < NCB; b++) {
                accf[j][b] = floatx4{0.f, 0.f, 0.f, 0.f};
                for (int i = 0; i < 4; i++) accd[j][b][i] = 0.0;
            }
        // windows of MET list entries staged in LDS: first source, pivot base
        // and cell offset of every entry
        for (int32_t w0 = efirst; w0 < e1; w0 += MET) {
            const int32_t wn = e1 - w0 < MET ? e1 - w0 : MET;
            __syncthreads();
            for (int32_t j = t; j < wn; j += NT) {
                const int32_t e = w0 + j, b = il[e], pre = ilpre[e];
                est[j] = pre;
                ebase[j] = piv_ptr[b] - pre;
                esh[0][j] = (float)(coord[b] - cc0) * h;
                esh[1][j] = (float)(coord[nc + b] - cc1) * h;
                esh[2][j] = d == 3 ? (float)(coord[2 * nc + b] - cc2) * h : 0.f;
            }
            if (t == 0) est[wn] = w0 + wn < e1 ? ilpre[w0 + wn] : S;
            __syncthreads();
            if (est[0] >= se) break;
            const int32_t ws = est[0] > sb ? est[0] : sb, we = est[wn] < se ? est[wn] : se;
            for (int32_t s0 = ws; s0 < we; s0 += TS) {
                const int32_t ns = we - s0 < TS ? we - s0 : TS;
                __syncthreads();
                if (t < ns) {
                    const int32_t s = s0 + t;
                    int32_t lo = 0, hi = wn - 1;
                    while (lo < hi) {
                        int32_t mid = (lo + hi + 1) >> 1;
                        if (est[mid] <= s) lo = mid; else hi = mid - 1;
                    }
                    const int32_t idx = ebase[lo] + s;
                    float4 v;
                    v.x = pc[idx] + esh[0][lo];
                    v.y = pc[npiv + idx] + esh[1][lo];
                    v.z = d == 3 ? pc[2 * npiv + idx] + esh[2][lo] : 0.f;
                    v.w = v.x * v.x + v.y * v.y + v.z * v.z;
                    sx[t] = v;
                    sidx[t] = idx;
                    if constexpr (TS == NT) {
                        // one source per thread: it loads its own weight row
                        const float4 *wr = reinterpret_cast<const float4 *>(w32 + (int64_t)idx * RP);
                        float4 *wd = reinterpret_cast<float4 *>(swt + t * SW);
#pragma unroll
                        for (int q = 0; q < RP / 4; q++)
                            wd[q] = 4 * q < R ? wr[q] : make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                } else if (t < ((ns + 63) & ~63)) {
                    // padding up to a multiple of 64 sources (TS is one): far
                    // from every target, zero weights, so it adds exact zeros
                    sx[t] = make_float4(1e15f, 1e15f, 1e15f, 3e30f);
                    sidx[t] = -1;
                    if constexpr (TS == NT) {
                        float4 *wd = reinterpret_cast<float4 *>(swt + t * SW);
#pragma unroll
                        for (int q = 0; q < RP / 4; q++) wd[q] = make_float4(0.f, 0.f, 0.f, 0.f);
                    }
                }
                __syncthreads();
                // with fewer sources than threads per tile, the FP32 weight
                // rows are loaded by the whole workgroup, four columns per
                // thread and step: the columns up to R (padding columns of w
                // are zero), then zeros
                if constexpr (TS != NT) {
                    constexpr int NV = RP / 4;
                    const int rows = (ns + 63) & ~63;
                    for (int i = t; i < rows * NV; i += NT) {
                        const int row = i / NV, q = i % NV;
                        const int32_t idx = sidx[row];
                        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                        if (idx >= 0 && 4 * q < R) v = reinterpret_cast<const float4 *>(w32 + (int64_t)idx * RP)[q];
                        reinterpret_cast<float4 *>(swt + row * SW)[q] = v;
                    }
                    __syncthreads();
                }
                // groups of four steps: the FP32 accumulators stay in the
                // matrix-core registers across a group and are added into
                // the FP64 sums once per group.  A group of phase ph reads
                // sources below (g0 / (16 nph) + 1) 16 nph <= the padded
                // tile end, since 16 nph divides 64.
                // (the phase count is a template constant of the loop, so the
                // four steps' LDS addresses differ by immediate offsets)
                auto groups = [&](auto nph_c) {
                    constexpr int NPH = decltype(nph_c)::value;
                    for (int32_t g0 = ph * 4; g0 < ns; g0 += 16 * NPH) {
#pragma unroll
                        for (int k = 0; k < 4; k++) {
                            const int32_t src = g0 + k * 4 * NPH + (lane >> 4);
                            const float4 q = sx[src];
                            float kvv[TB];
#pragma unroll
                            for (int j = 0; j < TB; j++) {
                                float r2 = tn[j] + q.w;
                                r2 = fmaf(tz[j], q.z, r2);
                                r2 = fmaf(ty[j], q.y, r2);
                                r2 = fmaf(tx[j], q.x, r2);
                                kvv[j] = kv32<KIND>(r2, prm);
                            }
#pragma unroll
                            for (int b = 0; b < NCB; b++) {
                                const float bw = swt[src * SW + b * 16 + (lane & 15)];
#pragma unroll
                                for (int j = 0; j < TB; j++)
                                    accf[j][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(kvv[j], bw, accf[j][b], 0, 0, 0);
                            }
                        }
#pragma unroll
                        for (int j = 0; j < TB; j++)
#pragma unroll
                            for (int b = 0; b < NCB; b++) {
#pragma unroll
                                for (int i = 0; i < 4; i++) accd[j][b][i] += (double)accf[j][b][i];
                                accf[j][b] = floatx4{0.f, 0.f, 0.f, 0.f};
                            }
                    }
                };
                if (wact) {
                    if (nph == 1) groups(std::integral_constant<int, 1>{});
                    else if (nph == 2) groups(std::integral_constant<int, 2>{});
                    else groups(std::integral_constant<int, 4>{});
                }
            }
        }
        // phases of the same unit are added in order ph = 0, 1, ...
        __syncthreads();
        if (nph > 1 && wact)
            for (int j = 0; j < TB; j++)
                for (int b = 0; b < NCB; b++)
                    for (int i = 0; i < 4; i++)
                        red[((wave * 64 + lane) * TB + j) * NCB * 4 + b * 4 + i] = accd[j][b][i];
        __syncthreads();
        if (wact && ph == 0) {
            for (int p2 = 1; p2 < nph; p2++) {
                const int w2 = p2 * nb + myb;
                for (int j = 0; j < TB; j++)
                    for (int b = 0; b < NCB; b++)
                        for (int i = 0; i < 4; i++)
                            accd[j][b][i] += red[((w2 * 64 + lane) * TB + j) * NCB * 4 + b * 4 + i];
            }
            for (int j = 0; j < TB; j++)
                for (int b = 0; b < NCB; b++)
                    for (int i = 0; i < 4; i++) {
                        const int32_t r = (tu * TB + j) * 16 + 4 * (lane >> 4) + i;
                        if (r < kk) dst[(int64_t)(po + r) * RP + b * 16 + (lane & 15)] = accd[j][b][i];
                    }
        }
        __syncthreads();
    }
}

// M2L in FP64 on the matrix cores (v_mfma_f64_16x16x4f64): the plain FP64
// kernel (MODE 1) or the refined one (MODE 2) generated once per (target,
// source) pair.  Output layout of this instruction: lane l, element i holds
// row 4 i + l / 16, column l % 16.
typedef double doublex4 __attribute__((ext_vector_type(4)));
template <int KIND, int MODE, int NCB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_m2l_mfma64(int64_t nc, int P, const int32_t *k, const int32_t *piv_ptr,
                                                   const int32_t *il_ptr, const int32_t *il, const int32_t *ilpre,
                                                   const int32_t *ilsum, const double *pc, int64_t npiv, int d,
                                                   const double *w, int R, double *u, double *part_out, double prm)
{
    constexpr int RP = NCB * 16;
    constexpr int TS = 64;
    __shared__ double4 sx[TS];
    __shared__ int32_t sidx[TS];
    __shared__ __align__(16) double swt[TS * RP > NT * NCB * 4 ? TS * RP : NT * NCB * 4];
    double *red = swt;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int64_t c = blockIdx.x / P;
    const int pp = blockIdx.x % P;
    const int32_t kk = k[c], po = piv_ptr[c], S = ilsum[c];
    const int32_t sb = (int32_t)(((int64_t)S * pp) / P), se = (int32_t)(((int64_t)S * (pp + 1)) / P);
    const int32_t e0 = il_ptr[c], e1 = il_ptr[c + 1];
    double *dst = P > 1 ? part_out + (int64_t)pp * npiv * RP : u;
    const int32_t ntb = (kk + 15) / 16;
    for (int32_t tb0 = 0; tb0 < ntb; tb0 += 4) {
        const int nb = ntb - tb0 < 4 ? ntb - tb0 : 4;
        const int nph = 4 / nb;
        const int myb = wave % nb, ph = wave / nb;
        const bool wact = ph < nph;
        const int32_t tb = tb0 + myb;
        int32_t row = tb * 16 + (lane & 15);
        int32_t rc = row < kk ? row : kk - 1;
        const double tx = pc[po + rc], ty = pc[npiv + po + rc], tz = d == 3 ? pc[2 * npiv + po + rc] : 0.0;
        doublex4 acc[NCB];
#pragma unroll
        for (int b = 0; b < NCB; b++) acc[b] = doublex4{0.0, 0.0, 0.0, 0.0};
        for (int32_t s0 = sb; s0 < se; s0 += TS) {
            const int32_t ns = se - s0 < TS ? se - s0 : TS;
            __syncthreads();
            if (t < ns) {
                const int32_t s = s0 + t;
                const int32_t e = list_entry(ilpre, e0, e1, s);
                const int32_t idx = piv_ptr[il[e]] + (s - ilpre[e]);
                sx[t] = make_double4(pc[idx], pc[npiv + idx], d == 3 ? pc[2 * npiv + idx] : 0.0, 0.0);
                sidx[t] = idx;
            }
            __syncthreads();
            // the tile's weight rows, two columns per thread and step over the
            // whole workgroup (padding columns are zero)
            for (int i = t; i < ns * (RP / 2); i += NT) {
                const int row = i / (RP / 2), q = i % (RP / 2);
                double2 v = make_double2(0.0, 0.0);
                if (2 * q < R) v = reinterpret_cast<const double2 *>(w + (int64_t)sidx[row] * RP)[q];
                reinterpret_cast<double2 *>(swt + row * RP)[q] = v;
            }
            __syncthreads();
            if (wact)
                for (int32_t s4 = ph * 4; s4 < ns; s4 += 4 * nph) {
                    int32_t src = s4 + (lane >> 4);
                    double kvv = 0.0;
                    int32_t srcc = src < ns ? src : ns - 1;
                    if (src < ns) {
                        double4 q = sx[src];
                        double dx = tx - q.x, dy = ty - q.y, dz = tz - q.z;
                        double d2 = dx * dx + dy * dy + dz * dz;
                        kvv = MODE == 1 ? kv64<KIND>(d2, prm) : kv_refined<KIND>(d2, prm);
                    }
#pragma unroll
                    for (int b = 0; b < NCB; b++)
                        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(kvv, swt[srcc * RP + b * 16 + (lane & 15)],
                                                                     acc[b], 0, 0, 0);
                }
        }
        __syncthreads();
        if (nph > 1 && wact)
            for (int b = 0; b < NCB; b++)
                for (int i = 0; i < 4; i++) red[(wave * 64 + lane) * NCB * 4 + b * 4 + i] = acc[b][i];
        __syncthreads();
        if (wact && ph == 0) {
            for (int p2 = 1; p2 < nph; p2++) {
                int w2 = p2 * nb + myb;
                for (int b = 0; b < NCB; b++)
                    for (int i = 0; i < 4; i++) acc[b][i] += red[(w2 * 64 + lane) * NCB * 4 + b * 4 + i];
            }
            for (int b = 0; b < NCB; b++)
                for (int i = 0; i < 4; i++) {
                    int32_t r = tb * 16 + 4 * i + (lane >> 4);
                    if (r < kk) dst[(int64_t)(po + r) * RP + b * 16 + (lane & 15)] = acc[b][i];
                }
        }
        __syncthreads();
    }
}

// Near field for RP columns on the matrix cores plus the far field, written
// back in tree order (k_scatter_multi then forms Y).
// Coordinates FP64; the mixed form (T = float) rounds the differences to FP32,
// generates K in FP32 and multiplies it by the x_hi and x_lo tiles with
// v_mfma_f32_16x16x4f32 (partial sums folded into FP64 every 16 sources);
// T = double uses v_mfma_f64_16x16x4f64.
template <typename T, int KIND, int NCB>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NCB == 1 ? 6 : 4))) void k_p2p_mfma(int64_t nc, const int32_t *first, const int32_t *count,
                                                 const int32_t *nb_ptr, const int32_t *nb, const int32_t *nbpre,
                                                 const int32_t *nbsum, const double *pts, int64_t n, int d,
                                                 const T *xw, const T *xw2, const double *far, double *yt, int R,
                                                 T prm)
{
    constexpr int RP = NCB * 16;
    constexpr int TS = 64;
    constexpr bool mixed = sizeof(T) == 4;
    static_assert(TS == 64 && TS <= NT, "every step index stays inside one 64-source tile");
    // LDS row stride (bank spread); with RP + 4 the 64-column mixed form
    // stays under 40 KB and, bounded to 128 VGPRs (four waves per EU, no
    // spills), runs four waves per SIMD: c3 near field 0.132 against 0.113
    // of the FP32 matrix peak (RP + 16, three waves)
    constexpr int SW = (mixed && !(NCB & 1)) ? RP + 4 : RP;
    // the weight tiles and, after the tile loop, the phase reduction share
    // one LDS buffer
    constexpr int WBYTES = (int)sizeof(T) * TS * SW * (mixed ? 2 : 1);
    constexpr int RBYTES = (int)sizeof(double) * NT * NCB * 4;
    __shared__ double4 sx[TS];
    __shared__ int32_t sidx[TS];
    __shared__ __align__(16) double sraw[(WBYTES > RBYTES ? WBYTES : RBYTES) / 8];
    T *swt = reinterpret_cast<T *>(sraw);
    T *swt2 = mixed ? swt + TS * SW : swt;   // used by the mixed form only
    double *red = sraw;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int64_t c = blockIdx.x;
    const int32_t kk = count[c], po = first[c], S = nbsum[c];
    const int32_t e0 = nb_ptr[c], e1 = nb_ptr[c + 1];
    const int32_t ntb = (kk + 15) / 16;
    for (int32_t tb0 = 0; tb0 < ntb; tb0 += 4) {
        const int nblk = ntb - tb0 < 4 ? ntb - tb0 : 4;
        const int nph = 4 / nblk;
        const int myb = wave % nblk, ph = wave / nblk;
        const bool wact = ph < nph;
        const int32_t tb = tb0 + myb;
        int32_t row = tb * 16 + (lane & 15);
        int32_t rc = row < kk ? row : kk - 1;
        const double tx = pts[po + rc], ty = pts[n + po + rc], tz = d == 3 ? pts[2 * n + po + rc] : 0.0;
        double accd[NCB][4];
        floatx4 af[NCB], af2[NCB];
        doublex4 ad[NCB];
#pragma unroll
        for (int b = 0; b < NCB; b++) {
            for (int i = 0; i < 4; i++) accd[b][i] = 0.0;
            af[b] = floatx4{0.f, 0.f, 0.f, 0.f};
            af2[b] = floatx4{0.f, 0.f, 0.f, 0.f};
            ad[b] = doublex4{0.0, 0.0, 0.0, 0.0};
        }
        for (int32_t s0 = 0; s0 < S; s0 += TS) {
            const int32_t ns = S - s0 < TS ? S - s0 : TS;
            __syncthreads();
            if (t < ns) {
                const int32_t s = s0 + t;
                const int32_t e = list_entry(nbpre, e0, e1, s);
                const int32_t idx = first[nb[e]] + (s - nbpre[e]);
                sx[t] = make_double4(pts[idx], pts[n + idx], d == 3 ? pts[2 * n + idx] : 0.0, 0.0);
                sidx[t] = idx;
            } else if (t < TS) {
                // padding of the tile: far from every target, zero weights
                sx[t] = make_double4(1e15, 1e15, 1e15, 0.0);
                sidx[t] = -1;
            }
            __syncthreads();
            // the tile's weight rows, 16 bytes per thread and step over the
            // whole workgroup (columns from R on and padding rows are zero)
            {
                constexpr int V = 16 / (int)sizeof(T);   // values per 16 bytes
                constexpr int NV = RP / V;                // 16-byte pieces per row
                for (int i = t; i < TS * NV; i += NT) {
                    const int row = i / NV, q = i % NV;
                    const int32_t idx = sidx[row];
                    const bool live = idx >= 0 && V * q < R;
                    if constexpr (mixed) {
                        float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
                        if (live) {
                            a = reinterpret_cast<const float4 *>(xw + (int64_t)idx * RP)[q];
                            b = reinterpret_cast<const float4 *>(xw2 + (int64_t)idx * RP)[q];
                        }
                        reinterpret_cast<float4 *>(swt + row * SW)[q] = a;
                        reinterpret_cast<float4 *>(swt2 + row * SW)[q] = b;
                    } else {
                        double2 a = make_double2(0.0, 0.0);
                        if (live) a = reinterpret_cast<const double2 *>(xw + (int64_t)idx * RP)[q];
                        reinterpret_cast<double2 *>(swt + row * SW)[q] = a;
                    }
                }
            }
            __syncthreads();
            // groups of four steps; the FP32 form adds its partial sums
            // into FP64 once per group.  Every source index stays below TS
            // (a multiple of 16 nph); the padding adds exact zeros.
            if (wact)
                for (int32_t g0 = ph * 4; g0 < ns; g0 += 16 * nph) {
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        const int32_t src = g0 + k * 4 * nph + (lane >> 4);
                        const double4 q = sx[src];
                        const T dx = (T)(tx - q.x), dy = (T)(ty - q.y), dz = (T)(tz - q.z);
                        const T kvv = kv_self<KIND, T>(dx * dx + dy * dy + dz * dz, prm);
#pragma unroll
                        for (int b = 0; b < NCB; b++) {
                            if constexpr (mixed) {
                                af[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(kvv, swt[src * SW + b * 16 + (lane & 15)],
                                                                             af[b], 0, 0, 0);
                                af2[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(kvv, swt2[src * SW + b * 16 + (lane & 15)],
                                                                              af2[b], 0, 0, 0);
                            } else {
                                ad[b] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)kvv,
                                                                             (double)swt[src * SW + b * 16 + (lane & 15)],
                                                                             ad[b], 0, 0, 0);
                            }
                        }
                    }
                    if constexpr (mixed) {
#pragma unroll
                        for (int b = 0; b < NCB; b++) {
#pragma unroll
                            for (int i = 0; i < 4; i++) accd[b][i] += (double)af[b][i] + (double)af2[b][i];
                            af[b] = floatx4{0.f, 0.f, 0.f, 0.f};
                            af2[b] = floatx4{0.f, 0.f, 0.f, 0.f};
                        }
                    }
                }
        }
        // result rows of this lane: FP32 layout row 4 (l/16) + i, FP64 layout row 4 i + l/16
        if constexpr (!mixed)
#pragma unroll
            for (int b = 0; b < NCB; b++)
                for (int i = 0; i < 4; i++) accd[b][i] = ad[b][i];
        __syncthreads();
        if (nph > 1 && wact)
            for (int b = 0; b < NCB; b++)
                for (int i = 0; i < 4; i++) red[(wave * 64 + lane) * NCB * 4 + b * 4 + i] = accd[b][i];
        __syncthreads();
        if (wact && ph == 0) {
            for (int p2 = 1; p2 < nph; p2++) {
                int w2 = p2 * nblk + myb;
                for (int b = 0; b < NCB; b++)
                    for (int i = 0; i < 4; i++) accd[b][i] += red[(w2 * 64 + lane) * NCB * 4 + b * 4 + i];
            }
            for (int b = 0; b < NCB; b++)
                for (int i = 0; i < 4; i++) {
                    int32_t r = tb * 16 + (mixed ? 4 * (lane >> 4) + i : 4 * i + (lane >> 4));
                    int col = b * 16 + (lane & 15);
                    if (r < kk && col < R) {
                        const int64_t p = po + r;
                        const double f = far ? far[p * RP + col] : 0.0;
                        yt[p * RP + col] = f + accd[b][i];
                    }
                }
        }
        __syncthreads();
    }
}

__global__ void k_sum_parts_multi(int64_t len, int P, const double *part, double *u)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= len) return;
    double s = 0.0;
    for (int p = 0; p < P; p++) s += part[(int64_t)p * len + i];
    u[i] = s;
}

int parts_for(const Level &L)
{
    const int64_t want = 4096;
    if (L.ncell >= want) return 1;
    int64_t P = (want + L.ncell - 1) / L.ncell;
    int64_t maxp = (L.max_ilsum + 1023) / 1024;
    if (P > maxp) P = maxp;
    if (P > 64) P = 64;
    return P < 1 ? 1 : (int)P;
}

// transverse pass of one level for a block of NCB * 16 columns, split P ways
template <int NCB>
void m2l_level_multi(nnca_h2 *H, int l, int P, bool mixed, hipStream_t s, int tsel = 0)
{
    constexpr int RP = NCB * 16;
    auto &W = H->multi;
    Level &L = H->lev[l];
    const int kap = H->kappa, kind = H->kind;
    const double prm64 = kernel_prm64(kind, H->hparam);
    const float prm32 = kernel_prm32(kind, H->hparam);
    double *part = P > 1 ? W.part : nullptr;
    const int g = (int)(L.ncell * P);
    if (mixed && l > kap - H->fp32_levels) {
#define MF(K, TSL) k_m2l_mfma<K, NCB, TSL><<<g, NT, 0, s>>>(L.ncell, P, L.k, L.piv_ptr, L.il_ptr, L.il, L.ilpre, L.ilsum, L.pc32, L.npiv, L.coord, L.hcell, (float)L.h, H->dim, W.w32[l], W.R, W.u[l], part, prm32)
#define MFK(TSL) \
        if (kind == NNCA_K_INV_R) MF(NNCA_K_INV_R, TSL); \
        else if (kind == NNCA_K_LOG_R) MF(NNCA_K_LOG_R, TSL); \
        else if (kind == NNCA_K_LOG_REG) MF(NNCA_K_LOG_REG, TSL); \
        else if (kind == NNCA_K_INV_REG) MF(NNCA_K_INV_REG, TSL); \
        else if (kind == NNCA_K_EXP_R) MF(NNCA_K_EXP_R, TSL); \
        else MF(NNCA_K_GAUSS, TSL);
        if (tsel) { MFK(1) } else { MFK(0) }
#undef MFK
#undef MF
    } else {
#define VM(K, M) k_m2l_mfma64<K, M, NCB><<<g, NT, 0, s>>>(L.ncell, P, L.k, L.piv_ptr, L.il_ptr, L.il, L.ilpre, L.ilsum, L.pc64, L.npiv, H->dim, W.w[l], W.R, W.u[l], part, prm64)
        if (!mixed) {
            if (kind == NNCA_K_INV_R) VM(NNCA_K_INV_R, 1);
            else if (kind == NNCA_K_LOG_R) VM(NNCA_K_LOG_R, 1);
            else if (kind == NNCA_K_LOG_REG) VM(NNCA_K_LOG_REG, 1);
            else if (kind == NNCA_K_INV_REG) VM(NNCA_K_INV_REG, 1);
            else if (kind == NNCA_K_EXP_R) VM(NNCA_K_EXP_R, 1);
            else VM(NNCA_K_GAUSS, 1);
        } else {
            if (kind == NNCA_K_INV_R) VM(NNCA_K_INV_R, 2);
            else if (kind == NNCA_K_LOG_R) VM(NNCA_K_LOG_R, 2);
            else if (kind == NNCA_K_LOG_REG) VM(NNCA_K_LOG_REG, 2);
            else if (kind == NNCA_K_INV_REG) VM(NNCA_K_INV_REG, 2);
            else if (kind == NNCA_K_EXP_R) VM(NNCA_K_EXP_R, 2);
            else VM(NNCA_K_GAUSS, 2);
        }
#undef VM
    }
    HIPCHECK(hipGetLastError());
    if (P > 1) {
        k_sum_parts_multi<<<grid_for(L.npiv * RP, 256), 256, 0, s>>>(L.npiv * RP, P, part, W.u[l]);
        HIPCHECK(hipGetLastError());
    }
}

// the partial-result workspace (sized once, for the default split factors
// at the workspace width) holds the split factors in use
void check_part(nnca_h2 *H, int RP, const std::vector<int32_t> *tab)
{
    auto &W = H->multi;
    for (int l = H->lmin; l <= H->kappa; l++) {
        const Level &L = H->lev[l];
        const int P = tab ? (*tab)[l] / 2 : parts_for(L);
        if (P > 1 && (int64_t)P * L.npiv * RP > W.part_cap) fail(NNCA_ERR_INTERNAL, "split workspace not sized");
    }
}

// Autotuner of the transverse pass: for every level, time the launch (and the
// ordered sum of the partial vectors) for split factors P = 1, 2, 4, ..., 64
// and, on the FP32 levels of the mixed form, both tile shapes (the sources
// per LDS tile of k_m2l_mfma: TSEL 0 or 1), on the multipole vectors already
// in place, and keep the fastest.  Factors that leave a part without a full
// source tile, put more than 2^18 workgroups in flight or need more partial
// vectors than the workspace holds are not tried.  A level's choice is coded
// as 2 P + TSEL.
//
// With NNCA_TUNE_CACHE naming a file, choices are looked up there first and
// new ones appended to it, one line per level shape:
//   <arch> m2l <f32|f64> ncb=<NCB> cells=<b> srcs=<b> rank=<b> <2 P + TSEL>
// where f32 / f64 is the form of the level's launch and each <b> is the
// ceiling of log2 of the level's cell count, largest source count per cell
// and largest rank.
namespace {

std::string tune_key(const Level &L, bool f32form, int ncb)
{
    auto bucket = [](int64_t v) {
        int b = 0;
        while (((int64_t)1 << b) < v) b++;
        return b;
    };
    hipDeviceProp_t prop;
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    HIPCHECK(hipGetDeviceProperties(&prop, dev));
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    return arch + " m2l " + (f32form ? "f32" : "f64") + " ncb=" + std::to_string(ncb) +
           " cells=" + std::to_string(bucket(L.ncell)) + " srcs=" + std::to_string(bucket(L.max_ilsum)) +
           " rank=" + std::to_string(bucket(L.max_k));
}

std::map<std::string, int32_t> read_tune_cache(const char *path)
{
    std::map<std::string, int32_t> m;
    FILE *f = std::fopen(path, "r");
    if (!f) return m;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        std::string ln(line);
        while (!ln.empty() && (ln.back() == '\n' || ln.back() == '\r')) ln.pop_back();
        const size_t sp = ln.rfind(' ');
        if (sp == std::string::npos) continue;
        char *end = nullptr;
        const long v = std::strtol(ln.c_str() + sp + 1, &end, 10);
        if (end == ln.c_str() + sp + 1 || v < 2 || v > 129) continue;   // 2 P + TSEL, P in 1..64
        m[ln.substr(0, sp)] = (int32_t)v;
    }
    std::fclose(f);
    return m;
}

}  // namespace

template <int NCB>
std::vector<int32_t> tune_m2l_multi(nnca_h2 *H, bool mixed, hipStream_t s)
{
    constexpr int RP = NCB * 16;
    std::vector<int32_t> best(H->kappa + 1, 2);
    const char *cache_path = std::getenv("NNCA_TUNE_CACHE");
    std::map<std::string, int32_t> cache;
    if (cache_path && *cache_path) cache = read_tune_cache(cache_path);
    std::vector<std::string> fresh;
    hipEvent_t a, b;
    HIPCHECK(hipEventCreate(&a));
    HIPCHECK(hipEventCreate(&b));
    try {
        for (int l = H->lmin; l <= H->kappa; l++) {
            const Level &L = H->lev[l];
            const bool f32form = mixed && l > H->kappa - H->fp32_levels;
            const std::string key = tune_key(L, f32form, NCB);
            auto hit = cache.find(key);
            if (hit != cache.end()) {
                const int P = hit->second / 2;
                if (P == 1 || ((int64_t)P * L.npiv * RP <= H->multi.part_cap && (int64_t)P * L.ncell <= (1 << 18))) {
                    best[l] = hit->second;
                    continue;
                }
            }
            std::vector<int32_t> cand;
            for (int P = 1; P <= 64; P *= 2) {
                if (P > 1 && (int64_t)P * 128 > L.max_ilsum) break;
                if ((int64_t)P * L.ncell > (1 << 18)) break;
                if (P > 1 && (int64_t)P * L.npiv * RP > H->multi.part_cap) break;
                cand.push_back(2 * P);
                if (f32form) cand.push_back(2 * P + 1);
            }
            float tbest = 0.f;
            for (int32_t code : cand) {
                const int P = code / 2, tsel = code % 2;
                m2l_level_multi<NCB>(H, l, P, mixed, s, tsel);   // warm
                HIPCHECK(hipEventRecord(a, s));
                for (int rep = 0; rep < 3; rep++) m2l_level_multi<NCB>(H, l, P, mixed, s, tsel);
                HIPCHECK(hipEventRecord(b, s));
                HIPCHECK(hipEventSynchronize(b));
                float ms = 0.f;
                HIPCHECK(hipEventElapsedTime(&ms, a, b));
                if (code == cand[0] || ms < tbest) {
                    tbest = ms;
                    best[l] = code;
                }
            }
            cache[key] = best[l];
            fresh.push_back(key + " " + std::to_string(best[l]));
        }
    } catch (...) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        throw;
    }
    HIPCHECK(hipEventDestroy(a));
    HIPCHECK(hipEventDestroy(b));
    if (cache_path && *cache_path && !fresh.empty()) {
        // appended, one line per new level shape; an unwritable file only
        // means the next process tunes again
        if (FILE *f = std::fopen(cache_path, "a")) {
            for (const std::string &ln : fresh) std::fprintf(f, "%s\n", ln.c_str());
            std::fclose(f);
        }
    }
    return best;
}

template <int NCB, typename TI, typename TO>
void multi_block(nnca_h2 *H, const TI *X, TO *Y, int R, int64_t ldx, int64_t ldy, int precision, hipStream_t s)
{
    constexpr int RP = NCB * 16;
    const int64_t n = H->n;
    const int kap = H->kappa, lmin = H->lmin;
    const bool mixed = precision == NNCA_PREC_MIXED;
    const int kind = H->kind;
    auto &W = H->multi;
    {
        Span sp(H, s, PASS_GATHER, -1);
        k_gather_multi<TI><<<(unsigned)((n + 63) / 64), 256, 0, s>>>(n, R, RP, H->rank, X, ldx, W.xs,
                                                                     mixed ? W.xhi : nullptr, mixed ? W.xlo : nullptr);
        HIPCHECK(hipGetLastError());
    }
    const double prm64 = kernel_prm64(kind, H->hparam);
    const float prm32 = kernel_prm32(kind, H->hparam);
    double *far = nullptr;
    if (kap >= lmin) {
        for (int l = kap; l >= lmin; l--) {
            Level &L = H->lev[l];
            const double *src = l == kap ? W.xs : W.w[l + 1];
            const int ipc = (int)((L.max_k + 63) / 64) * NCB;
            const unsigned nb = (unsigned)(L.ncell * ipc);
            Span sp(H, s, PASS_UP, l);
            if (nb < SPLIT_BELOW)
                k_up_multi_split<<<nb, 64 * SPLIT_WAVES, 0, s>>>(ipc, RP, L.piv_ptr, L.tt_off, L.ipos, L.rem_ptr,
                                                                 L.rem_pos, L.crem_off, L.crem64, src, W.w[l]);
            else
                k_up_multi<<<nb, 64, 0, s>>>(ipc, RP, L.piv_ptr, L.tt_off, L.ipos, L.rem_ptr, L.rem_pos,
                                             L.crem_off, L.crem64, src, W.w[l]);
            HIPCHECK(hipGetLastError());
        }
        // FP32 copies of the multipole vectors the FP32 transverse pass reads
        W.R = R;
        if (mixed)
            for (int l = std::max(lmin, kap - H->fp32_levels + 1); l <= kap; l++) {
                const int64_t cnt = H->lev[l].npiv * RP;
                k_to_f32<<<grid_for(cnt, 256), 256, 0, s>>>(cnt, W.w[l], W.w32[l]);
                HIPCHECK(hipGetLastError());
            }
        const std::vector<int32_t> *tab = nullptr;
        if (H->autotune) {
            const int key = NCB * 2 + (mixed ? 1 : 0);
            auto it = H->m2l_tuned.find(key);
            if (it == H->m2l_tuned.end()) it = H->m2l_tuned.emplace(key, tune_m2l_multi<NCB>(H, mixed, s)).first;
            tab = &it->second;
        }
        check_part(H, RP, tab);
        for (int l = lmin; l <= kap; l++) {
            Span sp(H, s, PASS_M2L, l);   // the launch and, for split levels, the ordered sum of its parts
            if (tab) m2l_level_multi<NCB>(H, l, (*tab)[l] / 2, mixed, s, (*tab)[l] % 2);
            else m2l_level_multi<NCB>(H, l, parts_for(H->lev[l]), mixed, s);
        }
        far = W.far;
        for (int l = lmin; l <= kap; l++) {
            Level &L = H->lev[l];
            double *out = l == kap ? far : W.u[l + 1];
            const int nqc = (int)((L.max_k + 63) / 64);
            const int ipc = (nqc + (int)((L.max_nrem + 63) / 64)) * NCB;
            const unsigned nb = (unsigned)(L.ncell * ipc);
            Span sp(H, s, PASS_DOWN, l);
            if (nb < SPLIT_BELOW)
                k_down_multi_split<<<nb, 64 * SPLIT_WAVES, 0, s>>>(ipc, nqc, RP, L.piv_ptr, L.tt_off, L.ipos,
                                                                   L.rem_ptr, L.rem_pos, L.crem_off, L.crem_t,
                                                                   W.u[l], out, l == kap ? 0 : 1);
            else
                k_down_multi<<<nb, 64, 0, s>>>(ipc, nqc, RP, L.piv_ptr, L.tt_off, L.ipos, L.rem_ptr, L.rem_pos,
                                               L.crem_off, L.crem_t, W.u[l], out, l == kap ? 0 : 1);
            HIPCHECK(hipGetLastError());
        }
    }
    const Level &F = H->lev[kap];
    Span sp(H, s, PASS_P2P, kap);   // the near field and the combine
#define PP(T, K, A, B, PRM) k_p2p_mfma<T, K, NCB><<<(int)F.ncell, NT, 0, s>>>(F.ncell, F.first, F.count, F.nb_ptr, F.nb, H->nbpre, H->nbsum, H->pts64, n, H->dim, A, B, far, W.far, R, PRM)
    if (mixed) {
        if (kind == NNCA_K_INV_R) PP(float, NNCA_K_INV_R, W.xhi, W.xlo, prm32);
        else if (kind == NNCA_K_LOG_R) PP(float, NNCA_K_LOG_R, W.xhi, W.xlo, prm32);
        else if (kind == NNCA_K_LOG_REG) PP(float, NNCA_K_LOG_REG, W.xhi, W.xlo, prm32);
        else if (kind == NNCA_K_INV_REG) PP(float, NNCA_K_INV_REG, W.xhi, W.xlo, prm32);
        else if (kind == NNCA_K_EXP_R) PP(float, NNCA_K_EXP_R, W.xhi, W.xlo, prm32);
        else PP(float, NNCA_K_GAUSS, W.xhi, W.xlo, prm32);
    } else {
        if (kind == NNCA_K_INV_R) PP(double, NNCA_K_INV_R, W.xs, (const double *)nullptr, prm64);
        else if (kind == NNCA_K_LOG_R) PP(double, NNCA_K_LOG_R, W.xs, (const double *)nullptr, prm64);
        else if (kind == NNCA_K_LOG_REG) PP(double, NNCA_K_LOG_REG, W.xs, (const double *)nullptr, prm64);
        else if (kind == NNCA_K_INV_REG) PP(double, NNCA_K_INV_REG, W.xs, (const double *)nullptr, prm64);
        else if (kind == NNCA_K_EXP_R) PP(double, NNCA_K_EXP_R, W.xs, (const double *)nullptr, prm64);
        else PP(double, NNCA_K_GAUSS, W.xs, (const double *)nullptr, prm64);
    }
#undef PP
    HIPCHECK(hipGetLastError());
    k_scatter_multi<TO><<<(unsigned)((n + 63) / 64), 256, 0, s>>>(n, R, RP, H->rank, W.far, Y, ldy);
    HIPCHECK(hipGetLastError());
}

}  // namespace

// many-column workspace for blocks of up to RP (a multiple of 16, <= 64)
// columns: tree-order inputs and outputs, the multipole and local vectors of
// every level, FP32 copies of the multipole vectors of the FP32 levels, and
// the partial vectors of the default split factors
void alloc_multi(nnca_h2 *H, int RP)
{
    auto &W = H->multi;
    free_multi(H);
    const int64_t n = H->n;
    W.xs = dalloc<double>(n * RP);
    W.far = dalloc<double>(n * RP);
    W.xhi = dalloc<float>(n * RP);
    W.xlo = dalloc<float>(n * RP);
    W.w.assign(H->kappa + 2, nullptr);
    W.u.assign(H->kappa + 2, nullptr);
    W.w32.assign(H->kappa + 2, nullptr);
    int64_t part = 1;
    for (int l = H->lmin; l <= H->kappa; l++) {
        const Level &L = H->lev[l];
        W.w[l] = dalloc<double>(L.npiv * RP);
        if (l > H->kappa - H->fp32_levels) W.w32[l] = dalloc<float>(L.npiv * RP);
        W.u[l] = dalloc<double>(L.npiv * RP);
        part = std::max(part, (int64_t)parts_for(L) * L.npiv * RP);
    }
    W.part = dalloc<double>(part);
    W.part_cap = part;
    W.rp = RP;
}

void free_multi(nnca_h2 *H)
{
    auto &W = H->multi;
    dfree(W.xs); dfree(W.far); dfree(W.xhi); dfree(W.xlo); dfree(W.part);
    for (auto p : W.w) dfree(p);
    for (auto p : W.u) dfree(p);
    for (auto p : W.w32) dfree(p);
    W = nnca_h2::Multi();
}

template <typename TI, typename TO>
static void multi_typed(nnca_h2 *H, const TI *X, TO *Y, int64_t nrhs, int64_t ldx, int64_t ldy, int precision,
                        hipStream_t s)
{
    const int width = H->multi.rp;   // blocks of the workspace's width
    for (int64_t c0 = 0; c0 < nrhs; c0 += width) {
        const int R = (int)std::min<int64_t>(width, nrhs - c0);
        const int NCB = (R + 15) / 16;
        const TI *Xb = X + c0 * ldx;
        TO *Yb = Y + c0 * ldy;
        switch (NCB) {
        case 1: multi_block<1>(H, Xb, Yb, R, ldx, ldy, precision, s); break;
        case 2: multi_block<2>(H, Xb, Yb, R, ldx, ldy, precision, s); break;
        case 3: multi_block<3>(H, Xb, Yb, R, ldx, ldy, precision, s); break;
        default: multi_block<4>(H, Xb, Yb, R, ldx, ldy, precision, s); break;
        }
    }
}

void run_matvec_multi(nnca_h2 *H, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy, int dtype,
                      int precision, hipStream_t s)
{
    if (H->multi.rp < 16) fail(NNCA_ERR_INTERNAL, "many-column workspace missing");
    if (dtype == NNCA_F32) multi_typed(H, (const float *)X, (float *)Y, nrhs, ldx, ldy, precision, s);
    else multi_typed(H, (const double *)X, (double *)Y, nrhs, ldx, ldy, precision, s);
}

}  // namespace nnca
