// H2 matrix-vector product of Sec. 4 on gfx950: upward pass (P2M, M2M),
// transverse pass (M2L blocks S_{B,B'} = K(t^{B,i}, t^{B',i}) evaluated on the
// fly at the pivot sets), downward pass (L2L, L2P) and the near field (P2P,
// evaluated on the fly), in FP64 or in the mixed FP32 form.
//
// Layout: every level keeps its pivots contiguous per cell in Morton order, so
// the candidate rows t~ of a non-leaf cell (its children's pivots) are one
// contiguous range of the next level's arrays and the multipole / local
// vectors of a level are plain arrays indexed like its pivots.  The transfer
// operator C_B is stored as its non-identity rows only (the pivot rows of
// C_B are exactly the identity).
//
// Mixed precision: coordinates are FP32 offsets from the owning cell's
// centre; a source of cell B' seen from cell B is shifted by
// (c_B' - c_B) h in FP32, so differences of nearby points keep their
// relative accuracy.  The input is split x = x_hi + x_lo; everything runs on
// x_hi and the near field also on x_lo; the partial results are added in FP64.
#include <cstring>
#include <algorithm>

#include "nnca_internal.h"
#include "kernel_values.h"

namespace nnca {

namespace {

constexpr int NT = 256;
constexpr int CHUNK = 16;   // terms summed in the working precision before an FP64 fold

template <typename T> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };

// ---------------------------------------------------------------------------
// input gather (original -> tree order) and split

// TI: element type of the caller's vector (FP32 input is widened exactly)
template <typename TI>
__global__ void k_gather64(int64_t n, const int32_t *order, const TI *x, double *xs)
{
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < n) xs[p] = (double)x[order[p]];
}

template <typename TI>
__global__ void k_gather_split(int64_t n, const int32_t *order, const TI *x, double *xs, float *hi, float *lo)
{
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    double v = (double)x[order[p]];
    xs[p] = v;
    float h = (float)v;
    hi[p] = h;
    lo[p] = (float)(v - (double)h);
}

// ---------------------------------------------------------------------------
// Transfer passes, in FP64 in both precisions: the nested interpolation
// operators C_B of a tolerance-driven ACA have entries of size 10-100, which
// would amplify FP32 rounding of the nested vectors.  One thread per output
// entry over the whole level (pivot entries first, then the other rows).

// upward pass: w^{B,o} = C_B^T x~ with x~ = x^B at a leaf (P2M), else the
// children's w^{B_c,o} stacked (M2M).  C_B's pivot rows are the identity.
__global__ void k_up(int64_t npiv, const int32_t *piv_cell, const int32_t *piv_ptr, const int32_t *tt_off,
                     const int32_t *ipos, const int32_t *rem_ptr, const int32_t *rem_pos, const int64_t *crem_off,
                     const double *crem, const double *xin, double *w)
{
    int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= npiv) return;
    int32_t c = piv_cell[g];
    int32_t po = piv_ptr[c], kk = piv_ptr[c + 1] - po, q = (int32_t)g - po;
    int32_t to = tt_off[c], ro = rem_ptr[c], nr = rem_ptr[c + 1] - ro;
    const double *C = crem + crem_off[c] + q;
    double acc = xin[to + ipos[g]];
    for (int32_t r = 0; r < nr; r++) acc += C[(int64_t)r * kk] * xin[to + rem_pos[ro + r]];
    w[g] = acc;
}

// the same for levels whose cells have non-pivot rows: workgroup (c, y) takes
// columns [y colw, (y + 1) colw) of cell c (levels with few cells split their
// columns over several workgroups), the inputs of the non-pivot rows staged
// in LDS, rows split among thread groups
constexpr int UP_TILE = 1024;
__global__ __launch_bounds__(256) void k_up_cell(const int32_t *piv_ptr, const int32_t *tt_off, const int32_t *ipos,
                                                 const int32_t *rem_ptr, const int32_t *rem_pos,
                                                 const int64_t *crem_off, const double *crem, const double *xin,
                                                 double *w, int32_t colw)
{
    __shared__ double xr[UP_TILE];
    __shared__ double red[256];
    const int t = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int32_t po = piv_ptr[c], kk = piv_ptr[c + 1] - po, to = tt_off[c];
    const int32_t ro = rem_ptr[c], nr = rem_ptr[c + 1] - ro;
    const double *C = crem + crem_off[c];
    const int64_t cb64 = (int64_t)blockIdx.y * colw;
    if (cb64 >= kk) return;   // uniform for the workgroup
    const int32_t cb = (int32_t)cb64, ce = kk - cb < colw ? kk : cb + colw;
    for (int32_t tb = cb; tb < ce; tb += 256) {
        const int32_t cnt = ce - tb < 256 ? ce - tb : 256;
        const int32_t G = 256 / cnt, ti = t % cnt, g = t / cnt;
        double acc = 0.0;
        for (int32_t r0 = 0; r0 < nr; r0 += UP_TILE) {
            const int32_t rn = nr - r0 < UP_TILE ? nr - r0 : UP_TILE;
            __syncthreads();
            for (int32_t i = t; i < rn; i += 256) xr[i] = xin[to + rem_pos[ro + r0 + i]];
            __syncthreads();
            if (g < G) {
                // four independent partial sums keep four row loads in flight
                double a1 = 0.0, a2 = 0.0, a3 = 0.0;
                int32_t r = g;
                const double *Cq = C + tb + ti;
                for (; r + 3 * G < rn; r += 4 * G) {
                    acc += Cq[(int64_t)(r0 + r) * kk] * xr[r];
                    a1 += Cq[(int64_t)(r0 + r + G) * kk] * xr[r + G];
                    a2 += Cq[(int64_t)(r0 + r + 2 * G) * kk] * xr[r + 2 * G];
                    a3 += Cq[(int64_t)(r0 + r + 3 * G) * kk] * xr[r + 3 * G];
                }
                for (; r < rn; r += G) acc += Cq[(int64_t)(r0 + r) * kk] * xr[r];
                acc += (a1 + a2) + a3;
            }
        }
        red[t] = acc;
        __syncthreads();
        if (t < cnt) {
            double sum = xin[to + ipos[po + tb + t]];
            for (int32_t gg = 0; gg < G; gg++) sum += red[gg * cnt + t];
            w[po + tb + t] = sum;
        }
        __syncthreads();
    }
}

// y_j = near + far of the point whose tree position is rank_j: random reads,
// contiguous writes (the same sum, in the same order, as adding the far field
// to the near-field sums in place).  far may be NULL (no far field).  TO: the
// caller's element type (FP32 output is the rounded FP64 sum).
template <typename TO>
__global__ void k_near_far_out(int64_t n, const int32_t *rank, const double *near, const double *far, TO *y)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t p = rank[j];
    y[j] = (TO)(far ? near[p] + far[p] : near[p]);
}

__global__ void k_invert_order(int64_t n, const int32_t *order, int32_t *rank)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < n) rank[order[p]] = (int32_t)p;
}

// downward pass: the stacked C_B u^{B,i} added to the children's u (L2L) or
// written as the far field of the leaf's points (L2P).  crem_t holds every
// cell's block transposed (k x (m-k)) so that neighbouring rows read
// neighbouring addresses.
// With `order` (leaf level), the rows are points and go to out[order[row]],
// the result in the original point order.
__global__ void k_down(int64_t npiv, int64_t nrem, const int32_t *piv_cell, const int32_t *rem_cell,
                       const int32_t *piv_ptr, const int32_t *tt_off, const int32_t *ipos, const int32_t *rem_ptr,
                       const int32_t *rem_pos, const int64_t *crem_off, const double *crem_t, const double *u,
                       double *out, int accumulate, const int32_t *order)
{
    int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g < npiv) {
        int32_t c = piv_cell[g];
        int32_t dst = tt_off[c] + ipos[g];
        if (order) dst = order[dst];
        out[dst] = accumulate ? out[dst] + u[g] : u[g];
        return;
    }
    g -= npiv;
    if (g >= nrem) return;
    int32_t c = rem_cell[g];
    int32_t po = piv_ptr[c], kk = piv_ptr[c + 1] - po;
    int32_t ro = rem_ptr[c], nr = rem_ptr[c + 1] - ro, r = (int32_t)g - ro;
    const double *Ct = crem_t + crem_off[c] + r;
    const double *ub = u + po;
    // eight independent partial sums keep eight loads in flight
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int32_t q = 0;
    for (; q + 7 < kk; q += 8) {
#pragma unroll
        for (int i = 0; i < 8; i++) a[i] += Ct[(int64_t)(q + i) * nr] * ub[q + i];
    }
    for (; q < kk; q++) a[0] += Ct[(int64_t)q * nr] * ub[q];
    double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    int32_t dst = tt_off[c] + rem_pos[g];
    if (order) dst = order[dst];
    out[dst] = accumulate ? out[dst] + acc : acc;
}

// ---------------------------------------------------------------------------
// Interaction kernels.  One workgroup per target cell.  Each thread carries R
// targets (register blocking); the cell's targets are covered by `tpg`
// threads and the workgroup holds G = 256 / tpg such groups, group g taking
// every G-th source of each 256-wide LDS tile.  Partial sums are formed in
// the working precision over CHUNK sources and folded into FP64.

constexpr int RB = 4;   // targets per thread

struct Split {
    int32_t cnt, tpg, G, ti, g;
    __device__ Split(int32_t total, int32_t base, int t)
    {
        cnt = total - base < NT * RB ? total - base : NT * RB;
        tpg = (cnt + RB - 1) / RB;
        G = NT / tpg;
        ti = t % tpg;
        g = t / tpg;
    }
};

// Arithmetic of one transverse-pass launch.
//   M_F32:    FP32 offsets from the cell centres, FP32 kernel and products,
//             FP32 partial sums of CHUNK terms folded into FP64.
//   M_F64:    FP64 throughout, K = 1/sqrt(r^2) correctly rounded (the plain
//             FP64 matvec).
//   M_F64R:   FP64 coordinates, differences and r^2; 1/r from an FP32
//             reciprocal-square-root seed and one FP64 Newton step (relative
//             error ~1e-14); FP64 products.  Used by the mixed matvec on the
//             coarse levels, whose rounding errors the nested interpolation
//             operators of all finer levels amplify.
enum { M_F32 = 0, M_F64 = 1, M_F64R = 2 };

template <int MODE> struct M2LTypes;
template <> struct M2LTypes<M_F32> { using C = float; using V = float4; };
template <> struct M2LTypes<M_F64> { using C = double; using V = double4; };
template <> struct M2LTypes<M_F64R> { using C = double; using V = double4; };

constexpr int ET = 256;   // interaction-list entries staged in LDS at a time

// transverse pass at one level: u^{B,i} = sum_{B' in IL(B)} K(t^{B,i}, s^{B',o}) w^{B',o}.
// Targets: the pivots of cell B (pc, piv_ptr); sources: the pivots of the IL
// cells (pcs, piv_ptr_s), which are the same arrays in the symmetric case
// (s^{B',o} = t^{B',i}) and the outgoing half's in the general case.
// Launched with nc * P workgroups: part p of a cell takes the p-th of P equal
// slices of its source list; with P > 1 the partial vectors go to `part_out`
// (P x npiv) and are added in a fixed order by k_sum_parts.
template <int KIND, int MODE, int TILE>
__global__ __launch_bounds__(NT) void k_m2l(int64_t nc, int P, const int32_t *k, const int32_t *piv_ptr,
                                            const int32_t *il_ptr, const int32_t *il, const int32_t *ilpre,
                                            const int32_t *ilsum,
                                            const typename M2LTypes<MODE>::C *pc, int64_t npiv,
                                            const typename M2LTypes<MODE>::C *pcs, int64_t npivs,
                                            const int32_t *piv_ptr_s,
                                            const int32_t *coord, const float *hc, float h0, int d,
                                            const double *w, double *u, double *part_out, double prm64,
                                            const int32_t *corder, int64_t slots)
{
    using T = typename M2LTypes<MODE>::C;
    using T4 = typename M2LTypes<MODE>::V;
    constexpr int SPT = TILE / NT;   // sources loaded per thread per tile
    // the source tile and, after the last tile of a target block, the
    // per-thread row sums share one LDS buffer
    constexpr size_t SRC_BYTES = sizeof(T4) * TILE, PART_BYTES = sizeof(double) * NT * RB;
    __shared__ __align__(16) unsigned char smem[SRC_BYTES > PART_BYTES ? SRC_BYTES : PART_BYTES];
    T4 *src = reinterpret_cast<T4 *>(smem);
    double *part = reinterpret_cast<double *>(smem);
    __shared__ int32_t est[ET + 1], ebase[ET];
    __shared__ float esh[3][ET];
    const int t = threadIdx.x;
    int64_t c;
    int pp;
    if (corder) {   // slot q / P of XCD x's run, part q % P
        const int64_t q = blockIdx.x >> 3;
        c = corder[(blockIdx.x & 7) * slots + q / P];
        pp = (int)(q % P);
        if (c < 0) return;   // padding slot (uniform exit)
    } else {
        c = blockIdx.x / P;
        pp = blockIdx.x % P;
    }
    const int32_t kk = k[c], po = piv_ptr[c], S = ilsum[c];
    const int32_t sb = (int32_t)(((int64_t)S * pp) / P), se = (int32_t)(((int64_t)S * (pp + 1)) / P);
    const int32_t e0 = il_ptr[c], e1 = il_ptr[c + 1];
    const T prm = (T)prm64;
    int32_t cc[3] = {coord[c], coord[nc + c], d == 3 ? coord[2 * nc + c] : 0};
    const float h = hc ? hc[c] : h0;   // cell side (per cell when the level mixes problems)
    double *dst = P > 1 ? part_out + (int64_t)pp * npiv : u;
    for (int32_t tb = 0; tb < kk; tb += NT * RB) {
        Split sp(kk, tb, t);
        const bool act = sp.g < sp.G;
        T tx[RB], ty[RB], tz[RB];
        double acc[RB];
#pragma unroll
        for (int r = 0; r < RB; r++) {
            int32_t i = sp.ti + r * sp.tpg;
            i = i < sp.cnt ? i : sp.cnt - 1;
            int32_t q = po + tb + i;
            tx[r] = pc[q];
            ty[r] = pc[npiv + q];
            tz[r] = d == 3 ? pc[2 * npiv + q] : T(0);
            acc[r] = 0.0;
        }
        // first list entry holding source sb
        int32_t efirst = e0;
        {
            int32_t lo = e0, hi = e1 - 1;
            while (lo < hi) {
                int32_t mid = (lo + hi + 1) >> 1;
                if (ilpre[mid] <= sb) lo = mid; else hi = mid - 1;
            }
            efirst = lo;
        }
        // windows of ET list entries staged in LDS: first source, pivot
        // base and (FP32 form) the cell offset of every entry
        for (int32_t w0 = efirst; w0 < e1; w0 += ET) {
            const int32_t wn = e1 - w0 < ET ? e1 - w0 : ET;
            __syncthreads();
            for (int32_t j = t; j < wn; j += NT) {
                const int32_t e = w0 + j, b = il[e], pre = ilpre[e];
                est[j] = pre;
                ebase[j] = piv_ptr_s[b] - pre;
                if (MODE == M_F32) {
                    esh[0][j] = (float)(coord[b] - cc[0]) * h;
                    esh[1][j] = (float)(coord[nc + b] - cc[1]) * h;
                    esh[2][j] = d == 3 ? (float)(coord[2 * nc + b] - cc[2]) * h : 0.f;
                }
            }
            if (t == 0) est[wn] = w0 + wn < e1 ? ilpre[w0 + wn] : S;
            __syncthreads();
            const int32_t ws = est[0] > sb ? est[0] : sb, we = est[wn] < se ? est[wn] : se;
            if (est[0] >= se) break;
        for (int32_t s0 = ws; s0 < we; s0 += TILE) {
            const int32_t send = we - s0 < TILE ? we : s0 + TILE;
            // contiguous sources per thread: one search, then at most a few steps
            T4 v[SPT];
            const int32_t sfirst = s0 + t * SPT;
            int32_t ej = 0;
            if (sfirst < send) {
                int32_t lo = 0, hi = wn - 1;
                while (lo < hi) {
                    int32_t mid = (lo + hi + 1) >> 1;
                    if (est[mid] <= sfirst) lo = mid; else hi = mid - 1;
                }
                ej = lo;
            }
#pragma unroll
            for (int q = 0; q < SPT; q++) {
                const int32_t s = sfirst + q;
                v[q].x = 0; v[q].y = 0; v[q].z = 0; v[q].w = 0;
                if (s < send) {
                    while (est[ej + 1] <= s) ej++;
                    const int32_t idx = ebase[ej] + s;
                    v[q].x = pcs[idx];
                    v[q].y = pcs[npivs + idx];
                    v[q].z = d == 3 ? pcs[2 * npivs + idx] : T(0);
                    v[q].w = (T)w[idx];
                    if (MODE == M_F32) {
                        v[q].x += esh[0][ej];
                        v[q].y += esh[1][ej];
                        v[q].z += esh[2][ej];
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < SPT; q++) src[t * SPT + q] = v[q];
            __syncthreads();
            const int32_t ns = send - s0;
            if (act) {
                if (MODE == M_F32) {
                    for (int32_t j = sp.g; j < ns;) {
                        int32_t je = j + CHUNK * sp.G < ns ? j + CHUNK * sp.G : ns;
                        T a[RB];
#pragma unroll
                        for (int r = 0; r < RB; r++) a[r] = T(0);
                        for (; j < je; j += sp.G) {
                            T4 q = src[j];
#pragma unroll
                            for (int r = 0; r < RB; r++) {
                                T dx = tx[r] - q.x, dy = ty[r] - q.y, dz = tz[r] - q.z;
                                T d2 = dx * dx + dy * dy + dz * dz;
                                a[r] += kv<KIND, T>(d2, prm) * q.w;
                            }
                        }
#pragma unroll
                        for (int r = 0; r < RB; r++) acc[r] += (double)a[r];
                    }
                } else {
                    for (int32_t j = sp.g; j < ns; j += sp.G) {
                        T4 q = src[j];
#pragma unroll
                        for (int r = 0; r < RB; r++) {
                            double dx = tx[r] - q.x, dy = ty[r] - q.y, dz = tz[r] - q.z;
                            double d2 = dx * dx + dy * dy + dz * dz;
                            double kvv = MODE == M_F64 ? kv64<KIND>(d2, prm64) : kv_refined<KIND, MODE>(d2, prm64);
                            acc[r] += kvv * q.w;
                        }
                    }
                }
            }
        }
        }
        __syncthreads();
        if (act)
#pragma unroll
            for (int r = 0; r < RB; r++) part[(sp.g * sp.tpg + sp.ti) * RB + r] = acc[r];
        __syncthreads();
        for (int32_t i = t; i < sp.cnt; i += NT) {
            int32_t ti = i % sp.tpg, r = i / sp.tpg;
            double sum = 0.0;
            for (int gg = 0; gg < sp.G; gg++) sum += part[(gg * sp.tpg + ti) * RB + r];
            dst[po + tb + i] = sum;
        }
        __syncthreads();
    }
}

// u = sum over p of the P partial vectors, in order p = 0, 1, ...
__global__ void k_sum_parts(int64_t npiv, int P, const double *part, double *u)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= npiv) return;
    double s = 0.0;
    for (int p = 0; p < P; p++) s += part[(int64_t)p * npiv + i];
    u[i] = s;
}

// near field of one leaf plus the combine: y = far + sum_{B' in N(B)} K x.
// Coordinates are FP64 in both precisions; the mixed path rounds the FP64
// coordinate differences to FP32 and evaluates K and the products in FP32
// on the split weights x_hi, x_lo (close pairs would otherwise lose their
// relative accuracy to the rounding of the coordinates themselves).  The far
// field and the partial results are added in FP64.
// Targets: the cell's points (first, count, pts); sources: the neighbours'
// points at sfirst in spts (the same arrays in the symmetric case; Q's in the
// general case).
template <typename T, int KIND>
__global__ __launch_bounds__(NT) void k_p2p(int64_t c0, const int32_t *first, const int32_t *count,
                                            const int32_t *nb_ptr, const int32_t *nb, const int32_t *nbpre,
                                            const int32_t *nbsum, const double *pts, int64_t n,
                                            const int32_t *sfirst, const double *spts, int64_t sn, int d,
                                            const T *xw, const T *xw2, const double *far,
                                            const int32_t *order, double *y, T prm)
{
    struct Src {
        double x, y, z;
        T w, w2;
    };
    __shared__ Src src[NT];
    __shared__ double part[NT * RB], part2[NT * RB];
    __shared__ int32_t est[ET + 1], ebase[ET];
    const int t = threadIdx.x;
    // leaf cell of this workgroup (launches may cover a range [c0, c1));
    // every array is indexed by global cell number, also first[] of the
    // neighbour cells below
    const int64_t c = c0 + blockIdx.x;
    const int32_t kk = count[c], po = first[c], S = nbsum[c];
    const int32_t e0 = nb_ptr[c], e1 = nb_ptr[c + 1];
    const bool mixed = sizeof(T) == 4;
    for (int32_t tb = 0; tb < kk; tb += NT * RB) {
        Split sp(kk, tb, t);
        const bool act = sp.g < sp.G;
        double tx[RB], ty[RB], tz[RB];
        double acc[RB], acc2[RB];
#pragma unroll
        for (int r = 0; r < RB; r++) {
            int32_t i = sp.ti + r * sp.tpg;
            i = i < sp.cnt ? i : sp.cnt - 1;
            int32_t q = po + tb + i;
            tx[r] = pts[q];
            ty[r] = pts[n + q];
            tz[r] = d == 3 ? pts[2 * n + q] : 0.0;
            acc[r] = 0.0;
            acc2[r] = 0.0;
        }
        // windows of ET neighbour entries staged in LDS (first source, point base)
        for (int32_t w0 = e0; w0 < e1; w0 += ET) {
            const int32_t wn = e1 - w0 < ET ? e1 - w0 : ET;
            __syncthreads();
            for (int32_t j = t; j < wn; j += NT) {
                const int32_t e = w0 + j, pre = nbpre[e];
                est[j] = pre;
                ebase[j] = sfirst[nb[e]] - pre;
            }
            if (t == 0) est[wn] = w0 + wn < e1 ? nbpre[w0 + wn] : S;
            __syncthreads();
            const int32_t ws = est[0], we = est[wn];
        for (int32_t s0 = ws; s0 < we; s0 += NT) {
            int32_t s = s0 + t;
            Src v;
            v.x = 0; v.y = 0; v.z = 0; v.w = 0; v.w2 = 0;
            if (s < we) {
                int32_t lo = 0, hi = wn - 1;
                while (lo < hi) {
                    int32_t mid = (lo + hi + 1) >> 1;
                    if (est[mid] <= s) lo = mid; else hi = mid - 1;
                }
                int32_t idx = ebase[lo] + s;
                v.x = spts[idx];
                v.y = spts[sn + idx];
                v.z = d == 3 ? spts[2 * sn + idx] : 0.0;
                v.w = xw[idx];
                if (mixed) v.w2 = xw2[idx];
            }
            __syncthreads();
            src[t] = v;
            __syncthreads();
            int32_t ns = we - s0 < NT ? we - s0 : NT;
            if (act) {
                for (int32_t j = sp.g; j < ns;) {
                    int32_t je = j + CHUNK * sp.G < ns ? j + CHUNK * sp.G : ns;
                    T a[RB], a2[RB];
#pragma unroll
                    for (int r = 0; r < RB; r++) { a[r] = T(0); a2[r] = T(0); }
                    for (; j < je; j += sp.G) {
                        const Src q = src[j];
#pragma unroll
                        for (int r = 0; r < RB; r++) {
                            T dx = (T)(tx[r] - q.x), dy = (T)(ty[r] - q.y), dz = (T)(tz[r] - q.z);
                            T d2 = dx * dx + dy * dy + dz * dz;
                            T kvv = kv_self<KIND, T>(d2, prm);
                            a[r] += kvv * q.w;
                            if (mixed) a2[r] += kvv * q.w2;
                        }
                    }
#pragma unroll
                    for (int r = 0; r < RB; r++) {
                        acc[r] += (double)a[r];
                        acc2[r] += (double)a2[r];
                    }
                }
            }
        }
        }
        __syncthreads();
        if (act)
#pragma unroll
            for (int r = 0; r < RB; r++) {
                part[(sp.g * sp.tpg + sp.ti) * RB + r] = acc[r];
                part2[(sp.g * sp.tpg + sp.ti) * RB + r] = acc2[r];
            }
        __syncthreads();
        for (int32_t i = t; i < sp.cnt; i += NT) {
            int32_t ti = i % sp.tpg, r = i / sp.tpg;
            double s1 = 0.0, s2 = 0.0;
            for (int gg = 0; gg < sp.G; gg++) {
                s1 += part[(gg * sp.tpg + ti) * RB + r];
                s2 += part2[(gg * sp.tpg + ti) * RB + r];
            }
            int32_t p = po + tb + i;
            double f = far ? far[p] : 0.0;
            y[order ? order[p] : p] = (f + s1) + s2;
        }
        __syncthreads();
    }
}

// dense FP64 direct sum for error reports: one target per thread
template <int KIND>
__global__ __launch_bounds__(NT) void k_direct(const double *p, int64_t n, int d, int64_t ld, const double *x,
                                               double *y, double prm)
{
    __shared__ double4 src[NT];
    int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x;
    double tx = 0, ty = 0, tz = 0;
    if (i < n) {
        tx = p[i];
        ty = p[ld + i];
        tz = d == 3 ? p[2 * ld + i] : 0.0;
    }
    double acc = 0.0;
    for (int64_t s0 = 0; s0 < n; s0 += NT) {
        int64_t s = s0 + threadIdx.x;
        double4 v = make_double4(0, 0, 0, 0);
        if (s < n) {
            v.x = p[s];
            v.y = p[ld + s];
            v.z = d == 3 ? p[2 * ld + s] : 0.0;
            v.w = x[s];
        }
        __syncthreads();
        src[threadIdx.x] = v;
        __syncthreads();
        int64_t ns = n - s0 < NT ? n - s0 : NT;
        for (int64_t j = 0; j < ns; j++) {
            double4 q = src[j];
            double dx = tx - q.x, dy = ty - q.y, dz = tz - q.z;
            double d2 = dx * dx + dy * dy + dz * dz;
            acc += kv_self<KIND, double>(d2, prm) * q.w;
        }
    }
    if (i < n) y[i] = acc;
}

// ---------------------------------------------------------------------------
// set-up kernels

__global__ void k_list_prefix(int64_t nc, const int32_t *ptr, const int32_t *lst, const int32_t *size,
                              int32_t *pre, int32_t *sum)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int32_t s = 0;
    for (int32_t e = ptr[c]; e < ptr[c + 1]; e++) {
        pre[e] = s;
        s += size[lst[e]];
    }
    sum[c] = s;
}

// FP64 coordinates of the pivots and their FP32 offsets from the cell centre
__global__ void k_pivot_coords(int64_t nc, const int32_t *piv_ptr, const int32_t *piv_id, const double *P,
                               int64_t n, int d, const int32_t *coord, double lo0, double lo1, double lo2,
                               double h, int64_t npiv, double *pc64, float *pc32)
{
    int64_t c = blockIdx.x;
    double lo[3] = {lo0, lo1, lo2};
    for (int32_t q = piv_ptr[c] + threadIdx.x; q < piv_ptr[c + 1]; q += blockDim.x) {
        int32_t id = piv_id[q];
        for (int a = 0; a < 3; a++) {
            double v = a < d ? P[a * n + id] : 0.0;
            double ctr = a < d ? lo[a] + ((double)coord[a * nc + c] + 0.5) * h : 0.0;
            pc64[a * npiv + q] = v;
            pc32[a * npiv + q] = (float)(v - ctr);
        }
    }
}

// owner cell of every entry of a CSR range array
__global__ void k_fill_owner(int64_t nc, const int32_t *ptr, int32_t *owner)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    for (int32_t e = ptr[c]; e < ptr[c + 1]; e++) owner[e] = (int32_t)c;
}

// per-cell (m-k) x k blocks -> k x (m-k)
__global__ void k_transpose_blocks(int64_t nc, const int32_t *piv_ptr, const int32_t *rem_ptr,
                                   const int64_t *crem_off, const double *a, double *at)
{
    int64_t c = blockIdx.x;
    int32_t kk = piv_ptr[c + 1] - piv_ptr[c], nr = rem_ptr[c + 1] - rem_ptr[c];
    const double *src = a + crem_off[c];
    double *dst = at + crem_off[c];
    for (int32_t e = threadIdx.x; e < kk * nr; e += blockDim.x) {
        int32_t r = e / kk, q = e % kk;
        dst[(int64_t)q * nr + r] = src[e];
    }
}

// Symmetric transverse pass of one level.  K(x, y) = K(y, x) and B' in IL(B)
// <=> B in IL(B'), so the block of the pair (B', B) is the transpose of the
// block of (B, B').  The workgroups of cell B take the pairs it owns: for
// each source pivot s of an owned partner B' they form K(t^{B,i}, s) once and
// use it twice, for the row sums u^{B,i} += K w^{B',o} (in registers) and for
// the column sum (K^T w^{B,o})_s (over a thread's targets, then over the
// lanes of its group), which goes to the pair's slot of the column buffer.
// k_m2l_gather then adds to every cell the slots of the pairs its partners
// own, in list order.  Two arithmetic forms, as in the plain pass:
//   M_F32   cell-local FP32 coordinates, FP32 kernel and products, row sums
//           in FP32 chunks folded into FP64, FP32 column slots;
//   M_F64R  FP64 coordinates and products, 1/r from an FP32 seed and one
//           FP64 Newton step, FP64 column slots (the coarse levels of the
//           mixed matvec);
//   M_F64   FP64 throughout: coordinate differences, K = 1/sqrt(r^2)
//           correctly rounded, FP64 products and column slots (the FP64
//           matvec: the same schedule as the mixed one, only the arithmetic
//           differs).
// Levels with few cells split each cell's owned sources over P workgroups;
// their row sums go to P partial vectors added in order by k_sum_parts.

// Sum over an aligned group of TPG (a power of two, at most 32) lanes, left
// in every lane of the group: DPP quad permutations (xor 1, xor 2) and row
// mirrors (lane i <-> 7 - i, then i <-> 15 - i, each pairing the two halves
// of the group so far), then a swizzle exchanging the 16-lane halves.  The
// exchanges move bits, so an FP64 value moves as two 32-bit halves.
template <int CTRL>
__device__ inline float lane_xchg(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double lane_xchg(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false),
                            __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false));
}
__device__ inline float swap16(float v) { return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F)); }
__device__ inline double swap16(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_ds_swizzle(hi, 0x401F), __builtin_amdgcn_ds_swizzle(lo, 0x401F));
}
template <int TPG, typename T>
__device__ inline T group_sum(T v)
{
    if (TPG > 1) v += lane_xchg<0xB1>(v);
    if (TPG > 2) v += lane_xchg<0x4E>(v);
    if (TPG > 4) v += lane_xchg<0x141>(v);
    if (TPG > 8) v += lane_xchg<0x140>(v);
    if (TPG > 16) v += swap16(v);
    return v;
}

// a load at a 32-bit byte offset from a base pointer (the base stays in
// scalar registers; no 64-bit address arithmetic per lane)
template <typename T>
__device__ inline T ld_off(const T *base, uint32_t byte_off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

constexpr int SYM_MAXK = 256;   // largest rank of a level on this pass (one target tile)
constexpr int SYM_TS = 512;     // sources per LDS tile

struct SymArgs {
    const int32_t *k, *piv_ptr, *own_ptr, *own_il, *own_pre, *own_sum, *own_slot;
    const float *pc32;
    const double *pc64;
    int64_t npiv, nc;
    const int32_t *coord;
    const float *hc;
    float h0;
    int d, P;
    const double *w;
    double *u, *part;
    float *col32;
    double *col64;
    double prm;
    const int32_t *corder;   // 8 runs of `slots` cells (one per XCD), -1 = empty
    int64_t slots;
};

template <int MODE> struct SymT;
template <> struct SymT<M_F32> { using T = float; using T4 = float4; };
template <> struct SymT<M_F64R> { using T = double; using T4 = double4; };
template <> struct SymT<M_F64> { using T = double; using T4 = double4; };

template <int MODE>
struct SymShared {
    using T4 = typename SymT<MODE>::T4;
    union {   // the tiles, then (after the last tile) the per-thread row sums
        struct {
            T4 src[SYM_TS];
            int32_t sslot[SYM_TS];
            typename SymT<MODE>::T sn[SYM_TS];   // |s|^2 of the (shifted) source
            typename SymT<MODE>::T scol[SYM_TS];   // column sums of the tile's sources
        } tile;
        double part[NT * 8];
    } u;
    int32_t est[ET + 1], ebase[ET], eslot[ET];
    float esh[3][ET];
};

// Part pp of cell c.  Targets: groups of TPG lanes (aligned inside a
// wavefront, TPG * R >= k), G = NT / TPG groups; target i is held by lane
// i % TPG as its (i / TPG)-th register.  Group g takes sources g, g + G, ...
// of each tile; all its lanes run the same sources, so the column partial of
// a source is summed inside the group by group_sum (a butterfly: every lane
// of the group ends with the sum), written to the tile's column slots in LDS
// and flushed to the column buffer after the tile.  Tiles are padded to whole
// rounds of G sources with zero-weight sources far from every target, so all
// groups run the same number of steps.
//
// r^2 = |t|^2 + |s|^2 - 2 t.s: one addition and three FMAs per pair with -2t
// and |t|^2 per target and |s|^2 per source, against three differences, a
// product and two FMAs.  FP32 form: in the target cell's frame, where |t|,
// |s| are at most a few cell widths and an admissible r is at least one, so
// the cancellation costs a few units in the last place of r^2.  FP64-refined
// form: absolute coordinates, (|t|^2 + |s|^2) / r^2 at most a few thousand
// (a relative error of r^2 below 1e-12, far under the FP32 rounding of the
// finer levels).  FP64 form: r^2 from the coordinate differences, as in the
// plain pass.
template <int KIND, int MODE, int TPG, int R>
__device__ void sym_cell(const SymArgs &A, SymShared<MODE> &sh, int64_t c, int pp, int32_t kk)
{
    using T = typename SymT<MODE>::T;
    using T4 = typename SymT<MODE>::T4;
    constexpr bool F32 = MODE == M_F32;
    constexpr bool DIFF = MODE == M_F64;   // r^2 from coordinate differences
    constexpr int G = NT / TPG;
    constexpr int SPT = SYM_TS / NT;
    const int t = threadIdx.x, g = t / TPG, ti = t % TPG;
    const int32_t po = A.piv_ptr[c], S = A.own_sum[c];
    const int32_t sb = (int32_t)(((int64_t)S * pp) / A.P), se = (int32_t)(((int64_t)S * (pp + 1)) / A.P);
    const int32_t e0 = A.own_ptr[c], e1 = A.own_ptr[c + 1];
    const int64_t nc = A.nc, npiv = A.npiv;
    const int d = A.d;
    const int32_t cc[3] = {A.coord[c], A.coord[nc + c], d == 3 ? A.coord[2 * nc + c] : 0};
    const float h = A.hc ? A.hc[c] : A.h0;
    const T *pc;
    if constexpr (F32) pc = A.pc32; else pc = A.pc64;
    double *dst = A.P > 1 ? A.part + (int64_t)pp * npiv : A.u;
    T tx[R], ty[R], tz[R], tw[R], tn[R];
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int32_t i = ti + r * TPG;
        const bool ok = i < kk;
        const int32_t q = po + (ok ? i : 0);
        tx[r] = pc[q];
        ty[r] = pc[npiv + q];
        tz[r] = d == 3 ? pc[2 * npiv + q] : T(0);
        tw[r] = ok ? (T)A.w[q] : T(0);   // padding targets add nothing to column sums
        acc[r] = 0.0;
        if constexpr (!DIFF) {
            tn[r] = tx[r] * tx[r] + ty[r] * ty[r] + tz[r] * tz[r];
            tx[r] *= T(-2);
            ty[r] *= T(-2);
            tz[r] *= T(-2);
        }
    }
    const T prm = (T)A.prm;
    // first owned entry holding source sb
    int32_t efirst = e0;
    {
        int32_t lo = e0, hi = e1 - 1;
        while (lo < hi) {
            int32_t mid = (lo + hi + 1) >> 1;
            if (A.own_pre[mid] <= sb) lo = mid; else hi = mid - 1;
        }
        efirst = lo;
    }
    for (int32_t w0 = efirst; w0 < e1; w0 += ET) {
        const int32_t wn = e1 - w0 < ET ? e1 - w0 : ET;
        __syncthreads();
        for (int32_t j = t; j < wn; j += NT) {
            const int32_t e = w0 + j, b = A.own_il[e], pre = A.own_pre[e];
            sh.est[j] = pre;
            sh.ebase[j] = A.piv_ptr[b] - pre;
            sh.eslot[j] = A.own_slot[e];
            if (F32) {
                sh.esh[0][j] = (float)(A.coord[b] - cc[0]) * h;
                sh.esh[1][j] = (float)(A.coord[nc + b] - cc[1]) * h;
                sh.esh[2][j] = d == 3 ? (float)(A.coord[2 * nc + b] - cc[2]) * h : 0.f;
            }
        }
        if (t == 0) sh.est[wn] = w0 + wn < e1 ? A.own_pre[w0 + wn] : S;
        for (int32_t j = wn + 1 + t; j <= ET; j += NT) sh.est[j] = INT32_MAX;   // past the window
        __syncthreads();
        if (sh.est[0] >= se) break;
        const int32_t ws = sh.est[0] > sb ? sh.est[0] : sb, we = sh.est[wn] < se ? sh.est[wn] : se;
        for (int32_t s0 = ws; s0 < we; s0 += SYM_TS) {
            const int32_t ns = we - s0 < SYM_TS ? we - s0 : SYM_TS;
            // contiguous sources per thread: one search, then a few steps
            T4 v[SPT];
            int32_t sl[SPT];
            T sn[SPT];
            const int32_t sfirst = s0 + t * SPT;
            // the last entry starting at or before sfirst: a fixed, branchless
            // search over the ET + 1 starts (est[0] <= sfirst for every source
            // of the window; starts past the window are INT32_MAX)
            int32_t lo = 0;
#pragma unroll
            for (int hstep = ET / 2; hstep >= 1; hstep >>= 1) lo = sh.est[lo + hstep] <= sfirst ? lo + hstep : lo;
#pragma unroll
            for (int q = 0; q < SPT; q++) {
                const int32_t s = sfirst + q;
                // every list entry holds at least one source (cells without
                // pivots own no pairs and are no partners): one step at most
                if (q > 0) lo = sh.est[lo + 1] <= s ? lo + 1 : lo;
                if (s >= s0 + ns) {   // padding of a round: weight 0, far from every target
                    v[q].x = T(1e15); v[q].y = v[q].x; v[q].z = v[q].x; v[q].w = 0;
                    sl[q] = 0;
                    sn[q] = T(3e30);
                } else {
                    // 32-bit byte offsets from the arrays' bases (scalar registers)
                    const uint32_t idx = (uint32_t)(sh.ebase[lo] + s);
                    v[q].x = ld_off(pc, idx * (uint32_t)sizeof(T));
                    v[q].y = ld_off(pc + npiv, idx * (uint32_t)sizeof(T));
                    v[q].z = d == 3 ? ld_off(pc + 2 * npiv, idx * (uint32_t)sizeof(T)) : T(0);
                    v[q].w = (T)ld_off(A.w, idx * 8u);
                    if (F32) {
                        v[q].x += sh.esh[0][lo];
                        v[q].y += sh.esh[1][lo];
                        v[q].z += sh.esh[2][lo];
                    }
                    if constexpr (!DIFF) sn[q] = v[q].x * v[q].x + v[q].y * v[q].y + v[q].z * v[q].z;
                    else sn[q] = T(0);
                    sl[q] = sh.eslot[lo] + s;
                }
            }
            __syncthreads();   // the previous tile is done with src and sslot
#pragma unroll
            for (int q = 0; q < SPT; q++) {
                const int32_t pos = t * SPT + q;
                sh.u.tile.src[pos] = v[q];
                sh.u.tile.sslot[pos] = sl[q];
                sh.u.tile.sn[pos] = sn[q];
            }
            __syncthreads();
            T a[R];
#pragma unroll
            for (int r = 0; r < R; r++) a[r] = T(0);
            const int32_t nr = (ns + G - 1) / G;   // rounds: source g + it G in round it
            // a wave in its rounds issues ahead of waves staging a tile (the
            // SIMD's arbiter otherwise favours the older wave): c2 leaf
            // 0.77-0.78 against 0.79-0.80 ms per launch
            __builtin_amdgcn_s_setprio(1);
            for (int it = 0; it < nr; it++) {
                const int32_t j = g + it * G;
                const T4 q = sh.u.tile.src[j];
                T qn = T(0);
                qn = sh.u.tile.sn[j];
                T cp = T(0);
#pragma unroll
                for (int r = 0; r < R; r++) {
                    T kv_;
                    T r2;
                    if constexpr (DIFF) {
                        const T dx = tx[r] - q.x, dy = ty[r] - q.y, dz = tz[r] - q.z;
                        r2 = (dx * dx + dy * dy) + dz * dz;
                    } else {
                        r2 = tn[r] + qn;
                        r2 = fma(tz[r], q.z, r2);
                        r2 = fma(ty[r], q.y, r2);
                        r2 = fma(tx[r], q.x, r2);
                    }
                    if constexpr (F32) kv_ = kv32<KIND>(r2, prm);
                    else if constexpr (DIFF) kv_ = kv64<KIND>(r2, prm);
                    else kv_ = kv_refined<KIND, MODE>(r2, prm);
                    a[r] += kv_ * q.w;
                    cp += kv_ * tw[r];
                }
                sh.u.tile.scol[j] = group_sum<TPG>(cp);   // the same value from every lane of the group
                // (the tile's last round folds after the loop)
                if (F32 && (it & (CHUNK - 1)) == CHUNK - 1 && it + 1 < nr) {
#pragma unroll
                    for (int r = 0; r < R; r++) {
                        acc[r] += (double)a[r];
                        a[r] = T(0);
                    }
                }
            }
            __builtin_amdgcn_s_setprio(0);
            __syncthreads();
            for (int32_t j = t; j < ns; j += NT) {
                if constexpr (F32) A.col32[sh.u.tile.sslot[j]] = sh.u.tile.scol[j];
                else A.col64[sh.u.tile.sslot[j]] = sh.u.tile.scol[j];
            }
#pragma unroll
            for (int r = 0; r < R; r++) acc[r] += (double)a[r];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; r++) sh.u.part[(g * TPG + ti) * R + r] = acc[r];
    __syncthreads();
    for (int32_t i = t; i < kk; i += NT) {
        const int32_t li = i % TPG, r = i / TPG;
        double sum = 0.0;
        for (int gg = 0; gg < G; gg++) sum += sh.u.part[(gg * TPG + li) * R + r];
        dst[po + i] = sum;
    }
}

// Shape sets, picked per level from its largest rank: the registers of the
// largest shape in a kernel set its occupancy.  SET 0 (ranks <= 80): at most
// five registers per lane (80 VGPRs, six waves per SIMD); SET 1 (<= 224): at
// most seven (five waves); SET 2: SET 1 and eight registers per lane for
// ranks above 224; SET 3 (the FP64-refined form up to rank 160): at most
// five registers per lane, wider groups for the larger ranks.
template <int KIND, int MODE, int SET>
__global__ __launch_bounds__(NT) void k_m2l_sym(SymArgs A)
{
    __shared__ SymShared<MODE> sh;
    // slot q / P of XCD x's run (see prepare_symmetric), part q % P
    const int x = blockIdx.x & 7;
    const int64_t q = blockIdx.x >> 3;
    const int64_t c = A.corder[x * A.slots + q / A.P];
    const int pp = (int)(q % A.P);
    if (c < 0) return;   // padding slot (uniform exit)
    const int32_t kk = A.k[c];
    if (kk == 0) return;   // such a cell owns no pairs and has no rows (uniform exit)
    // lanes per group and registers per lane fitted to the rank
    if (kk <= 8) sym_cell<KIND, MODE, 2, 4>(A, sh, c, pp, kk);
    else if (kk <= 16) sym_cell<KIND, MODE, 4, 4>(A, sh, c, pp, kk);
    else if (kk <= 20) sym_cell<KIND, MODE, 4, 5>(A, sh, c, pp, kk);
    else if constexpr (SET == 0 || SET == 3) {
        if (kk <= 24) sym_cell<KIND, MODE, 8, 3>(A, sh, c, pp, kk);
        else if (kk <= 32) sym_cell<KIND, MODE, 8, 4>(A, sh, c, pp, kk);
        else if (kk <= 40) sym_cell<KIND, MODE, 8, 5>(A, sh, c, pp, kk);
        else if (kk <= 48) sym_cell<KIND, MODE, 16, 3>(A, sh, c, pp, kk);
        else if (kk <= 64) sym_cell<KIND, MODE, 16, 4>(A, sh, c, pp, kk);
        else if (SET == 0 || kk <= 80) sym_cell<KIND, MODE, 16, 5>(A, sh, c, pp, kk);
        else if constexpr (SET == 3) {
            if (kk <= 96) sym_cell<KIND, MODE, 32, 3>(A, sh, c, pp, kk);
            else if (kk <= 128) sym_cell<KIND, MODE, 32, 4>(A, sh, c, pp, kk);
            else sym_cell<KIND, MODE, 32, 5>(A, sh, c, pp, kk);
        }
    } else {
        if (kk <= 24) sym_cell<KIND, MODE, 4, 6>(A, sh, c, pp, kk);
        else if (kk <= 28) sym_cell<KIND, MODE, 4, 7>(A, sh, c, pp, kk);
        else if (kk <= 32) sym_cell<KIND, MODE, 8, 4>(A, sh, c, pp, kk);
        else if (kk <= 40) sym_cell<KIND, MODE, 8, 5>(A, sh, c, pp, kk);
        else if (kk <= 48) sym_cell<KIND, MODE, 8, 6>(A, sh, c, pp, kk);
        else if (kk <= 56) sym_cell<KIND, MODE, 8, 7>(A, sh, c, pp, kk);
        else if (kk <= 64) sym_cell<KIND, MODE, 16, 4>(A, sh, c, pp, kk);
        else if (kk <= 80) sym_cell<KIND, MODE, 16, 5>(A, sh, c, pp, kk);
        else if (kk <= 96) sym_cell<KIND, MODE, 16, 6>(A, sh, c, pp, kk);
        else if (kk <= 112) sym_cell<KIND, MODE, 16, 7>(A, sh, c, pp, kk);
        else if (kk <= 128) sym_cell<KIND, MODE, 32, 4>(A, sh, c, pp, kk);
        else if (kk <= 160) sym_cell<KIND, MODE, 32, 5>(A, sh, c, pp, kk);
        else if (kk <= 192) sym_cell<KIND, MODE, 32, 6>(A, sh, c, pp, kk);
        else if (SET == 1 || kk <= 224) sym_cell<KIND, MODE, 32, 7>(A, sh, c, pp, kk);
        else if constexpr (SET == 2) sym_cell<KIND, MODE, 32, 8>(A, sh, c, pp, kk);
    }
}

// u^{B,i} += the column sums of the pairs owned by B's partners, in list order
template <typename C>
__global__ void k_m2l_gather(int64_t npiv, const int32_t *piv_cell, const int32_t *piv_ptr, const int32_t *non_ptr,
                             const int32_t *non_slot, const C *colbuf, double *u)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= npiv) return;
    const int32_t c = piv_cell[g], j = (int32_t)g - piv_ptr[c];
    double sum = u[g];
    int32_t e = non_ptr[c];
    const int32_t e1 = non_ptr[c + 1];
    // eight independent loads in flight, added in list order
    for (; e + 8 <= e1; e += 8) {
        C v[8];
#pragma unroll
        for (int q = 0; q < 8; q++) v[q] = colbuf[non_slot[e + q] + j];
#pragma unroll
        for (int q = 0; q < 8; q++) sum += (double)v[q];
    }
    for (; e < e1; e++) sum += (double)colbuf[non_slot[e] + j];
    u[g] = sum;
}

// Sources per LDS tile: long inner loops also for cells with few targets.
constexpr int M2L_TILE = 4 * NT;

// Split factor: enough workgroups to fill the chip on levels with few cells
// and to even out cells of unequal work, about 16384 per level (the plain
// pass at 2^20 points: mixed 3.97 against 4.21 ms per matvec with 4096, FP64
// 17.7 against 18.4 ms; the general product likewise)
static int m2l_parts(const nnca::Level &L)
{
    const int64_t want = 16384;
    if (L.ncell >= want) return 1;
    int64_t P = (want + L.ncell - 1) / L.ncell;
    int64_t maxp = (L.max_ilsum + 1023) / 1024;   // keep at least ~1k sources per part
    if (P > maxp) P = maxp;
    if (P > 64) P = 64;
    return P < 1 ? 1 : (int)P;
}

// transverse pass of level L with the sources of level S (S = L in the
// symmetric case; the other half in the general case): targets at pc,
// sources at pcs, local vectors into L.u64 from the multipole vectors S.w64
template <int MODE, typename C>
static void launch_m2l_pair(int kind, nnca_h2 *H, const nnca::Level &L, const nnca::Level &S, const C *pc,
                            const C *pcs, double prm, hipStream_t s, hipEvent_t after = nullptr)
{
    const int64_t nc = L.ncell;
    const int P = m2l_parts(L);
    double *part = nullptr;
    if (P > 1) {
        if (H->m2l_part_cap < (int64_t)P * L.npiv) fail(NNCA_ERR_INTERNAL, "split workspace not sized");
        part = H->m2l_part;
    }
    const int g = L.m2l_order ? (int)(8 * L.m2l_slots * P) : (int)(nc * P);
#define M2L_ARGS nc, P, L.k, L.piv_ptr, L.il_ptr, L.il, L.ilpre, L.ilsum, pc, L.npiv, pcs, S.npiv, S.piv_ptr, L.coord, L.hcell, (float)L.h, H->dim, S.w64, L.u64, part, prm, L.m2l_order, L.m2l_slots
#define M2L_CASE(K) k_m2l<K, MODE, M2L_TILE><<<g, NT, 0, s>>>(M2L_ARGS);
    if (kind == NNCA_K_INV_R) { M2L_CASE(NNCA_K_INV_R) }
    else if (kind == NNCA_K_LOG_R) { M2L_CASE(NNCA_K_LOG_R) }
    else if (kind == NNCA_K_LOG_REG) { M2L_CASE(NNCA_K_LOG_REG) }
    else if (kind == NNCA_K_INV_REG) { M2L_CASE(NNCA_K_INV_REG) }
    else if (kind == NNCA_K_EXP_R) { M2L_CASE(NNCA_K_EXP_R) }
    else if (kind == K_GAUSS_DH) { M2L_CASE(K_GAUSS_DH) }
    else { M2L_CASE(NNCA_K_GAUSS) }
#undef M2L_CASE
#undef M2L_ARGS
    HIPCHECK(hipGetLastError());
    if (after) HIPCHECK(hipEventRecord(after, s));
    if (P > 1) {
        k_sum_parts<<<grid_for(L.npiv, 256), 256, 0, s>>>(L.npiv, P, part, L.u64);
        HIPCHECK(hipGetLastError());
    }
}

template <int MODE, typename C>
static void launch_m2l_mode(int kind, nnca_h2 *H, const nnca::Level &L, const C *pc, double prm, hipStream_t s,
                            hipEvent_t after = nullptr)
{
    launch_m2l_pair<MODE, C>(kind, H, L, L, pc, pc, prm, s, after);
}

// split factor of the symmetric pass, on the owned sources: enough
// workgroups for about 8192 per level (two per cell at level kappa-1 of the
// 2^20 cube, whose 4096 cells vary in work; with the XCD-aware, largest-
// first launch order 0.73 ms per launch against 0.745 for four parts, 0.77
// for eight; in cell order four parts had been best, 0.80 against 0.89-0.91
// ms unsplit; the leaf level's 32768 cells run unsplit)
static int sym_parts(const nnca::Level &L)
{
    const int64_t want = 8192;
    if (L.ncell >= want) return 1;
    int64_t P = (want + L.ncell - 1) / L.ncell;
    int64_t maxp = (L.max_own + 1023) / 1024;
    if (P > maxp) P = maxp;
    if (P > 64) P = 64;
    return P < 1 ? 1 : (int)P;
}

template <int KIND, int MODE>
static void sym_launch(int32_t max_k, int g, const SymArgs &A, hipStream_t s)
{
    if constexpr (MODE != M_F32)
        if (max_k > 80 && max_k <= 160) {
            k_m2l_sym<KIND, MODE, 3><<<g, NT, 0, s>>>(A);
            return;
        }
    if (max_k <= 80) k_m2l_sym<KIND, MODE, 0><<<g, NT, 0, s>>>(A);
    else if (max_k <= 224) k_m2l_sym<KIND, MODE, 1><<<g, NT, 0, s>>>(A);
    else k_m2l_sym<KIND, MODE, 2><<<g, NT, 0, s>>>(A);
}

// `after`, if given, is recorded on s right after the transverse kernel
// (before its combine step).
template <int MODE>
static void launch_m2l_sym(int kind, nnca_h2 *H, const nnca::Level &L, int level, double prm, hipStream_t s,
                           hipEvent_t after = nullptr)
{
    const int64_t nc = L.ncell;
    const int P = sym_parts(L);
    double *part = nullptr;
    if (P > 1) {
        if (H->m2l_part_cap < (int64_t)P * L.npiv) fail(NNCA_ERR_INTERNAL, "split workspace not sized");
        part = H->m2l_part;
    }
    {
        Span sp(H, s, PASS_M2L, level);
        // the cells of rank <= 80 (all cells when the level is not split),
        // then those above
        for (int cls = 0; cls < 2; cls++) {
            const int64_t slots = cls == 0 ? L.sym_slots : L.sym_slots_hi;
            if (slots == 0) continue;
            const int32_t mk = cls == 0 && L.sym_slots_hi > 0 ? 80 : L.max_k;
            SymArgs A{L.k, L.piv_ptr, L.own_ptr, L.own_il, L.own_pre, L.own_sum, L.own_slot, L.pc32, L.pc64, L.npiv,
                      nc, L.coord, L.hcell, (float)L.h, H->dim, P, L.w64, L.u64, part, L.col32, L.col64, prm,
                      L.sym_order + (cls == 0 ? 0 : 8 * L.sym_slots), slots};
            const int g = (int)(8 * slots * P);
#define SYM_CASE(K) sym_launch<K, MODE>(mk, g, A, s)
            if (kind == NNCA_K_INV_R) SYM_CASE(NNCA_K_INV_R);
            else if (kind == NNCA_K_LOG_R) SYM_CASE(NNCA_K_LOG_R);
            else if (kind == NNCA_K_LOG_REG) SYM_CASE(NNCA_K_LOG_REG);
            else if (kind == NNCA_K_INV_REG) SYM_CASE(NNCA_K_INV_REG);
            else if (kind == NNCA_K_EXP_R) SYM_CASE(NNCA_K_EXP_R);
            else if (kind == K_GAUSS_DH) SYM_CASE(K_GAUSS_DH);
            else SYM_CASE(NNCA_K_GAUSS);
#undef SYM_CASE
            HIPCHECK(hipGetLastError());
        }
    }
    if (after) HIPCHECK(hipEventRecord(after, s));
    Span sp(H, s, PASS_M2L_COMBINE, level);
    if (P > 1) {
        k_sum_parts<<<grid_for(L.npiv, 256), 256, 0, s>>>(L.npiv, P, part, L.u64);
        HIPCHECK(hipGetLastError());
    }
    if (MODE == M_F32)
        k_m2l_gather<float><<<grid_for(L.npiv, 256), 256, 0, s>>>(L.npiv, L.piv_cell, L.piv_ptr, L.non_ptr,
                                                                  L.non_slot, L.col32, L.u64);
    else
        k_m2l_gather<double><<<grid_for(L.npiv, 256), 256, 0, s>>>(L.npiv, L.piv_cell, L.piv_ptr, L.non_ptr,
                                                                   L.non_slot, L.col64, L.u64);
    HIPCHECK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Symmetric near field (mixed matvec).  K(x,y) = K(y,x) and B' in N(B) <=>
// B in N(B') make the near block of (B', B) the transpose of that of (B, B')
// (Sec. 5), so each pair of distinct neighbouring leaves is evaluated by one
// of them, its owner (the rule of the symmetric transverse pass).  A
// workgroup of the owner B takes B's points as targets: first its own points
// as sources (row sums only; 1/r and log vanish at r = 0), then the points of
// its owned neighbours, each kernel value used for the row sums of B (x_hi
// and x_lo parts, FP32 chunks folded into FP64) and for the column sums of
// the neighbour's point (over a thread's targets and the lanes of its group,
// FP32 slots).  k_p2p_gather then adds to every point its row sums and the
// slots of the pairs its neighbours own, in list order, and writes y.
// Coordinate differences in FP64, rounded to FP32, as in k_p2p.
constexpr int PS_TS = NT;      // sources per tile
constexpr int PS_ME = 128;     // owned neighbour entries per cell (at most 127)

struct P2PSymArgs {
    const int32_t *first, *count, *own_ptr, *own_nb, *own_pre, *own_sum, *own_slot;
    const double *pts;
    int64_t n;
    int d;
    const float *xhi, *xlo;
    float *col_hi, *col_lo;
    double *row;
    float prm;
};

struct P2PSrc {
    double x, y, z;
    float whi, wlo;
};

struct P2PSymShared {
    union {   // the tiles, then the per-thread row sums
        struct {
            P2PSrc src[PS_TS];
            int32_t sslot[PS_TS];
            float shi[PS_TS], slo[PS_TS];
        } tile;
        double part[NT * 4 * 2];
    } u;
    int32_t est[PS_ME + 1], ebase[PS_ME], eslot[PS_ME];
};

template <int KIND, int TPG, int R>
__device__ __attribute__((always_inline)) inline void p2p_sym_cell(const P2PSymArgs &A, P2PSymShared &sh, int64_t c,
                                                                   int32_t kk)
{
    constexpr int G = NT / TPG;
    const int t = threadIdx.x, g = t / TPG, ti = t % TPG;
    const int64_t n = A.n;
    const int d = A.d;
    const int32_t po = A.first[c];
    double tx[R], ty[R], tz[R], acc[R];
    float whi[R], wlo[R], a[R], a2[R];   // a2: the x_lo part, ~6e-8 of the sum: FP32 throughout
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int32_t i = ti + r * TPG;
        const bool ok = i < kk;
        const int32_t q = po + (ok ? i : 0);
        tx[r] = A.pts[q];
        ty[r] = A.pts[n + q];
        tz[r] = d == 3 ? A.pts[2 * n + q] : 0.0;
        whi[r] = ok ? A.xhi[q] : 0.f;   // padding targets add nothing to column sums
        wlo[r] = ok ? A.xlo[q] : 0.f;
        acc[r] = 0.0;
        a[r] = 0.f;
        a2[r] = 0.f;
    }
    auto fold = [&]() {
#pragma unroll
        for (int r = 0; r < R; r++) {
            acc[r] += (double)a[r];
            a[r] = 0.f;
        }
    };
    // source position p of a tile: point idx, or padding (zero weight, far
    // from every target: finite kernel values)
    auto stage = [&](int32_t p, bool real, int32_t idx, int32_t slot) {
        P2PSrc v;
        if (real) {
            v.x = A.pts[idx];
            v.y = A.pts[n + idx];
            v.z = d == 3 ? A.pts[2 * n + idx] : 0.0;
            v.whi = A.xhi[idx];
            v.wlo = A.xlo[idx];
        } else {
            v.x = 1e15;
            v.y = 1e15;
            v.z = 1e15;
            v.whi = 0.f;
            v.wlo = 0.f;
        }
        sh.u.tile.src[p] = v;
        sh.u.tile.sslot[p] = slot;
    };
    // 1. the cell's own points: row sums only
    for (int32_t s0 = 0; s0 < kk; s0 += PS_TS) {
        const int32_t ns = kk - s0 < PS_TS ? kk - s0 : PS_TS;
        __syncthreads();
        stage(t, t < ns, po + s0 + t, 0);
        __syncthreads();
        const int32_t nr = (ns + G - 1) / G;
        for (int it = 0; it < nr; it++) {
            const P2PSrc q = sh.u.tile.src[g + it * G];
#pragma unroll
            for (int r = 0; r < R; r++) {
                const float dx = (float)(tx[r] - q.x), dy = (float)(ty[r] - q.y), dz = (float)(tz[r] - q.z);
                const float kv_ = kv_self<KIND, float>(dx * dx + dy * dy + dz * dz, A.prm);
                a[r] += kv_ * q.whi;
                a2[r] += kv_ * q.wlo;
            }
            if ((it & (CHUNK - 1)) == CHUNK - 1) fold();
        }
        fold();
    }
    // 2. the owned neighbours' points: row and column sums
    const int32_t e0 = A.own_ptr[c], ne = A.own_ptr[c + 1] - e0, S = A.own_sum[c];
    __syncthreads();
    for (int32_t j = t; j < ne; j += NT) {
        const int32_t e = e0 + j, b = A.own_nb[e], pre = A.own_pre[e];
        sh.est[j] = pre;
        sh.ebase[j] = A.first[b] - pre;
        sh.eslot[j] = A.own_slot[e];
    }
    for (int32_t j = ne + t; j <= PS_ME; j += NT) sh.est[j] = j == ne ? S : INT32_MAX;
    for (int32_t s0 = 0; s0 < S; s0 += PS_TS) {
        const int32_t ns = S - s0 < PS_TS ? S - s0 : PS_TS;
        __syncthreads();   // entry table ready; the previous tile's slots flushed
        {
            const int32_t s = s0 + t;
            int32_t lo = 0;
#pragma unroll
            for (int h = PS_ME / 2; h >= 1; h >>= 1) lo = sh.est[lo + h] <= s ? lo + h : lo;
            const bool real = t < ns;
            stage(t, real, real ? sh.ebase[lo] + s : 0, real ? sh.eslot[lo] + s : 0);
        }
        __syncthreads();
        const int32_t nr = (ns + G - 1) / G;
        for (int it = 0; it < nr; it++) {
            const int32_t j = g + it * G;
            const P2PSrc q = sh.u.tile.src[j];
            float chi = 0.f, clo = 0.f;
#pragma unroll
            for (int r = 0; r < R; r++) {
                const float dx = (float)(tx[r] - q.x), dy = (float)(ty[r] - q.y), dz = (float)(tz[r] - q.z);
                const float kv_ = kv32<KIND>(dx * dx + dy * dy + dz * dz, A.prm);   // distinct cells: r > 0
                a[r] += kv_ * q.whi;
                a2[r] += kv_ * q.wlo;
                chi += kv_ * whi[r];
                clo += kv_ * wlo[r];
            }
            sh.u.tile.shi[j] = group_sum<TPG>(chi);   // every lane of the group holds the sum
            sh.u.tile.slo[j] = group_sum<TPG>(clo);
            if ((it & (CHUNK - 1)) == CHUNK - 1) fold();
        }
        fold();
        __syncthreads();
        for (int32_t j = t; j < ns; j += NT) {
            A.col_hi[sh.u.tile.sslot[j]] = sh.u.tile.shi[j];
            A.col_lo[sh.u.tile.sslot[j]] = sh.u.tile.slo[j];
        }
    }
    // row sums over the groups
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; r++) {
        sh.u.part[((g * TPG + ti) * R + r) * 2] = acc[r];
        sh.u.part[((g * TPG + ti) * R + r) * 2 + 1] = (double)a2[r];
    }
    __syncthreads();
    for (int32_t i = t; i < kk; i += NT) {
        const int32_t li = i % TPG, r = i / TPG;
        double s1 = 0.0, s2 = 0.0;
        for (int gg = 0; gg < G; gg++) {
            s1 += sh.u.part[((gg * TPG + li) * R + r) * 2];
            s2 += sh.u.part[((gg * TPG + li) * R + r) * 2 + 1];
        }
        A.row[po + i] = s1;
        A.row[n + po + i] = s2;
    }
}

// owner cells [c0, c0 + gridDim.x); targets per cell at most 4 * 32.  Five
// waves per SIMD (the register allocator otherwise settles at 102 VGPRs,
// four waves; with the hint it needs 80-86 and spills nothing).
template <int KIND>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(5))) void k_p2p_sym(int64_t c0, P2PSymArgs A)
{
    __shared__ P2PSymShared sh;
    const int64_t c = c0 + blockIdx.x;
    const int32_t kk = A.count[c];
    if (kk == 0) return;   // uniform for the workgroup
    if (kk <= 8) p2p_sym_cell<KIND, 2, 4>(A, sh, c, kk);
    else if (kk <= 16) p2p_sym_cell<KIND, 4, 4>(A, sh, c, kk);
    else if (kk <= 32) p2p_sym_cell<KIND, 8, 4>(A, sh, c, kk);
    else if (kk <= 64) p2p_sym_cell<KIND, 16, 4>(A, sh, c, kk);
    else p2p_sym_cell<KIND, 32, 4>(A, sh, c, kk);
}

// y (original order) = the near-field row sums of every point plus the slots
// of the pairs its neighbours own, added in list order (x_hi and x_lo parts
// apart, then together)
__global__ void k_p2p_gather(int64_t n, const int32_t *pcell, const int32_t *first, const int32_t *non_ptr,
                             const int32_t *non_slot, const float *col_hi, const float *col_lo, const double *row,
                             const int32_t *order, double *y)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t c = pcell[p], j = (int32_t)p - first[c];
    double s1 = row[p], s2 = row[n + p];
    for (int32_t e = non_ptr[c]; e < non_ptr[c + 1]; e++) {
        const int32_t sl = non_slot[e] + j;
        s1 += (double)col_hi[sl];
        s2 += (double)col_lo[sl];
    }
    y[order ? order[p] : p] = s1 + s2;
}

// the near field of leaf cells [c0, c1)
template <typename T>
void launch_p2p(int kind, nnca_h2 *H, const T *xw, const T *xw2, const double *far, double *y, T prm,
                hipStream_t s, int64_t c0 = 0, int64_t c1 = -1, bool tree_order = false)
{
    const int32_t *order = tree_order ? nullptr : H->order;
    const nnca::Level &L = H->lev[H->kappa];
    if (c1 < 0) c1 = L.ncell;
    const int64_t nc = c1 - c0;
    if (nc <= 0) return;
#define P2P_CASE(K) k_p2p<T, K><<<(int)nc, NT, 0, s>>>(c0, L.first, L.count, L.nb_ptr, L.nb, H->nbpre, H->nbsum, H->pts64, H->n, L.first, H->pts64, H->n, H->dim, xw, xw2, far, order, y, prm)
    if (kind == NNCA_K_INV_R) P2P_CASE(NNCA_K_INV_R);
    else if (kind == NNCA_K_LOG_R) P2P_CASE(NNCA_K_LOG_R);
    else if (kind == NNCA_K_LOG_REG) P2P_CASE(NNCA_K_LOG_REG);
    else if (kind == NNCA_K_INV_REG) P2P_CASE(NNCA_K_INV_REG);
    else if (kind == NNCA_K_EXP_R) P2P_CASE(NNCA_K_EXP_R);
    else if (kind == K_GAUSS_DH) P2P_CASE(K_GAUSS_DH);
    else P2P_CASE(NNCA_K_GAUSS);
#undef P2P_CASE
    HIPCHECK(hipGetLastError());
}

// the symmetric near field of owner cells [c0, c1) (mixed matvec)
static void launch_p2p_sym(int kind, nnca_h2 *H, const float *xhi, const float *xlo, float prm, hipStream_t s,
                           int64_t c0, int64_t c1)
{
    const nnca::Level &F = H->lev[H->kappa];
    const int64_t nc = c1 - c0;
    if (nc <= 0) return;
    P2PSymArgs A{F.first, F.count, H->pown_ptr, H->pown_nb, H->pown_pre, H->pown_sum, H->pown_slot, H->pts64,
                 H->n, H->dim, xhi, xlo, H->pcol_hi, H->pcol_lo, H->prow, prm};
#define PS_CASE(K) k_p2p_sym<K><<<(int)nc, NT, 0, s>>>(c0, A)
    if (kind == NNCA_K_INV_R) PS_CASE(NNCA_K_INV_R);
    else if (kind == NNCA_K_LOG_R) PS_CASE(NNCA_K_LOG_R);
    else if (kind == NNCA_K_LOG_REG) PS_CASE(NNCA_K_LOG_REG);
    else if (kind == NNCA_K_INV_REG) PS_CASE(NNCA_K_INV_REG);
    else if (kind == NNCA_K_EXP_R) PS_CASE(NNCA_K_EXP_R);
    else if (kind == K_GAUSS_DH) PS_CASE(K_GAUSS_DH);
    else PS_CASE(NNCA_K_GAUSS);
#undef PS_CASE
    HIPCHECK(hipGetLastError());
}


// One right-hand side.  xs64: x in tree order (FP64).  Mixed: x_hi, x_lo.
// The transfer passes run in FP64 for both precisions; the M2L and near-field
// kernels run in T with the kernel `kind` (the handle's, or the length-scale
// derivative of the Gaussian).  do_up = false reuses the multipole vectors
// already in the levels; do_p2p = false stops after the downward pass (the
// levels then hold every multipole vector and every local vector, the latter
// with all contributions of the coarser levels added).
template <typename T>
void one_column(nnca_h2 *H, const double *xs64, const T *xhi, const T *xlo, void *y, bool y32, hipStream_t s,
                int kind, bool do_up, bool do_p2p)
{
    const bool f32 = sizeof(T) == 4;
    const int kap = H->kappa, lmin = H->lmin;
    const T prm = f32 ? (T)kernel_prm32(kind, H->hparam) : (T)kernel_prm64(kind, H->hparam);
    double *far = nullptr;
    // With a far field, the near field runs on the handle's second stream
    // while the far-field passes run here (it reads only x and the points);
    // both write their sums in tree order, and after the join one kernel
    // forms y (original order) from them through the inverse permutation.  It runs in two parts of equal work, both
    // beside memory-bound passes: the first beside the upward pass, the
    // second after the leaf level's transverse kernel, beside its combine
    // step and the downward pass (the transverse kernels, bound by VALU
    // issue, then have the chip to themselves).
    const bool overlap = do_p2p && kap >= lmin;
    const int64_t ncl = H->lev[kap].ncell;
    const int64_t csplit = H->p2p_split > 0 && H->p2p_split <= ncl ? H->p2p_split : ncl / 2;
    // the mixed matvec evaluates each pair of neighbouring leaves once
    // (k_p2p_sym, then k_p2p_gather writes y)
    const bool psym = f32 && H->p2p_sym && !(H->apply_flags & NNCA_APPLY_NO_SYMMETRIC);
    auto near_part = [&](int64_t c0, int64_t c1) {
        Span sp(H, H->aux, PASS_P2P, kap);
        if (psym) launch_p2p_sym(kind, H, (const float *)xhi, (const float *)xlo, (float)prm, H->aux, c0, c1);
        else if (f32) launch_p2p<T>(kind, H, xhi, xlo, nullptr, H->near64, prm, H->aux, c0, c1, true);
        else launch_p2p<T>(kind, H, (const T *)xs64, nullptr, nullptr, H->near64, prm, H->aux, c0, c1, true);
    };
    auto near_gather = [&]() {
        Span sp(H, H->aux, PASS_P2P, kap);
        const nnca::Level &F = H->lev[kap];
        k_p2p_gather<<<grid_for(H->n, 256), 256, 0, H->aux>>>(H->n, H->pcell, F.first, H->pnon_ptr, H->pnon_slot,
                                                              H->pcol_hi, H->pcol_lo, H->prow, nullptr,
                                                              H->near64);
        HIPCHECK(hipGetLastError());
    };
    if (overlap) {
        HIPCHECK(hipEventRecord(H->ev_fork, s));
        HIPCHECK(hipStreamWaitEvent(H->aux, H->ev_fork, 0));
        if (psym) {   // half the work: all of it beside the upward pass and the coarse levels
            near_part(0, ncl);
            near_gather();
            HIPCHECK(hipEventRecord(H->ev_join, H->aux));
        } else {
            near_part(0, csplit);
        }
    }
    if (kap >= lmin) {
        // upward pass
        for (int l = kap; l >= lmin && do_up; l--) {
            nnca::Level &L = H->lev[l];
            const double *src = (l == kap) ? xs64 : H->lev[l + 1].w64;
            Span sp(H, s, PASS_UP, l);
            // one thread per output entry where cells have few non-pivot
            // rows (the leaf level: at most the leaf size, most leaves full
            // rank); a workgroup per cell (column slices) above
            if (L.nrem == 0 || l == kap)
                k_up<<<grid_for(L.npiv, 256), 256, 0, s>>>(L.npiv, L.piv_cell, L.piv_ptr, L.tt_off, L.ipos,
                                                           L.rem_ptr, L.rem_pos, L.crem_off, L.crem64, src, L.w64);
            else {
                // few cells: 32 columns per workgroup; else a whole cell each
                const int32_t colw = L.ncell < 2048 ? 32 : INT32_MAX;
                const unsigned gy = L.ncell < 2048 ? (unsigned)((L.max_k + 31) / 32) : 1u;
                k_up_cell<<<dim3((unsigned)L.ncell, gy > 0 ? gy : 1u), 256, 0, s>>>(
                    L.piv_ptr, L.tt_off, L.ipos, L.rem_ptr, L.rem_pos, L.crem_off, L.crem64, src, L.w64, colw);
            }
            HIPCHECK(hipGetLastError());
        }
        // transverse pass; the mixed matvec keeps the coarse levels
        // (l <= kappa - fp32_levels) in refined FP64 arithmetic
        const double prm64 = kernel_prm64(kind, H->hparam);
        const int lf64 = kap - H->fp32_levels;
        for (int l = lmin; l <= kap; l++) {
            nnca::Level &L = H->lev[l];
            const bool sym = L.sym && !(H->apply_flags & NNCA_APPLY_NO_SYMMETRIC);
            hipEvent_t after = overlap && l == kap ? H->ev_leafk : nullptr;
            if (sym) {   // the launcher times its kernel and its combine step apart
                if (!f32) launch_m2l_sym<M_F64>(kind, H, L, l, prm64, s, after);
                else if (l <= lf64) launch_m2l_sym<M_F64R>(kind, H, L, l, prm64, s, after);
                else launch_m2l_sym<M_F32>(kind, H, L, l, (double)prm, s, after);
                continue;
            }
            Span sp(H, s, PASS_M2L, l);
            if (!f32) launch_m2l_mode<M_F64>(kind, H, L, L.pc64, prm64, s, after);
            else if (l <= lf64) launch_m2l_mode<M_F64R>(kind, H, L, L.pc64, prm64, s, after);
            else launch_m2l_mode<M_F32>(kind, H, L, L.pc32, (double)prm, s, after);
        }
        if (overlap && !psym) {
            HIPCHECK(hipStreamWaitEvent(H->aux, H->ev_leafk, 0));
            near_part(csplit, ncl);
            HIPCHECK(hipEventRecord(H->ev_join, H->aux));
        }
        // downward pass; the leaf level writes the far field in tree order
        far = H->far64;
        for (int l = lmin; l <= kap; l++) {
            nnca::Level &L = H->lev[l];
            const bool leaf = l == kap;
            double *out = leaf ? far : H->lev[l + 1].u64;
            Span sp(H, s, PASS_DOWN, l);
            k_down<<<grid_for(L.npiv + L.nrem, 256), 256, 0, s>>>(
                L.npiv, L.nrem, L.piv_cell, L.rem_cell, L.piv_ptr, L.tt_off, L.ipos, L.rem_ptr, L.rem_pos,
                L.crem_off, L.crem_t, L.u64, out, leaf ? 0 : 1, nullptr);
            HIPCHECK(hipGetLastError());
        }
        if (overlap) {
            HIPCHECK(hipStreamWaitEvent(s, H->ev_join, 0));
            Span sp(H, s, PASS_DOWN, kap);
            if (y32)
                k_near_far_out<<<grid_for(H->n, 256), 256, 0, s>>>(H->n, H->rank, H->near64, far, (float *)y);
            else
                k_near_far_out<<<grid_for(H->n, 256), 256, 0, s>>>(H->n, H->rank, H->near64, far, (double *)y);
            HIPCHECK(hipGetLastError());
        }
    }
    if (!do_p2p || overlap) return;
    // near field alone (no far field): in tree order, then y
    Span sp(H, s, PASS_P2P, kap);
    if (f32) launch_p2p<T>(kind, H, xhi, xlo, nullptr, H->near64, prm, s, 0, -1, true);
    else launch_p2p<T>(kind, H, (const T *)xs64, nullptr, nullptr, H->near64, prm, s, 0, -1, true);
    if (y32)
        k_near_far_out<<<grid_for(H->n, 256), 256, 0, s>>>(H->n, H->rank, H->near64, nullptr, (float *)y);
    else
        k_near_far_out<<<grid_for(H->n, 256), 256, 0, s>>>(H->n, H->rank, H->near64, nullptr, (double *)y);
    HIPCHECK(hipGetLastError());
}

}  // namespace

template <typename TI>
static void gather_typed(nnca_h2 *H, const TI *x, int precision, hipStream_t s)
{
    const int64_t n = H->n;
    Span sp(H, s, PASS_GATHER, -1);
    if (precision == NNCA_PREC_MIXED)
        k_gather_split<TI><<<grid_for(n, 256), 256, 0, s>>>(n, H->order, x, H->xs64, H->xhi, H->xlo);
    else
        k_gather64<TI><<<grid_for(n, 256), 256, 0, s>>>(n, H->order, x, H->xs64);
    HIPCHECK(hipGetLastError());
}

void gather_input(nnca_h2 *H, const double *x, int precision, hipStream_t s) { gather_typed(H, x, precision, s); }

static void column_passes_io(nnca_h2 *H, int precision, int kind, bool do_up, bool do_p2p, void *y, bool y32,
                             hipStream_t s)
{
    if (precision == NNCA_PREC_MIXED)
        one_column<float>(H, H->xs64, H->xhi, H->xlo, y, y32, s, kind, do_up, do_p2p);
    else one_column<double>(H, H->xs64, nullptr, nullptr, y, y32, s, kind, do_up, do_p2p);
}

void column_passes(nnca_h2 *H, int precision, int kind, bool do_up, bool do_p2p, double *y, hipStream_t s)
{
    column_passes_io(H, precision, kind, do_up, do_p2p, y, false, s);
}

// Ownership of the interacting pairs of a level for the symmetric transverse
// pass: the pair {B, B'} belongs to the smaller index when B + B' is even and
// to the larger one otherwise (about half of every list each); pairs with an
// empty cell carry nothing and are left out.  Levels whose ranks exceed
// SYM_MAXK or whose slot count exceeds 32-bit offsets keep the plain pass.
// The column slots are one FP64 buffer: the FP64 and FP64-refined forms use
// it as FP64 slots, the FP32 form (levels of the mixed matvec that run in
// FP32) as FP32 slots.
// Launch order of a level's cells.  Workgroups are dispatched to the eight
// XCDs round robin (workgroup b to XCD b mod 8), each with its own L2: XCD x
// gets the x-th of eight runs of the cells in tree (Morton) order holding
// equal work, so the sources it reads come from one compact region (about an
// eighth of the level's pivot data); inside a run the cells go largest work
// first, so the last wave of the launch holds the shortest workgroups.
// Cells without work follow, dealt to the runs round robin (in a general
// product the target cells outside the source set's region are many and
// contiguous in tree order: in one run they would lengthen the grid by their
// count of empty slots; 8.9 against 7.3 ms for the transposed product of
// 2^19 shifted targets and 2^20 sources).  Runs are padded to equal length
// with empty slots (-1) and appended to `ord`; returns the run length (0 when
// no cell has in[c] set).
static int64_t xcd_runs(const std::vector<int64_t> &wk, const std::vector<char> &in, std::vector<int32_t> &ord)
{
    const int64_t nc = (int64_t)wk.size();
    int64_t wtot = 0, cnt = 0;
    for (int64_t c = 0; c < nc; c++)
        if (in[c] && wk[c] > 0) {
            wtot += wk[c];
            cnt++;
        }
    std::vector<std::vector<int32_t>> ch(8);
    int64_t cum = 0;
    for (int64_t c = 0; c < nc; c++) {
        if (!in[c] || wk[c] == 0) continue;
        int x = (int)((cum * 8) / wtot);
        if (x > 7) x = 7;
        ch[x].push_back((int32_t)c);
        cum += wk[c];
    }
    for (auto &v : ch) std::stable_sort(v.begin(), v.end(), [&](int32_t a, int32_t b) { return wk[a] > wk[b]; });
    // cells without work (rows to clear only) go last, dealt round robin,
    // so that they do not lengthen one run (and the grid) by themselves
    int64_t z = 0;
    for (int64_t c = 0; c < nc; c++)
        if (in[c] && wk[c] == 0) ch[(z++) % 8].push_back((int32_t)c);
    if (cnt + z == 0) return 0;
    size_t ms = 1;
    for (auto &v : ch) ms = std::max(ms, v.size());
    const size_t base = ord.size();
    ord.resize(base + 8 * ms, -1);
    for (int x = 0; x < 8; x++)
        for (size_t i = 0; i < ch[x].size(); i++) ord[base + x * ms + i] = ch[x][i];
    return (int64_t)ms;
}

// the plain transverse pass's order: work = rank x sources of the list
static void plain_order(Level &L, const std::vector<int32_t> &ils)
{
    const int64_t nc = L.ncell;
    std::vector<int64_t> wk(nc);
    std::vector<char> in(nc);
    for (int64_t c = 0; c < nc; c++) {
        wk[c] = (int64_t)L.h_k[c] * ils[c];
        in[c] = 1;   // every cell keeps its slot (its rows are written even without sources)
    }
    std::vector<int32_t> ord;
    L.m2l_slots = xcd_runs(wk, in, ord);
    if (ord.empty()) ord.push_back(-1);
    L.m2l_order = dalloc<int32_t>(ord.size());
    HIPCHECK(hipMemcpy(L.m2l_order, ord.data(), sizeof(int32_t) * ord.size(), hipMemcpyHostToDevice));
}

void prepare_symmetric(nnca_h2 *H, Level &L, bool)
{
    if (L.sym || L.ncell < 1 || L.max_k > SYM_MAXK) return;
    const int64_t nc = L.ncell;
    std::vector<int32_t> ilp(nc + 1), il(L.nil > 0 ? L.nil : 1);
    HIPCHECK(hipMemcpy(ilp.data(), L.il_ptr, sizeof(int32_t) * (nc + 1), hipMemcpyDeviceToHost));
    if (L.nil) HIPCHECK(hipMemcpy(il.data(), L.il, sizeof(int32_t) * L.nil, hipMemcpyDeviceToHost));
    const std::vector<int32_t> &kh = L.h_k;
    if ((int64_t)kh.size() != nc) fail(NNCA_ERR_INTERNAL, "host ranks missing for the symmetric pass");
    auto owned = [](int64_t a, int64_t b) { return ((a + b) & 1) ? a > b : a < b; };
    std::vector<int32_t> optr(nc + 1, 0), oil, opre, osum(nc, 0), oslot, nptr(nc + 1, 0), nslot;
    std::vector<int64_t> slot_of(L.nil > 0 ? L.nil : 1, -1);
    int64_t col = 0;
    int32_t max_own = 0;
    for (int64_t c = 0; c < nc; c++) {
        int64_t pre = 0;
        for (int32_t e = ilp[c]; e < ilp[c + 1]; e++) {
            const int32_t b = il[e];
            if (kh[c] == 0 || kh[b] == 0 || !owned(c, b)) continue;
            oil.push_back(b);
            opre.push_back((int32_t)pre);
            oslot.push_back((int32_t)std::max<int64_t>(INT32_MIN, std::min<int64_t>(INT32_MAX, col - pre)));
            slot_of[e] = col;
            pre += kh[b];
            col += kh[b];
        }
        osum[c] = (int32_t)pre;
        max_own = std::max<int32_t>(max_own, (int32_t)pre);
        optr[c + 1] = (int32_t)oil.size();
    }
    if (col >= INT32_MAX) return;
    for (int64_t c = 0; c < nc; c++) {
        for (int32_t e = ilp[c]; e < ilp[c + 1]; e++) {
            const int32_t b = il[e];
            if (kh[c] == 0 || kh[b] == 0 || owned(c, b)) continue;
            auto beg = il.begin() + ilp[b], end = il.begin() + ilp[b + 1];
            auto it = std::lower_bound(beg, end, (int32_t)c);
            if (it == end || *it != c) fail(NNCA_ERR_INTERNAL, "interaction lists are not symmetric");
            nslot.push_back((int32_t)slot_of[it - il.begin()]);
        }
        nptr[c + 1] = (int32_t)nslot.size();
    }
    auto up = [&](const std::vector<int32_t> &v) {
        int32_t *d = dalloc<int32_t>(v.size());
        if (!v.empty()) HIPCHECK(hipMemcpy(d, v.data(), sizeof(int32_t) * v.size(), hipMemcpyHostToDevice));
        return d;
    };
    L.own_ptr = up(optr);
    L.own_il = up(oil);
    L.own_pre = up(opre);
    L.own_sum = up(osum);
    L.own_slot = up(oslot);
    L.non_ptr = up(nptr);
    L.non_slot = up(nslot);
    // launch order (xcd_runs).  c2 per launch: leaf 0.79 ms, level kappa-1
    // 0.74 ms; 0.87 and 0.80 in plain cell order; 0.81 and 0.75 with the
    // largest-first order over the whole level; 0.83 and 0.75 with the runs
    // in tree order.
    //
    // Rank classes.  A launch's shape set follows the largest rank it
    // holds, and the sets for ranks above 80 take more registers per lane
    // (fewer waves per SIMD).  Where cells of rank above 80 are at most a
    // quarter of the level, they get a launch of their own and the others
    // run with the set for ranks <= 80: level 7 of the 80^3 Chebyshev grid
    // (343 000 cells, mean rank 1.5, largest 88) 7.3 -> about 1.6 ms in the
    // FP32 form; splitting level kappa-1 of the 2^20 cube (most of its 4096
    // cells above 80) made it slower, 0.76 against 0.73 ms.  Cells of rank 0
    // own no pairs and get no slot.
    int64_t nhi = 0;
    for (int64_t c = 0; c < nc; c++) nhi += kh[c] > 80;
    const bool split = L.max_k > 80 && nhi > 0 && 4 * nhi <= nc;
    std::vector<int64_t> wk(nc);
    std::vector<char> in0(nc), in1(nc);
    for (int64_t c = 0; c < nc; c++) {
        wk[c] = (int64_t)kh[c] * osum[c];
        in0[c] = kh[c] > 0 && (!split || kh[c] <= 80);
        in1[c] = kh[c] > 80 && split;
    }
    std::vector<int32_t> ord;
    L.sym_slots = xcd_runs(wk, in0, ord);
    L.sym_slots_hi = split ? xcd_runs(wk, in1, ord) : 0;
    if (ord.empty()) ord.push_back(-1);
    L.sym_order = up(ord);
    L.col64 = dalloc<double>(col);
    L.col32 = reinterpret_cast<float *>(L.col64);
    L.ncol = col;
    L.max_own = max_own;
    L.sym = true;
}

// Lists and buffers of the symmetric near field (see k_p2p_sym); off when a
// leaf holds more than 128 points or owns more than PS_ME - 1 neighbours.
static void prepare_p2p_sym(nnca_h2 *H, const std::vector<int32_t> &hc)
{
    Level &F = H->lev[H->kappa];
    const int64_t nc = F.ncell, n = H->n;
    if (nc < 1 || H->max_leaf > 4 * 32 || F.nnb < 1) return;
    std::vector<int32_t> np(nc + 1), nbl(F.nnb), fi(nc);
    HIPCHECK(hipMemcpy(np.data(), F.nb_ptr, sizeof(int32_t) * (nc + 1), hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(nbl.data(), F.nb, sizeof(int32_t) * F.nnb, hipMemcpyDeviceToHost));
    HIPCHECK(hipMemcpy(fi.data(), F.first, sizeof(int32_t) * nc, hipMemcpyDeviceToHost));
    auto owned = [](int64_t a, int64_t b) { return ((a + b) & 1) ? a > b : a < b; };
    std::vector<int32_t> optr(nc + 1, 0), onb, opre, osum(nc, 0), oslot, nptr(nc + 1, 0), nslot;
    std::vector<int64_t> slot_of(F.nnb, -1);
    int64_t col = 0;
    for (int64_t c = 0; c < nc; c++) {
        int64_t pre = 0;
        for (int32_t e = np[c]; e < np[c + 1]; e++) {
            const int32_t b = nbl[e];
            if (b == c || !owned(c, b)) continue;
            onb.push_back(b);
            opre.push_back((int32_t)pre);
            oslot.push_back((int32_t)std::max<int64_t>(INT32_MIN, std::min<int64_t>(INT32_MAX, col - pre)));
            slot_of[e] = col;
            pre += hc[b];
            col += hc[b];
        }
        osum[c] = (int32_t)pre;
        optr[c + 1] = (int32_t)onb.size();
        if (optr[c + 1] - optr[c] > PS_ME - 1) return;
    }
    if (col >= INT32_MAX) return;
    for (int64_t c = 0; c < nc; c++) {
        for (int32_t e = np[c]; e < np[c + 1]; e++) {
            const int32_t b = nbl[e];
            if (b == c || owned(c, b)) continue;
            auto beg = nbl.begin() + np[b], end = nbl.begin() + np[b + 1];
            auto it = std::lower_bound(beg, end, (int32_t)c);
            if (it == end || *it != c) fail(NNCA_ERR_INTERNAL, "neighbour lists are not symmetric");
            nslot.push_back((int32_t)slot_of[it - nbl.begin()]);
        }
        nptr[c + 1] = (int32_t)nslot.size();
    }
    std::vector<int32_t> pc(n);
    for (int64_t c = 0; c < nc; c++)
        for (int32_t p = fi[c]; p < fi[c] + hc[c]; p++) pc[p] = (int32_t)c;
    auto up = [&](const std::vector<int32_t> &v) {
        int32_t *dv = dalloc<int32_t>(v.size());
        if (!v.empty()) HIPCHECK(hipMemcpy(dv, v.data(), sizeof(int32_t) * v.size(), hipMemcpyHostToDevice));
        return dv;
    };
    H->pown_ptr = up(optr);
    H->pown_nb = up(onb);
    H->pown_pre = up(opre);
    H->pown_sum = up(osum);
    H->pown_slot = up(oslot);
    H->pnon_ptr = up(nptr);
    H->pnon_slot = up(nslot);
    H->pcell = up(pc);
    H->pcol_n = col > 0 ? col : 1;
    H->pcol_hi = dalloc<float>(H->pcol_n);
    H->pcol_lo = dalloc<float>(H->pcol_n);
    H->prow = dalloc<double>(2 * n);
    H->p2p_sym = true;
}

// tree-order near-field buffer and the inverse permutation of the points
// (order is a permutation of [0, n))
void prepare_output(nnca_h2 *H, hipStream_t s)
{
    H->near64 = dalloc<double>(H->n);
    H->rank = dalloc<int32_t>(H->n);
    k_invert_order<<<grid_for(H->n, 256), 256, 0, s>>>(H->n, H->order, H->rank);
    HIPCHECK(hipGetLastError());
}

void prepare_apply(nnca_h2 *H)
{
    hipStream_t s = H->stream;
    const int d = H->dim;
    int64_t m2l = 0, trans = 0;
    for (int l = H->lmin; l <= H->kappa; l++) {
        Level &L = H->lev[l];
        int64_t nc = L.ncell;
        L.pc64 = dalloc<double>(3 * L.npiv);
        L.pc32 = dalloc<float>(3 * L.npiv);
        k_pivot_coords<<<(int)nc, 64, 0, s>>>(nc, L.piv_ptr, L.piv_id, H->pts64, H->n, d, L.coord, H->lo[0], H->lo[1],
                                              H->lo[2], L.h, L.npiv, L.pc64, L.pc32);
        int32_t nrem = 0;
        HIPCHECK(hipMemcpy(&nrem, L.rem_ptr + nc, sizeof(int32_t), hipMemcpyDeviceToHost));
        L.nrem = nrem;
        L.piv_cell = dalloc<int32_t>(L.npiv);
        L.rem_cell = dalloc<int32_t>(L.nrem);
        k_fill_owner<<<grid_for(nc, 256), 256, 0, s>>>(nc, L.piv_ptr, L.piv_cell);
        k_fill_owner<<<grid_for(nc, 256), 256, 0, s>>>(nc, L.rem_ptr, L.rem_cell);
        L.crem_t = dalloc<double>(L.ncrem);
        if (L.ncrem) k_transpose_blocks<<<(int)nc, 256, 0, s>>>(nc, L.piv_ptr, L.rem_ptr, L.crem_off, L.crem64, L.crem_t);
        L.ilpre = dalloc<int32_t>(L.nil);
        L.ilsum = dalloc<int32_t>(nc);
        k_list_prefix<<<grid_for(nc, 256), 256, 0, s>>>(nc, L.il_ptr, L.il, L.k, L.ilpre, L.ilsum);
        L.w64 = dalloc<double>(L.npiv);
        L.u64 = dalloc<double>(L.npiv);
        HIPCHECK(hipGetLastError());
        std::vector<int32_t> ils(nc);
        HIPCHECK(hipMemcpyAsync(ils.data(), L.ilsum, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        L.max_ilsum = 0;
        L.m2l_inter = 0;
        for (int64_t c = 0; c < nc; c++) {
            L.m2l_inter += (int64_t)L.h_k[c] * ils[c];
            L.max_ilsum = std::max(L.max_ilsum, ils[c]);
        }
        plain_order(L, ils);
        m2l += L.m2l_inter;
        trans += L.ncrem;
    }
    Level &F = H->lev[H->kappa];
    int64_t nc = F.ncell;
    int32_t *cnt = F.count;
    H->nbpre = dalloc<int32_t>(F.nnb);
    H->nbsum = dalloc<int32_t>(nc);
    k_list_prefix<<<grid_for(nc, 256), 256, 0, s>>>(nc, F.nb_ptr, F.nb, cnt, H->nbpre, H->nbsum);
    HIPCHECK(hipGetLastError());
    std::vector<int32_t> nbs(nc), hc(nc);
    HIPCHECK(hipMemcpyAsync(nbs.data(), H->nbsum, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(hc.data(), F.count, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    int64_t p2p = 0;
    H->max_leaf = 0;
    for (int64_t c = 0; c < nc; c++) {
        p2p += (int64_t)hc[c] * nbs[c];
        H->max_leaf = std::max(H->max_leaf, hc[c]);
    }
    // the near field runs in two parts of equal work (see one_column)
    H->p2p_split = nc;
    for (int64_t c = 0, acc = 0; c < nc; c++) {
        acc += (int64_t)hc[c] * nbs[c];
        if (2 * acc >= p2p) {
            H->p2p_split = c + 1;
            break;
        }
    }
    // The symmetric near field halves its arithmetic but ends in a gather; it
    // pays where the near field is a large share of the work (measured: the
    // Gaussian mixture of 200 000 points, near pairs 10.3% of the transverse
    // interactions, 6.23 against 6.34 ms per forward + backward step), not
    // where the two-part plain near field hides beside the memory-bound
    // passes (1/r at 2^20 points, 6.9%: 3.10 against 3.12-3.16 ms per matvec).
    if (p2p * 12 > m2l) prepare_p2p_sym(H, hc);
    // the mixed matvec runs the finest levels in the FP32 form, the coarser
    // ones in the FP64-refined form
    H->fp32_levels = mixed_fp32_levels(H->kind);
    for (int l = H->lmin; l <= H->kappa; l++)
        prepare_symmetric(H, H->lev[l], l <= H->kappa - H->fp32_levels);
    H->m2l_inter = m2l;
    H->p2p_inter = p2p;
    H->transfer_entries = trans;
    HIPCHECK(hipStreamCreateWithFlags(&H->aux, hipStreamNonBlocking));
    HIPCHECK(hipEventCreateWithFlags(&H->ev_fork, hipEventDisableTiming));
    HIPCHECK(hipEventCreateWithFlags(&H->ev_join, hipEventDisableTiming));
    HIPCHECK(hipEventCreateWithFlags(&H->ev_leafk, hipEventDisableTiming));
    H->xs64 = dalloc<double>(H->n);
    H->far64 = dalloc<double>(H->n);
    prepare_output(H, s);
    H->xhi = dalloc<float>(H->n);
    H->xlo = dalloc<float>(H->n);
    prepare_workspace(H);
}

// Levels of the mixed matvec whose transverse pass runs in FP32, counted
// from the leaves; the coarser ones run in refined FP64.  The nested
// interpolation operators amplify FP32 rounding injected at a level on its
// way down; measured against FP64 (three right-hand sides each): 1/r at 2^20
// points 3.8e-7 with two FP32 levels; the Gaussian mixture of 200 000 points
// 0.45-1.08e-6 with two, 0.14-0.38e-6 with one.  The 2D log kernel's
// operators have the largest entries.
int mixed_fp32_levels(int kind) { return kind == NNCA_K_INV_R || kind == NNCA_K_INV_REG ? 2 : 1; }

void run_matvec(nnca_h2 *H, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy, int dtype,
                int precision, hipStream_t s)
{
    // several columns: the many-column path where its workspace exists
    if (nrhs > 1 && H->multi.rp > 0) {
        run_matvec_multi(H, X, Y, nrhs, ldx, ldy, dtype, precision, s);
        return;
    }
    run_matvec_columns(H, X, Y, nrhs, ldx, ldy, dtype, precision, s);
}

void run_matvec_columns(nnca_h2 *H, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy, int dtype,
                        int precision, hipStream_t s)
{
    const bool f32 = dtype == NNCA_F32;
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    for (int64_t col = 0; col < nrhs; col++) {
        const char *x = (const char *)X + col * ldx * es;
        char *y = (char *)Y + col * ldy * es;
        if (f32) gather_typed(H, (const float *)x, precision, s);
        else gather_typed(H, (const double *)x, precision, s);
        column_passes_io(H, precision, H->kind, true, true, y, f32, s);
    }
}

void prepare_workspace(nnca_h2 *H)
{
    // partial vectors of the split one-column transverse launches: the larger
    // split of the plain and the symmetric pass on every level
    int64_t part = 0;
    for (int l = H->lmin; l <= H->kappa; l++) {
        const Level &L = H->lev[l];
        if (!L.has_piv) continue;
        const int P = std::max(m2l_parts(L), sym_parts(L));
        if (P > 1) part = std::max(part, (int64_t)P * L.npiv);
    }
    if (part > 0) {
        H->m2l_part = dalloc<double>(part);
        H->m2l_part_cap = part;
    }
    if (H->max_rhs > 1) alloc_multi(H, (std::min(H->max_rhs, 64) + 15) / 16 * 16);
}

void run_direct(const double *pts, int64_t n, int dim, int64_t ld, int kind, double hparam, const double *X,
                double *Y, int64_t nrhs, int64_t ldx, int64_t ldy, hipStream_t s)
{
    double prm = kernel_prm64(kind, hparam);
    for (int64_t col = 0; col < nrhs; col++) {
        const double *x = X + col * ldx;
        double *y = Y + col * ldy;
        int g = grid_for(n, NT);
        if (kind == NNCA_K_INV_R) k_direct<NNCA_K_INV_R><<<g, NT, 0, s>>>(pts, n, dim, ld, x, y, prm);
        else if (kind == NNCA_K_LOG_R) k_direct<NNCA_K_LOG_R><<<g, NT, 0, s>>>(pts, n, dim, ld, x, y, prm);
        else if (kind == NNCA_K_LOG_REG) k_direct<NNCA_K_LOG_REG><<<g, NT, 0, s>>>(pts, n, dim, ld, x, y, prm);
        else if (kind == NNCA_K_INV_REG) k_direct<NNCA_K_INV_REG><<<g, NT, 0, s>>>(pts, n, dim, ld, x, y, prm);
        else if (kind == NNCA_K_EXP_R) k_direct<NNCA_K_EXP_R><<<g, NT, 0, s>>>(pts, n, dim, ld, x, y, prm);
        else k_direct<NNCA_K_GAUSS><<<g, NT, 0, s>>>(pts, n, dim, ld, x, y, prm);
        HIPCHECK(hipGetLastError());
    }
}

// ---------------------------------------------------------------------------
// General case P != Q (Sec. 2.3, Sec. 4).  The product y = A~ x runs
//   upward     on the outgoing half (sources): w^{B,o} = V_B^T x^B at a leaf,
//              the stacked T_{B B_c} applied to the children's w above;
//   transverse targets t^{B,i} of the incoming half, sources s^{B',o} of
//              the outgoing half: u^{B,i} = sum_{IL} K(t^{B,i}, s^{B',o}) w^{B',o};
//   downward   on the incoming half: U_B / C_{B_c B} as in the symmetric case;
//   near field K(t^B, s^{B'}) x^{B'} over N(B), targets P, sources Q.
// The transposed product A~^T g runs the same kernels with the halves and
// the point sets exchanged: up with U_B^T and C_{B_c B}^T over P, across with
// K(t^{B',i}, s^{B,o})^T (the kernels are radial, so K(q, p) = K(p, q)), down
// with V_B and T_{B B_c}^T over Q, near field over the neighbours' targets.
// The transverse pass has no symmetric form here (its blocks are not
// shared between the two directions); the near field neither.

namespace {

// per-level apply data of one half: pivot coordinates in that half's point
// array, owners, transposed blocks, multipole and local vectors, and for
// every interaction list the prefix of the other half's ranks (its sources)
void prepare_half(nnca_h2 *H, std::vector<Level> &lv, const std::vector<Level> &other, const double *pts,
                  int64_t n, int64_t &m2l, int64_t &trans)
{
    hipStream_t s = H->stream;
    const int d = H->dim;
    m2l = 0;
    trans = 0;
    for (int l = H->lmin; l <= H->kappa; l++) {
        Level &L = lv[l];
        const Level &O = other[l];
        const int64_t nc = L.ncell;
        L.pc64 = dalloc<double>(3 * L.npiv);
        L.pc32 = dalloc<float>(3 * L.npiv);
        k_pivot_coords<<<(int)nc, 64, 0, s>>>(nc, L.piv_ptr, L.piv_id, pts, n, d, L.coord, H->lo[0], H->lo[1],
                                              H->lo[2], L.h, L.npiv, L.pc64, L.pc32);
        int32_t nrem = 0;
        HIPCHECK(hipMemcpy(&nrem, L.rem_ptr + nc, sizeof(int32_t), hipMemcpyDeviceToHost));
        L.nrem = nrem;
        L.piv_cell = dalloc<int32_t>(L.npiv);
        L.rem_cell = dalloc<int32_t>(L.nrem);
        k_fill_owner<<<grid_for(nc, 256), 256, 0, s>>>(nc, L.piv_ptr, L.piv_cell);
        k_fill_owner<<<grid_for(nc, 256), 256, 0, s>>>(nc, L.rem_ptr, L.rem_cell);
        L.crem_t = dalloc<double>(L.ncrem);
        if (L.ncrem) k_transpose_blocks<<<(int)nc, 256, 0, s>>>(nc, L.piv_ptr, L.rem_ptr, L.crem_off, L.crem64, L.crem_t);
        L.ilpre = dalloc<int32_t>(L.nil);
        L.ilsum = dalloc<int32_t>(nc);
        k_list_prefix<<<grid_for(nc, 256), 256, 0, s>>>(nc, L.il_ptr, L.il, O.k, L.ilpre, L.ilsum);
        L.w64 = dalloc<double>(L.npiv);
        L.u64 = dalloc<double>(L.npiv);
        HIPCHECK(hipGetLastError());
        std::vector<int32_t> ils(nc);
        HIPCHECK(hipMemcpyAsync(ils.data(), L.ilsum, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        L.max_ilsum = 0;
        L.m2l_inter = 0;
        for (int64_t c = 0; c < nc; c++) {
            L.m2l_inter += (int64_t)L.h_k[c] * ils[c];
            L.max_ilsum = std::max(L.max_ilsum, ils[c]);
        }
        plain_order(L, ils);
        m2l += L.m2l_inter;
        trans += L.ncrem;
    }
}

// one column of the general product (adj: the transposed product)
template <typename T>
void one_column_general(nnca_h2 *H, bool adj, const T *xhi, const T *xlo, void *y, bool y32, hipStream_t s)
{
    const bool f32 = sizeof(T) == 4;
    const int kind = H->kind, kap = H->kappa, lmin = H->lmin;
    std::vector<Level> &tl = adj ? H->lev_o : H->lev;   // targets' half: local vectors, downward pass
    std::vector<Level> &sl = adj ? H->lev : H->lev_o;   // sources' half: multipole vectors, upward pass
    const double *tpts = adj ? H->qpts64 : H->pts64, *spts = adj ? H->pts64 : H->qpts64;
    const int64_t nt = adj ? H->nq : H->n, ns = adj ? H->n : H->nq;
    const int32_t *trank = adj ? H->qrank : H->rank;
    const int32_t *nbpre = adj ? H->nbpre_o : H->nbpre, *nbsum = adj ? H->nbsum_o : H->nbsum;
    const T prm = f32 ? (T)kernel_prm32(kind, H->hparam) : (T)kernel_prm64(kind, H->hparam);
    const double prm64 = kernel_prm64(kind, H->hparam);
    const double *xs64 = H->xs64;
    double *far = nullptr;
    if (kap >= lmin) {
        for (int l = kap; l >= lmin; l--) {
            Level &L = sl[l];
            const double *src = (l == kap) ? xs64 : sl[l + 1].w64;
            Span sp(H, s, PASS_UP, l);
            if (L.nrem == 0 || l == kap)
                k_up<<<grid_for(L.npiv, 256), 256, 0, s>>>(L.npiv, L.piv_cell, L.piv_ptr, L.tt_off, L.ipos,
                                                           L.rem_ptr, L.rem_pos, L.crem_off, L.crem64, src, L.w64);
            else {
                const int32_t colw = L.ncell < 2048 ? 32 : INT32_MAX;
                const unsigned gy = L.ncell < 2048 ? (unsigned)((L.max_k + 31) / 32) : 1u;
                k_up_cell<<<dim3((unsigned)L.ncell, gy > 0 ? gy : 1u), 256, 0, s>>>(
                    L.piv_ptr, L.tt_off, L.ipos, L.rem_ptr, L.rem_pos, L.crem_off, L.crem64, src, L.w64, colw);
            }
            HIPCHECK(hipGetLastError());
        }
        const int lf64 = kap - H->fp32_levels;
        for (int l = lmin; l <= kap; l++) {
            Level &L = tl[l];
            const Level &S = sl[l];
            Span sp(H, s, PASS_M2L, l);
            if (!f32) launch_m2l_pair<M_F64>(kind, H, L, S, L.pc64, S.pc64, prm64, s);
            else if (l <= lf64) launch_m2l_pair<M_F64R>(kind, H, L, S, L.pc64, S.pc64, prm64, s);
            else launch_m2l_pair<M_F32>(kind, H, L, S, L.pc32, S.pc32, (double)prm, s);
        }
        far = H->far64;
        for (int l = lmin; l <= kap; l++) {
            Level &L = tl[l];
            const bool leaf = l == kap;
            double *out = leaf ? far : tl[l + 1].u64;
            Span sp(H, s, PASS_DOWN, l);
            k_down<<<grid_for(L.npiv + L.nrem, 256), 256, 0, s>>>(
                L.npiv, L.nrem, L.piv_cell, L.rem_cell, L.piv_ptr, L.tt_off, L.ipos, L.rem_ptr, L.rem_pos,
                L.crem_off, L.crem_t, L.u64, out, leaf ? 0 : 1, nullptr);
            HIPCHECK(hipGetLastError());
        }
    }
    // near field plus the far field, in the targets' tree order, then y
    Span sp(H, s, PASS_P2P, kap);
    const Level &F = tl[kap], &G = sl[kap];
    const T *xw = f32 ? xhi : (const T *)xs64;
    const T *xw2 = f32 ? xlo : nullptr;
#define P2PG_CASE(K) k_p2p<T, K><<<(int)F.ncell, NT, 0, s>>>(0, F.first, F.count, F.nb_ptr, F.nb, nbpre, nbsum, tpts, nt, G.first, spts, ns, H->dim, xw, xw2, far, nullptr, H->near64, prm)
    if (kind == NNCA_K_INV_R) P2PG_CASE(NNCA_K_INV_R);
    else if (kind == NNCA_K_LOG_R) P2PG_CASE(NNCA_K_LOG_R);
    else if (kind == NNCA_K_LOG_REG) P2PG_CASE(NNCA_K_LOG_REG);
    else if (kind == NNCA_K_INV_REG) P2PG_CASE(NNCA_K_INV_REG);
    else if (kind == NNCA_K_EXP_R) P2PG_CASE(NNCA_K_EXP_R);
    else P2PG_CASE(NNCA_K_GAUSS);
#undef P2PG_CASE
    HIPCHECK(hipGetLastError());
    if (y32) k_near_far_out<<<grid_for(nt, 256), 256, 0, s>>>(nt, trank, H->near64, nullptr, (float *)y);
    else k_near_far_out<<<grid_for(nt, 256), 256, 0, s>>>(nt, trank, H->near64, nullptr, (double *)y);
    HIPCHECK(hipGetLastError());
}

}  // namespace

void prepare_general(nnca_h2 *H)
{
    hipStream_t s = H->stream;
    int64_t m2l = 0, trans = 0, m2l_o = 0, trans_o = 0;
    prepare_half(H, H->lev, H->lev_o, H->pts64, H->n, m2l, trans);
    prepare_half(H, H->lev_o, H->lev, H->qpts64, H->nq, m2l_o, trans_o);
    // near field: targets P with the neighbours' Q points, and the other way
    const Level &F = H->lev[H->kappa], &G = H->lev_o[H->kappa];
    const int64_t nc = F.ncell;
    H->nbpre = dalloc<int32_t>(F.nnb);
    H->nbsum = dalloc<int32_t>(nc);
    H->nbpre_o = dalloc<int32_t>(F.nnb);
    H->nbsum_o = dalloc<int32_t>(nc);
    k_list_prefix<<<grid_for(nc, 256), 256, 0, s>>>(nc, F.nb_ptr, F.nb, G.count, H->nbpre, H->nbsum);
    k_list_prefix<<<grid_for(nc, 256), 256, 0, s>>>(nc, F.nb_ptr, F.nb, F.count, H->nbpre_o, H->nbsum_o);
    HIPCHECK(hipGetLastError());
    std::vector<int32_t> nbs(nc), hc(nc), hq(nc);
    HIPCHECK(hipMemcpyAsync(nbs.data(), H->nbsum, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(hc.data(), F.count, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(hq.data(), G.count, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    int64_t p2p = 0;
    H->max_leaf = 0;
    for (int64_t c = 0; c < nc; c++) {
        p2p += (int64_t)hc[c] * nbs[c];
        H->max_leaf = std::max(H->max_leaf, std::max(hc[c], hq[c]));
    }
    H->fp32_levels = mixed_fp32_levels(H->kind);
    H->m2l_inter = m2l;
    H->p2p_inter = p2p;
    H->transfer_entries = trans + trans_o;
    // per-call buffers, sized for the larger of the two sets
    H->io_cap = std::max(H->n, H->nq);
    H->xs64 = dalloc<double>(H->io_cap);
    H->far64 = dalloc<double>(H->io_cap);
    H->near64 = dalloc<double>(H->io_cap);
    H->xhi = dalloc<float>(H->io_cap);
    H->xlo = dalloc<float>(H->io_cap);
    H->rank = dalloc<int32_t>(H->n);
    H->qrank = dalloc<int32_t>(H->nq);
    k_invert_order<<<grid_for(H->n, 256), 256, 0, s>>>(H->n, H->order, H->rank);
    k_invert_order<<<grid_for(H->nq, 256), 256, 0, s>>>(H->nq, H->qorder, H->qrank);
    HIPCHECK(hipGetLastError());
    // split partial vectors of the transverse pass, for either direction
    int64_t part = 0;
    for (int l = H->lmin; l <= H->kappa; l++)
        for (const Level *L : {&H->lev[l], &H->lev_o[l]}) {
            const int P = m2l_parts(*L);
            if (P > 1) part = std::max(part, (int64_t)P * L->npiv);
        }
    if (part > 0) {
        H->m2l_part = dalloc<double>(part);
        H->m2l_part_cap = part;
    }
    HIPCHECK(hipStreamSynchronize(s));
}

void run_matvec_general(nnca_h2 *H, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy, int dtype,
                        int precision, bool adjoint, hipStream_t s)
{
    const bool f32 = dtype == NNCA_F32;
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    const int64_t ns = adjoint ? H->n : H->nq;
    const int32_t *sorder = adjoint ? H->order : H->qorder;
    const bool mixed = precision == NNCA_PREC_MIXED;
    for (int64_t col = 0; col < nrhs; col++) {
        const char *x = (const char *)X + col * ldx * es;
        char *y = (char *)Y + col * ldy * es;
        {
            Span sp(H, s, PASS_GATHER, -1);
            if (mixed && f32)
                k_gather_split<float><<<grid_for(ns, 256), 256, 0, s>>>(ns, sorder, (const float *)x, H->xs64, H->xhi, H->xlo);
            else if (mixed)
                k_gather_split<double><<<grid_for(ns, 256), 256, 0, s>>>(ns, sorder, (const double *)x, H->xs64, H->xhi, H->xlo);
            else if (f32)
                k_gather64<float><<<grid_for(ns, 256), 256, 0, s>>>(ns, sorder, (const float *)x, H->xs64);
            else
                k_gather64<double><<<grid_for(ns, 256), 256, 0, s>>>(ns, sorder, (const double *)x, H->xs64);
            HIPCHECK(hipGetLastError());
        }
        if (mixed) one_column_general<float>(H, adjoint, H->xhi, H->xlo, y, f32, s);
        else one_column_general<double>(H, adjoint, nullptr, nullptr, y, f32, s);
    }
}

}  // namespace nnca
