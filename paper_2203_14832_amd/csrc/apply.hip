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

namespace nnca {

namespace {

constexpr int NT = 256;
constexpr int CHUNK = 16;   // terms summed in the working precision before an FP64 fold

template <typename T> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };

// kernel values of the apply passes
template <int KIND>
__device__ inline float kv32(float d2, float prm)
{
    if (KIND == NNCA_K_INV_R) return __builtin_amdgcn_rsqf(d2);
    if (KIND == NNCA_K_LOG_R) return 0.5f * logf(d2);
    return __builtin_amdgcn_exp2f(-d2 * prm);  // prm = log2(e) / h^2
}
template <int KIND>
__device__ inline double kv64(double d2, double prm)
{
    if (KIND == NNCA_K_INV_R) return 1.0 / sqrt(d2);
    if (KIND == NNCA_K_LOG_R) return 0.5 * log(d2);
    return exp(-d2 * prm);  // prm = 1 / h^2
}
template <int KIND, typename T>
__device__ inline T kv(T d2, T prm)
{
    if constexpr (sizeof(T) == 4) return kv32<KIND>(d2, prm);
    else return kv64<KIND>(d2, prm);
}
// near field: 1/r and log r vanish at r = 0, the Gaussian is 1 there
template <int KIND, typename T>
__device__ inline T kv_self(T d2, T prm)
{
    T v = kv<KIND, T>(d2, prm);
    if (KIND == NNCA_K_GAUSS) return v;
    return d2 > T(0) ? v : T(0);
}

// ---------------------------------------------------------------------------
// input gather (original -> tree order) and split

__global__ void k_gather64(int64_t n, const int32_t *order, const double *x, double *xs)
{
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < n) xs[p] = x[order[p]];
}

__global__ void k_gather_split(int64_t n, const int32_t *order, const double *x, float *hi, float *lo)
{
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    double v = x[order[p]];
    float h = (float)v;
    hi[p] = h;
    lo[p] = (float)(v - (double)h);
}

// ---------------------------------------------------------------------------
// upward pass: w^{B,o} = C_B^T x~ with x~ = x^B at a leaf (P2M), else the
// children's w^{B_c,o} stacked (M2M).  One wavefront per cell.

template <typename T>
__global__ void k_up(int64_t nc, const int32_t *m, const int32_t *k, const int32_t *tt_off,
                     const int32_t *piv_ptr, const int32_t *ipos, const int32_t *rem_ptr,
                     const int32_t *rem_pos, const int64_t *crem_off, const T *crem, const T *xin, T *w)
{
    int64_t c = blockIdx.x;
    int lane = threadIdx.x;
    int32_t kk = k[c], to = tt_off[c], po = piv_ptr[c], ro = rem_ptr[c];
    int32_t nr = rem_ptr[c + 1] - ro;
    const T *C = crem + crem_off[c];
    for (int32_t q = lane; q < kk; q += 64) {
        double acc = (double)xin[to + ipos[po + q]];
        for (int32_t r = 0; r < nr; r++)
            acc += (double)(C[(int64_t)r * kk + q] * xin[to + rem_pos[ro + r]]);
        w[po + q] = (T)acc;
    }
}

// downward pass: the stacked C_B u^{B,i} added to the children's u (L2L) or
// written as the far field of the leaf's points (L2P).
template <typename T>
__global__ void k_down(int64_t nc, const int32_t *k, const int32_t *tt_off, const int32_t *piv_ptr,
                       const int32_t *ipos, const int32_t *rem_ptr, const int32_t *rem_pos,
                       const int64_t *crem_off, const T *crem, const T *u, T *out, int accumulate)
{
    int64_t c = blockIdx.x;
    int lane = threadIdx.x;
    int32_t kk = k[c], to = tt_off[c], po = piv_ptr[c], ro = rem_ptr[c];
    int32_t nr = rem_ptr[c + 1] - ro;
    const T *C = crem + crem_off[c];
    for (int32_t q = lane; q < kk; q += 64) {
        int32_t dst = to + ipos[po + q];
        out[dst] = accumulate ? out[dst] + u[po + q] : u[po + q];
    }
    for (int32_t r = lane; r < nr; r += 64) {
        const T *row = C + (int64_t)r * kk;
        double acc = 0.0;
        for (int32_t q = 0; q < kk; q++) acc += (double)(row[q] * u[po + q]);
        int32_t dst = to + rem_pos[ro + r];
        out[dst] = accumulate ? (T)((double)out[dst] + acc) : (T)acc;
    }
}

// ---------------------------------------------------------------------------
// Interaction kernels.  One workgroup per target cell; its targets are split
// into groups of `cnt` consecutive threads (G = 256 / cnt groups), each group
// taking every G-th source of a 256-wide LDS tile.

struct TargetSplit {
    int32_t cnt, G, ti, g;
    __device__ TargetSplit(int32_t total, int32_t base, int t)
    {
        cnt = total - base < NT ? total - base : NT;
        G = NT / cnt;
        ti = t % cnt;
        g = t / cnt;
    }
};

// transverse pass at one level: u^{B,i} = sum_{B' in IL(B)} K(t^{B,i}, t^{B',i}) w^{B',o}
template <typename T, int KIND>
__global__ __launch_bounds__(NT) void k_m2l(int64_t nc, const int32_t *k, const int32_t *piv_ptr,
                                            const int32_t *il_ptr, const int32_t *il, const int32_t *ilpre,
                                            const int32_t *ilsum, const T *pc, int64_t npiv,
                                            const int32_t *coord, T h, int d, const T *w, T *u, T prm)
{
    using T4 = typename V4<T>::type;
    __shared__ T4 src[NT];
    __shared__ double part[NT];
    const int t = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int32_t kk = k[c], po = piv_ptr[c], S = ilsum[c];
    const int32_t e0 = il_ptr[c], e1 = il_ptr[c + 1];
    const bool local = sizeof(T) == 4;
    int32_t cc[3] = {coord[c], coord[nc + c], d == 3 ? coord[2 * nc + c] : 0};
    for (int32_t tb = 0; tb < kk; tb += NT) {
        TargetSplit sp(kk, tb, t);
        const bool act = sp.g < sp.G;
        T tx = 0, ty = 0, tz = 0;
        if (act) {
            int32_t q = po + tb + sp.ti;
            tx = pc[q];
            ty = pc[npiv + q];
            tz = d == 3 ? pc[2 * npiv + q] : T(0);
        }
        double acc = 0;
        int32_t e = e0;
        for (int32_t s0 = 0; s0 < S; s0 += NT) {
            int32_t s = s0 + t;
            T4 v;
            v.x = 0; v.y = 0; v.z = 0; v.w = 0;
            if (s < S) {
                while (e + 1 < e1 && ilpre[e + 1] <= s) e++;
                int32_t b = il[e];
                int32_t idx = piv_ptr[b] + (s - ilpre[e]);
                v.x = pc[idx];
                v.y = pc[npiv + idx];
                v.z = d == 3 ? pc[2 * npiv + idx] : T(0);
                v.w = w[idx];
                if (local) {
                    v.x += (T)(coord[b] - cc[0]) * h;
                    v.y += (T)(coord[nc + b] - cc[1]) * h;
                    if (d == 3) v.z += (T)(coord[2 * nc + b] - cc[2]) * h;
                }
            }
            __syncthreads();
            src[t] = v;
            __syncthreads();
            int32_t ns = S - s0 < NT ? S - s0 : NT;
            if (act) {
                // short sums in T, folded into the FP64 accumulator every CHUNK terms
                for (int32_t j = sp.g; j < ns;) {
                    int32_t je = j + CHUNK * sp.G < ns ? j + CHUNK * sp.G : ns;
                    T a = 0;
#pragma unroll 4
                    for (; j < je; j += sp.G) {
                        T4 q = src[j];
                        T dx = tx - q.x, dy = ty - q.y, dz = tz - q.z;
                        T d2 = dx * dx + dy * dy + dz * dz;
                        a += kv<KIND, T>(d2, prm) * q.w;
                    }
                    acc += (double)a;
                }
            }
        }
        __syncthreads();
        part[t] = acc;
        __syncthreads();
        if (t < sp.cnt) {
            double sum = part[t];
            for (int gg = 1; gg < sp.G; gg++) sum += part[gg * sp.cnt + t];
            u[po + tb + t] = (T)sum;
        }
        __syncthreads();
    }
}

// near field of one leaf plus the combine: y = far + sum_{B' in N(B)} K x.
// Mixed: weights x_hi and x_lo, results added in FP64.
template <typename T, int KIND>
__global__ __launch_bounds__(NT) void k_p2p(int64_t nc, const int32_t *first, const int32_t *count,
                                            const int32_t *nb_ptr, const int32_t *nb, const int32_t *nbpre,
                                            const int32_t *nbsum, const T *pts, int64_t n, const int32_t *coord,
                                            T h, int d, const T *xw, const T *xw2, const T *far,
                                            const int32_t *order, double *y, T prm)
{
    using T4 = typename V4<T>::type;
    __shared__ T4 src[NT];
    __shared__ T src2[NT];
    __shared__ double part[NT], part2[NT];
    const int t = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int32_t kk = count[c], po = first[c], S = nbsum[c];
    const int32_t e0 = nb_ptr[c], e1 = nb_ptr[c + 1];
    const bool mixed = sizeof(T) == 4;
    int32_t cc[3] = {coord[c], coord[nc + c], d == 3 ? coord[2 * nc + c] : 0};
    for (int32_t tb = 0; tb < kk; tb += NT) {
        TargetSplit sp(kk, tb, t);
        const bool act = sp.g < sp.G;
        T tx = 0, ty = 0, tz = 0;
        if (act) {
            int32_t q = po + tb + sp.ti;
            tx = pts[q];
            ty = pts[n + q];
            tz = d == 3 ? pts[2 * n + q] : T(0);
        }
        double acc = 0, acc2 = 0;
        int32_t e = e0;
        for (int32_t s0 = 0; s0 < S; s0 += NT) {
            int32_t s = s0 + t;
            T4 v;
            v.x = 0; v.y = 0; v.z = 0; v.w = 0;
            T v2 = 0;
            if (s < S) {
                while (e + 1 < e1 && nbpre[e + 1] <= s) e++;
                int32_t b = nb[e];
                int32_t idx = first[b] + (s - nbpre[e]);
                v.x = pts[idx];
                v.y = pts[n + idx];
                v.z = d == 3 ? pts[2 * n + idx] : T(0);
                v.w = xw[idx];
                if (mixed) {
                    v2 = xw2[idx];
                    v.x += (T)(coord[b] - cc[0]) * h;
                    v.y += (T)(coord[nc + b] - cc[1]) * h;
                    if (d == 3) v.z += (T)(coord[2 * nc + b] - cc[2]) * h;
                }
            }
            __syncthreads();
            src[t] = v;
            src2[t] = v2;
            __syncthreads();
            int32_t ns = S - s0 < NT ? S - s0 : NT;
            if (act) {
                for (int32_t j = sp.g; j < ns;) {
                    int32_t je = j + CHUNK * sp.G < ns ? j + CHUNK * sp.G : ns;
                    T a = 0, a2 = 0;
#pragma unroll 4
                    for (; j < je; j += sp.G) {
                        T4 q = src[j];
                        T dx = tx - q.x, dy = ty - q.y, dz = tz - q.z;
                        T d2 = dx * dx + dy * dy + dz * dz;
                        T kvv = kv_self<KIND, T>(d2, prm);
                        a += kvv * q.w;
                        if (mixed) a2 += kvv * src2[j];
                    }
                    acc += (double)a;
                    acc2 += (double)a2;
                }
            }
        }
        __syncthreads();
        part[t] = acc;
        part2[t] = acc2;
        __syncthreads();
        if (t < sp.cnt) {
            double s1 = part[t], s2 = part2[t];
            for (int gg = 1; gg < sp.G; gg++) {
                s1 += part[gg * sp.cnt + t];
                s2 += part2[gg * sp.cnt + t];
            }
            int32_t p = po + tb + t;
            double f = far ? (double)far[p] : 0.0;
            y[order[p]] = mixed ? (f + s1) + s2 : f + s1;
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

__global__ void k_diff(int64_t nc, const int32_t *ptr, int32_t *out)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c < nc) out[c] = ptr[c + 1] - ptr[c];
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

__global__ void k_point_local(int64_t nc, const int32_t *first, const int32_t *count, const double *P, int64_t n,
                              int d, const int32_t *coord, double lo0, double lo1, double lo2, double h, float *out)
{
    int64_t c = blockIdx.x;
    double lo[3] = {lo0, lo1, lo2};
    for (int32_t q = first[c] + threadIdx.x; q < first[c] + count[c]; q += blockDim.x)
        for (int a = 0; a < 3; a++) {
            double ctr = a < d ? lo[a] + ((double)coord[a * nc + c] + 0.5) * h : 0.0;
            out[a * n + q] = a < d ? (float)(P[a * n + q] - ctr) : 0.0f;
        }
}

__global__ void k_to_f32(int64_t n, const double *a, float *b)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

template <typename T>
void launch_m2l(int kind, const nnca::Level &L, const T *pc, int d, const T *w, T *u, T prm, hipStream_t s)
{
    int64_t nc = L.ncell;
    T h = (T)L.h;
#define M2L_CASE(K) k_m2l<T, K><<<(int)nc, NT, 0, s>>>(nc, L.k, L.piv_ptr, L.il_ptr, L.il, L.ilpre, L.ilsum, pc, L.npiv, L.coord, h, d, w, u, prm)
    if (kind == NNCA_K_INV_R) M2L_CASE(NNCA_K_INV_R);
    else if (kind == NNCA_K_LOG_R) M2L_CASE(NNCA_K_LOG_R);
    else M2L_CASE(NNCA_K_GAUSS);
#undef M2L_CASE
    HIPCHECK(hipGetLastError());
}

template <typename T>
void launch_p2p(int kind, nnca_h2 *H, const T *pts, const T *xw, const T *xw2, const T *far, double *y, T prm,
                hipStream_t s)
{
    const nnca::Level &L = H->lev[H->kappa];
    int64_t nc = L.ncell;
    T h = (T)L.h;
#define P2P_CASE(K) k_p2p<T, K><<<(int)nc, NT, 0, s>>>(nc, L.first, L.count, L.nb_ptr, L.nb, H->nbpre, H->nbsum, pts, H->n, L.coord, h, H->dim, xw, xw2, far, H->order, y, prm)
    if (kind == NNCA_K_INV_R) P2P_CASE(NNCA_K_INV_R);
    else if (kind == NNCA_K_LOG_R) P2P_CASE(NNCA_K_LOG_R);
    else P2P_CASE(NNCA_K_GAUSS);
#undef P2P_CASE
    HIPCHECK(hipGetLastError());
}

// event pair around one launch when the handle is profiling
struct Span {
    nnca_h2 *H;
    hipStream_t s;
    bool on;
    nnca_h2::ProfRec r;
    Span(nnca_h2 *H_, hipStream_t s_, int pass, int level) : H(H_), s(s_), on(H_->profiling)
    {
        if (!on) return;
        r.pass = pass;
        r.level = level;
        HIPCHECK(hipEventCreate(&r.a));
        HIPCHECK(hipEventCreate(&r.b));
        HIPCHECK(hipEventRecord(r.a, s));
    }
    ~Span() noexcept(false)
    {
        if (!on) return;
        HIPCHECK(hipEventRecord(r.b, s));
        H->prof.push_back(r);
    }
};

template <typename T>
void one_column(nnca_h2 *H, const T *xin, const T *xin2, double *y, hipStream_t s)
{
    const bool f32 = sizeof(T) == 4;
    const int kap = H->kappa, lmin = H->lmin;
    const T prm = H->kind == NNCA_K_GAUSS ? (f32 ? (T)(1.4426950408889634 / (H->hparam * H->hparam))
                                                 : (T)(1.0 / (H->hparam * H->hparam)))
                                          : T(0);
    T *far = nullptr;
    if (kap >= lmin) {
        // upward pass
        for (int l = kap; l >= lmin; l--) {
            nnca::Level &L = H->lev[l];
            const T *src = (l == kap) ? xin : (f32 ? (const T *)H->lev[l + 1].w32 : (const T *)H->lev[l + 1].w64);
            T *w = f32 ? (T *)L.w32 : (T *)L.w64;
            const T *cr = f32 ? (const T *)L.crem32 : (const T *)L.crem64;
            Span sp(H, s, PASS_UP, l);
            k_up<T><<<(int)L.ncell, 64, 0, s>>>(L.ncell, L.m, L.k, L.tt_off, L.piv_ptr, L.ipos, L.rem_ptr, L.rem_pos,
                                                L.crem_off, cr, src, w);
            HIPCHECK(hipGetLastError());
        }
        // transverse pass
        for (int l = lmin; l <= kap; l++) {
            nnca::Level &L = H->lev[l];
            Span sp(H, s, PASS_M2L, l);
            if (f32) launch_m2l<T>(H->kind, L, (const T *)L.pc32, H->dim, (const T *)L.w32, (T *)L.u32, prm, s);
            else launch_m2l<T>(H->kind, L, (const T *)L.pc64, H->dim, (const T *)L.w64, (T *)L.u64, prm, s);
        }
        // downward pass
        far = f32 ? (T *)H->far32 : (T *)H->far64;
        for (int l = lmin; l <= kap; l++) {
            nnca::Level &L = H->lev[l];
            const T *cr = f32 ? (const T *)L.crem32 : (const T *)L.crem64;
            const T *u = f32 ? (const T *)L.u32 : (const T *)L.u64;
            T *out = (l == kap) ? far : (f32 ? (T *)H->lev[l + 1].u32 : (T *)H->lev[l + 1].u64);
            Span sp(H, s, PASS_DOWN, l);
            k_down<T><<<(int)L.ncell, 64, 0, s>>>(L.ncell, L.k, L.tt_off, L.piv_ptr, L.ipos, L.rem_ptr, L.rem_pos,
                                                  L.crem_off, cr, u, out, l == kap ? 0 : 1);
            HIPCHECK(hipGetLastError());
        }
    }
    // near field and combine
    Span sp(H, s, PASS_P2P, kap);
    if (f32) launch_p2p<T>(H->kind, H, (const T *)H->pts32, xin, xin2, far, y, prm, s);
    else launch_p2p<T>(H->kind, H, (const T *)H->pts64, xin, nullptr, far, y, prm, s);
}

}  // namespace

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
        L.crem32 = dalloc<float>(L.ncrem);
        if (L.ncrem) k_to_f32<<<grid_for(L.ncrem, 256), 256, 0, s>>>(L.ncrem, L.crem64, L.crem32);
        L.ilpre = dalloc<int32_t>(L.nil);
        L.ilsum = dalloc<int32_t>(nc);
        k_list_prefix<<<grid_for(nc, 256), 256, 0, s>>>(nc, L.il_ptr, L.il, L.k, L.ilpre, L.ilsum);
        L.w64 = dalloc<double>(L.npiv);
        L.u64 = dalloc<double>(L.npiv);
        L.w32 = dalloc<float>(L.npiv);
        L.u32 = dalloc<float>(L.npiv);
        HIPCHECK(hipGetLastError());
        std::vector<int32_t> ils(nc);
        HIPCHECK(hipMemcpyAsync(ils.data(), L.ilsum, sizeof(int32_t) * nc, hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        L.max_ilsum = 0;
        for (int64_t c = 0; c < nc; c++) {
            m2l += (int64_t)L.h_k[c] * ils[c];
            L.max_ilsum = std::max(L.max_ilsum, ils[c]);
        }
        trans += L.ncrem;
    }
    Level &F = H->lev[H->kappa];
    int64_t nc = F.ncell;
    int32_t *cnt = F.count;
    H->nbpre = dalloc<int32_t>(F.nnb);
    H->nbsum = dalloc<int32_t>(nc);
    k_list_prefix<<<grid_for(nc, 256), 256, 0, s>>>(nc, F.nb_ptr, F.nb, cnt, H->nbpre, H->nbsum);
    H->pts32 = dalloc<float>(3 * H->n);
    k_point_local<<<(int)nc, 64, 0, s>>>(nc, F.first, F.count, H->pts64, H->n, d, F.coord, H->lo[0], H->lo[1],
                                         H->lo[2], F.h, H->pts32);
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
    H->m2l_inter = m2l;
    H->p2p_inter = p2p;
    H->transfer_entries = trans;
    H->xs64 = dalloc<double>(H->n);
    H->far64 = dalloc<double>(H->n);
    H->xhi = dalloc<float>(H->n);
    H->xlo = dalloc<float>(H->n);
    H->far32 = dalloc<float>(H->n);
}

void run_matvec(nnca_h2 *H, const double *X, double *Y, int64_t nrhs, int64_t ldx, int64_t ldy, int precision,
                hipStream_t s)
{
    const int64_t n = H->n;
    for (int64_t col = 0; col < nrhs; col++) {
        const double *x = X + col * ldx;
        double *y = Y + col * ldy;
        if (precision == NNCA_PREC_MIXED) {
            {
                Span sp(H, s, PASS_GATHER, -1);
                k_gather_split<<<grid_for(n, 256), 256, 0, s>>>(n, H->order, x, H->xhi, H->xlo);
                HIPCHECK(hipGetLastError());
            }
            one_column<float>(H, H->xhi, H->xlo, y, s);
        } else {
            {
                Span sp(H, s, PASS_GATHER, -1);
                k_gather64<<<grid_for(n, 256), 256, 0, s>>>(n, H->order, x, H->xs64);
                HIPCHECK(hipGetLastError());
            }
            one_column<double>(H, H->xs64, nullptr, y, s);
        }
    }
}

void run_direct(const double *pts, int64_t n, int dim, int64_t ld, int kind, double hparam, const double *X,
                double *Y, int64_t nrhs, int64_t ldx, int64_t ldy, hipStream_t s)
{
    double prm = 1.0 / (hparam * hparam);
    for (int64_t col = 0; col < nrhs; col++) {
        const double *x = X + col * ldx;
        double *y = Y + col * ldy;
        int g = grid_for(n, NT);
        if (kind == NNCA_K_INV_R) k_direct<NNCA_K_INV_R><<<g, NT, 0, s>>>(pts, n, dim, ld, x, y, prm);
        else if (kind == NNCA_K_LOG_R) k_direct<NNCA_K_LOG_R><<<g, NT, 0, s>>>(pts, n, dim, ld, x, y, prm);
        else k_direct<NNCA_K_GAUSS><<<g, NT, 0, s>>>(pts, n, dim, ld, x, y, prm);
        HIPCHECK(hipGetLastError());
    }
}

}  // namespace nnca
