// Uniform 2^d tree (Sec. 2.1) and neighbour / interaction lists (Sec. 2.2,
// Table 1) built on the GPU.
//
// Order of the points: ascending Morton key at the finest level kmax =
// floor(60/d), ties by original index (stable radix sort of (key, index)).
// Cells of level l are the distinct key prefixes key >> d(kmax - l).
// Depth kappa: the first level at which no cell holds more than nu points,
// found from the sorted keys: points i and i+nu share a cell exactly down to
// the level given by the common prefix of their keys.
#include <cstring>

#include "nnca_internal.h"

#pragma clang fp contract(off)

namespace nnca {
namespace {

__device__ inline uint64_t morton(const int64_t *c, int d, int bits)
{
    uint64_t k = 0;
    for (int b = 0; b < bits; b++)
        for (int q = 0; q < d; q++) k |= (uint64_t)((c[q] >> b) & 1) << (d * b + q);
    return k;
}

__device__ inline int64_t find_key(const uint64_t *keys, int64_t nc, uint64_t key)
{
    int64_t lo = 0, hi = nc - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) >> 1;
        uint64_t v = keys[mid];
        if (v == key) return mid;
        if (v < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// d * den <= num * sum_q g_q^2 with g_q = max(|a_q - b_q| - 1, 0): the
// admissibility condition max(diam) <= eta dist for equal cubes.
__device__ inline bool admissible(const int64_t *a, const int64_t *b, int d, int64_t num, int64_t den)
{
    int64_t s = 0;
    for (int q = 0; q < d; q++) {
        int64_t g = a[q] > b[q] ? a[q] - b[q] : b[q] - a[q];
        g = g - 1;
        if (g < 0) g = 0;
        s += g * g;
    }
    return (int64_t)d * den <= num * s;
}

__global__ void k_finite(const double *p, int64_t n, int d, int64_t ld, int *bad)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int q = 0; q < d; q++) {
            double v = p[q * ld + i];
            if (!(v == v) || v == INFINITY || v == -INFINITY) *bad = 1;
        }
}

// per-block min / max of every axis; 256 threads
__global__ void k_bbox_partial(const double *p, int64_t n, int d, int64_t ld, double *part)
{
    __shared__ double smin[3][256], smax[3][256];
    int t = threadIdx.x;
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = blockIdx.x * (int64_t)256 + t; i < n; i += (int64_t)gridDim.x * 256)
        for (int q = 0; q < d; q++) {
            double v = p[q * ld + i];
            mn[q] = v < mn[q] ? v : mn[q];
            mx[q] = v > mx[q] ? v : mx[q];
        }
    for (int q = 0; q < 3; q++) { smin[q][t] = mn[q]; smax[q][t] = mx[q]; }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s)
            for (int q = 0; q < 3; q++) {
                smin[q][t] = smin[q][t + s] < smin[q][t] ? smin[q][t + s] : smin[q][t];
                smax[q][t] = smax[q][t + s] > smax[q][t] ? smax[q][t + s] : smax[q][t];
            }
        __syncthreads();
    }
    if (t == 0)
        for (int q = 0; q < 3; q++) {
            part[blockIdx.x * 6 + q] = smin[q][0];
            part[blockIdx.x * 6 + 3 + q] = smax[q][0];
        }
}

// finest Morton key of every point (original order) and its index
__global__ void k_keys(const double *p, int64_t n, int d, int64_t ld, double lo0, double lo1, double lo2,
                       double L, int kmax, uint64_t *key, int32_t *idx)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double lo[3] = {lo0, lo1, lo2};
    int64_t side = (int64_t)1 << kmax;
    int64_t c[3] = {0, 0, 0};
    if (L > 0.0)
        for (int q = 0; q < d; q++) {
            double u = (p[q * ld + i] - lo[q]) / L;
            int64_t v = (int64_t)floor(u * (double)side);
            c[q] = v < side - 1 ? v : side - 1;
        }
    key[i] = morton(c, d, kmax);
    idx[i] = (int32_t)i;
}

// deepest level needed by the pair of sorted points (i, i + nu)
__global__ void k_depth(const uint64_t *key, int64_t n, int64_t nu, int d, int kmax, int *kappa)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i + nu >= n) return;
    uint64_t x = key[i] ^ key[i + nu];
    int agree = (x == 0 ? 64 : __clzll((long long)x)) - (64 - d * kmax);
    int shared = agree / d;              // levels whose cell holds points i..i+nu
    int need = shared + 1;
    if (need > kmax) need = kmax;
    atomicMax(kappa, need);
}

// general case: flag[i] = 1 when the sorted point i belongs to P
__global__ void k_class_flag(const int32_t *order, int64_t n, int64_t split, int32_t *flag)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) flag[i] = order[i] < split ? 1 : 0;
}

// stable split of the sorted union into P's and Q's tree orders (pre: the
// exclusive count of P points before each sorted position); the keys of
// each set, and their original indices (Q's relative to split)
__global__ void k_split_sorted(const uint64_t *key, const int32_t *order, int64_t n, int64_t split,
                               const int32_t *pre, uint64_t *pkey, uint64_t *qkey, int32_t *porder,
                               int32_t *qorder)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t o = order[i];
    if (o < split) {
        if (pkey) pkey[pre[i]] = key[i];
        if (porder) porder[pre[i]] = o;
    } else {
        const int64_t q = i - pre[i];
        if (qkey) qkey[q] = key[i];
        if (qorder) qorder[q] = (int32_t)(o - split);
    }
}

// per cell: its range of P points and of Q points in the two tree orders
__global__ void k_split_ranges(int64_t nc, const int32_t *first, const int32_t *count, const int32_t *pre,
                               int32_t *pfirst, int32_t *pcount, int32_t *qfirst, int32_t *qcount)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int32_t f = first[c], e = f + count[c];
    const int32_t a = pre[f], b = pre[e];
    pfirst[c] = a;
    pcount[c] = b - a;
    qfirst[c] = f - a;
    qcount[c] = (e - b) - (f - a);
}

__global__ void k_gather_pts(const double *p, int64_t n, int d, int64_t ld, const int32_t *order, double *out)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t o = order[i];
    for (int q = 0; q < d; q++) out[q * n + i] = p[q * ld + o];
}

__global__ void k_flags(const uint64_t *key, int64_t n, int shift, int32_t *flag)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    flag[i] = (i == 0 || (key[i] >> shift) != (key[i - 1] >> shift)) ? 1 : 0;
}

__global__ void k_cells(const uint64_t *key, int64_t n, int shift, const int32_t *flag, const int32_t *cinc,
                        int32_t *first, uint64_t *ckey)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    int32_t c = cinc[i] - 1;
    first[c] = (int32_t)i;
    ckey[c] = key[i] >> shift;
}

__global__ void k_cell_info(int64_t nc, int64_t n, int d, int l, const int32_t *first, const uint64_t *ckey,
                            int32_t *count, int32_t *coord)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    count[c] = (int32_t)((c + 1 < nc ? first[c + 1] : n) - first[c]);
    uint64_t k = ckey[c];
    for (int q = 0; q < d; q++) {
        int64_t v = 0;
        for (int b = 0; b < l; b++) v |= (int64_t)((k >> (d * b + q)) & 1) << b;
        coord[q * nc + c] = (int32_t)v;
    }
}

__global__ void k_parent(int64_t nc, const int32_t *first, const int32_t *cinc_prev, int32_t *parent)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    parent[c] = cinc_prev ? cinc_prev[first[c]] - 1 : -1;
}

__global__ void k_child_first(int64_t nc, const int32_t *parent, int32_t *child_first)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int32_t p = parent[c];
    if (c == 0 || parent[c - 1] != p) child_first[p] = (int32_t)c;
}

__global__ void k_child_count(int64_t nc, const int32_t *parent, const int32_t *child_first, int32_t *child_count)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int32_t p = parent[c];
    if (c == nc - 1 || parent[c + 1] != p) child_count[p] = (int32_t)(c + 1 - child_first[p]);
}

// N(B) (which = 0) or IL(B) (which = 1) of every cell of level l: count
// (out == nullptr) or fill and sort ascending.
__global__ void k_lists(int which, int l, int d, int64_t nc, const int32_t *coord, const uint64_t *keys,
                        int64_t pnc, const int32_t *pcoord, const uint64_t *pkeys, const int32_t *parent,
                        const int32_t *pchild_first, const int32_t *pchild_count, int R, int64_t num,
                        int64_t den, int32_t *cnt_out, const int32_t *ptr, int32_t *out)
{
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= nc) return;
    int64_t me[3] = {0, 0, 0};
    for (int q = 0; q < d; q++) me[q] = coord[q * nc + c];
    int32_t cnt = 0;
    int32_t *dst = out ? out + ptr[c] : nullptr;
    int lv = which == 0 ? l : l - 1;
    int64_t side = (int64_t)1 << lv;
    int64_t base[3] = {0, 0, 0};
    int32_t p = -1;
    if (which == 0) {
        for (int q = 0; q < d; q++) base[q] = me[q];
    } else {
        if (l == 0) { if (!out) cnt_out[c] = 0; return; }
        p = parent[c];
        for (int q = 0; q < d; q++) base[q] = pcoord[q * pnc + p];
    }
    int64_t off[3] = {-R, -R, (d == 3) ? -R : 0};
    for (;;) {
        int64_t cc[3] = {0, 0, 0};
        bool ok = true;
        for (int q = 0; q < d; q++) {
            cc[q] = base[q] + off[q];
            if (cc[q] < 0 || cc[q] >= side) ok = false;
        }
        if (ok && !admissible(base, cc, d, num, den)) {
            if (which == 0) {
                int64_t id = find_key(keys, nc, morton(cc, d, lv));
                if (id >= 0) {
                    if (dst) dst[cnt] = (int32_t)id;
                    cnt++;
                }
            } else {
                int64_t pid = find_key(pkeys, pnc, morton(cc, d, lv));
                if (pid >= 0) {
                    int32_t f = pchild_first[pid], e = f + pchild_count[pid];
                    for (int32_t ch = f; ch < e; ch++) {
                        int64_t co[3] = {0, 0, 0};
                        for (int q = 0; q < d; q++) co[q] = coord[q * nc + ch];
                        if (admissible(me, co, d, num, den)) {
                            if (dst) dst[cnt] = ch;
                            cnt++;
                        }
                    }
                }
            }
        }
        int q = 0;
        while (q < d && ++off[q] > R) { off[q] = -R; q++; }
        if (q == d) break;
    }
    if (!out) {
        cnt_out[c] = cnt;
        return;
    }
    for (int32_t a = 1; a < cnt; a++) {
        int32_t v = dst[a];
        int32_t b = a - 1;
        while (b >= 0 && dst[b] > v) { dst[b + 1] = dst[b]; b--; }
        dst[b + 1] = v;
    }
}

// Prefix sums.  The values are integers, so the sums are exact in any
// order.  Blocks of SC_NT threads scan tiles of SC_TILE elements (SC_IPT
// consecutive elements per thread), one block scans the tile totals, and the
// totals' prefixes are added to the tiles.
constexpr int SC_NT = 256, SC_IPT = 8, SC_TILE = SC_NT * SC_IPT;

// exclusive scan of one value per thread over the block; *total = the sum
template <typename T>
__device__ T block_excl_scan(T v, T *sh, T &total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < SC_NT; o <<= 1) {
        const T x = t >= o ? sh[t - o] : T(0);
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    total = sh[SC_NT - 1];
    const T r = sh[t] - v;
    __syncthreads();
    return r;
}

template <typename T>
__global__ __launch_bounds__(SC_NT) void k_scan_tiles(const T *in, T *out, int64_t n, T *tile_sum, int inclusive)
{
    __shared__ T sh[SC_NT];
    const int t = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * SC_TILE + (int64_t)t * SC_IPT;
    T v[SC_IPT], sum = T(0);
#pragma unroll
    for (int i = 0; i < SC_IPT; i++) {
        v[i] = b0 + i < n ? in[b0 + i] : T(0);
        sum += v[i];
    }
    T tot;
    T run = block_excl_scan(sum, sh, tot);
#pragma unroll
    for (int i = 0; i < SC_IPT; i++) {
        if (b0 + i < n) out[b0 + i] = inclusive ? run + v[i] : run;
        run += v[i];
    }
    if (t == 0) tile_sum[blockIdx.x] = tot;
}

// exclusive scan of the nt tile totals, in place, by one block
template <typename T>
__global__ __launch_bounds__(SC_NT) void k_scan_sums(T *sum, int64_t nt)
{
    __shared__ T sh[SC_NT];
    T carry = T(0);
    for (int64_t c0 = 0; c0 < nt; c0 += SC_NT) {
        const int64_t g = c0 + threadIdx.x;
        const T v = g < nt ? sum[g] : T(0);
        T tot;
        const T pre = block_excl_scan(v, sh, tot);
        if (g < nt) sum[g] = carry + pre;
        carry += tot;
    }
}

template <typename T>
__global__ void k_scan_add(T *out, int64_t n, const T *tile_off)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g < n) out[g] += tile_off[g / SC_TILE];
}

template <typename T>
void scan(const T *in, T *out, int64_t n, bool inclusive, hipStream_t s)
{
    if (n <= 0) return;
    const int64_t nt = (n + SC_TILE - 1) / SC_TILE;
    if (nt > INT32_MAX) fail(NNCA_ERR_NOT_SUPPORTED, "scan too long");
    T *tsum = dalloc<T>(nt);
    try {
        k_scan_tiles<T><<<(unsigned)nt, SC_NT, 0, s>>>(in, out, n, tsum, inclusive ? 1 : 0);
        HIPCHECK(hipGetLastError());
        if (nt > 1) {
            k_scan_sums<T><<<1, SC_NT, 0, s>>>(tsum, nt);
            HIPCHECK(hipGetLastError());
            k_scan_add<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(out, n, tsum);
            HIPCHECK(hipGetLastError());
        }
        HIPCHECK(hipStreamSynchronize(s));
    } catch (...) {
        (void)hipStreamSynchronize(s);
        dfree(tsum);
        throw;
    }
    dfree(tsum);
}

// Stable LSD radix sort of (64-bit key, 32-bit value) pairs on key bits
// [0, bits), eight bits per pass.  Per pass: each block counts the digits of
// its tile of RS_TILE pairs; an exclusive scan of the counts laid out digit
// by digit, block by block, gives every (digit, block) its first output
// position; each block then writes its tile in index order, 256 pairs at a
// time, a pair's place among equal digits of its wavefront from the lanes
// below it (ballots on the eight digit bits), after those of the
// wavefronts below and of the earlier chunks.  Equal keys keep their input
// order, so input in index order sorts by (key, index).
constexpr int RS_NT = 256, RS_IPT = 16, RS_TILE = RS_NT * RS_IPT, RS_WAVES = RS_NT / 64;

__global__ __launch_bounds__(RS_NT) void k_rs_hist(const uint64_t *key, int64_t n, int shift, int32_t *hist,
                                                   int64_t nb)
{
    __shared__ int32_t h[256];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t tb = (int64_t)blockIdx.x * RS_TILE;
    for (int i = 0; i < RS_IPT; i++) {
        const int64_t g = tb + (int64_t)i * RS_NT + t;
        if (g < n) atomicAdd(&h[(int)((key[g] >> shift) & 255u)], 1);
    }
    __syncthreads();
    hist[(int64_t)t * nb + blockIdx.x] = h[t];
}

__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const uint64_t *kin, const int32_t *vin, uint64_t *kout,
                                                      int32_t *vout, int64_t n, int shift, const int32_t *off,
                                                      int64_t nb)
{
    __shared__ int32_t base[256];
    __shared__ int32_t wcnt[RS_WAVES][256];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    base[t] = off[(int64_t)t * nb + blockIdx.x];
    for (int q = 0; q < RS_WAVES; q++) wcnt[q][t] = 0;
    __syncthreads();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int64_t tb = (int64_t)blockIdx.x * RS_TILE;
    for (int i = 0; i < RS_IPT; i++) {
        const int64_t g = tb + (int64_t)i * RS_NT + t;
        const bool ok = g < n;
        const uint64_t k = ok ? kin[g] : 0ull;
        const int32_t v = ok ? vin[g] : 0;
        const int dg = (int)((k >> shift) & 255u);
        uint64_t m = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = ((dg >> b) & 1) != 0;
            const uint64_t bb = __ballot(ok && bit);
            m &= bit ? bb : ~bb;
        }
        const int rank = __popcll(m & below);
        if (ok && rank == 0) wcnt[w][dg] = __popcll(m);
        __syncthreads();
        if (ok) {
            int32_t pos = base[dg] + rank;
            for (int q = 0; q < w; q++) pos += wcnt[q][dg];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        int32_t c = 0;
        for (int q = 0; q < RS_WAVES; q++) {
            c += wcnt[q][t];
            wcnt[q][t] = 0;
        }
        base[t] += c;
        __syncthreads();
    }
}

// sorts (k_in, v_in) into (k_out, v_out); k_in and v_in are overwritten
void radix_sort_pairs(uint64_t *k_in, int32_t *v_in, uint64_t *k_out, int32_t *v_out, int64_t n, int bits,
                      hipStream_t s)
{
    if (n <= 0) return;
    if (n > INT32_MAX) fail(NNCA_ERR_NOT_SUPPORTED, "sort too long");
    const int passes = (bits + 7) / 8;
    if (passes == 0) {
        HIPCHECK(hipMemcpyAsync(k_out, k_in, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
        HIPCHECK(hipMemcpyAsync(v_out, v_in, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        HIPCHECK(hipStreamSynchronize(s));
        return;
    }
    const int64_t nb = (n + RS_TILE - 1) / RS_TILE;
    int32_t *hist = dalloc<int32_t>(256 * nb);
    uint64_t *kt = passes > 1 ? dalloc<uint64_t>(n) : nullptr;
    int32_t *vt = passes > 1 ? dalloc<int32_t>(n) : nullptr;
    auto release = [&] {
        dfree(hist);
        dfree(kt);
        dfree(vt);
    };
    try {
        uint64_t *ks = k_in;
        int32_t *vs = v_in;
        for (int p = 0; p < passes; p++) {
            uint64_t *kd = p == passes - 1 ? k_out : (ks == k_in ? kt : k_in);
            int32_t *vd = p == passes - 1 ? v_out : (vs == v_in ? vt : v_in);
            k_rs_hist<<<(unsigned)nb, RS_NT, 0, s>>>(ks, n, 8 * p, hist, nb);
            HIPCHECK(hipGetLastError());
            scan<int32_t>(hist, hist, 256 * nb, false, s);
            k_rs_scatter<<<(unsigned)nb, RS_NT, 0, s>>>(ks, vs, kd, vd, n, 8 * p, hist, nb);
            HIPCHECK(hipGetLastError());
            ks = kd;
            vs = vd;
        }
        HIPCHECK(hipStreamSynchronize(s));
    } catch (...) {
        (void)hipStreamSynchronize(s);
        release();
        throw;
    }
    release();
}

}  // namespace

void scan_i32(const int32_t *in, int32_t *out, int64_t n, bool inclusive, hipStream_t s)
{
    scan<int32_t>(in, out, n, inclusive, s);
}
void scan_i64(const int64_t *in, int64_t *out, int64_t n, bool inclusive, hipStream_t s)
{
    scan<int64_t>(in, out, n, inclusive, s);
}

// CSR of N(B) or IL(B) for one level
static void build_list(nnca_h2 *H, int l, int which, int R)
{
    Level &L = H->lev[l];
    hipStream_t s = H->stream;
    const Level *P = l > 0 ? &H->lev[l - 1] : nullptr;
    int64_t nc = L.ncell;
    int32_t *cnt = dalloc<int32_t>(nc + 1);
    int32_t *ptr = dalloc<int32_t>(nc + 1);
    HIPCHECK(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (nc + 1), s));
    int g = grid_for(nc, 128);
    k_lists<<<g, 128, 0, s>>>(which, l, H->dim, nc, L.coord, L.key, P ? P->ncell : 0, P ? P->coord : nullptr,
                              P ? P->key : nullptr, L.parent, P ? P->child_first : nullptr,
                              P ? P->child_count : nullptr, R, H->eta_num, H->eta_den, cnt, nullptr, nullptr);
    HIPCHECK(hipGetLastError());
    scan<int32_t>(cnt, ptr, nc + 1, false, s);
    int32_t total = 0;
    HIPCHECK(hipMemcpy(&total, ptr + nc, sizeof(int32_t), hipMemcpyDeviceToHost));
    int32_t *idx = dalloc<int32_t>(total + 1);
    k_lists<<<g, 128, 0, s>>>(which, l, H->dim, nc, L.coord, L.key, P ? P->ncell : 0, P ? P->coord : nullptr,
                              P ? P->key : nullptr, L.parent, P ? P->child_first : nullptr,
                              P ? P->child_count : nullptr, R, H->eta_num, H->eta_den, nullptr, ptr, idx);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(s));
    dfree(cnt);
    if (which == 0) { L.nb_ptr = ptr; L.nb = idx; L.nnb = total; }
    else { L.il_ptr = ptr; L.il = idx; L.nil = total; }
}

// exclusive count of P points before every sorted position, n + 1 entries
static int32_t *class_prefix(nnca_h2 *H, int64_t split)
{
    hipStream_t s = H->stream;
    const int64_t n = H->n;
    int32_t *flag = dalloc<int32_t>(n + 1);
    int32_t *pre = dalloc<int32_t>(n + 1);
    HIPCHECK(hipMemsetAsync(flag, 0, sizeof(int32_t) * (n + 1), s));
    k_class_flag<<<grid_for(n, 256), 256, 0, s>>>(H->order, n, split, flag);
    HIPCHECK(hipGetLastError());
    scan<int32_t>(flag, pre, n + 1, false, s);
    dfree(flag);
    return pre;
}

void build_tree(nnca_h2 *H, const double *pin, int64_t ld, int64_t split)
{
    hipStream_t s = H->stream;
    const int64_t n = H->n;
    const int d = H->dim;
    H->kmax = 60 / d;

    // reject non-finite coordinates
    int *bad = dalloc<int>(1);
    HIPCHECK(hipMemsetAsync(bad, 0, sizeof(int), s));
    k_finite<<<grid_for(n, 256) > 4096 ? 4096 : grid_for(n, 256), 256, 0, s>>>(pin, n, d, ld, bad);
    HIPCHECK(hipGetLastError());
    int hbad = 0;
    HIPCHECK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    dfree(bad);
    if (hbad) fail(NNCA_ERR_INVALID_ARG, "points contain a non-finite coordinate");

    // domain D: cube at the per-axis minimum with the largest extent as side
    int nb = grid_for(n, 256);
    if (nb > 1024) nb = 1024;
    double *part = dalloc<double>(6 * nb);
    k_bbox_partial<<<nb, 256, 0, s>>>(pin, n, d, ld, part);
    HIPCHECK(hipGetLastError());
    std::vector<double> hp(6 * nb);
    HIPCHECK(hipMemcpyAsync(hp.data(), part, sizeof(double) * 6 * nb, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    dfree(part);
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < nb; b++)
        for (int q = 0; q < d; q++) {
            mn[q] = hp[b * 6 + q] < mn[q] ? hp[b * 6 + q] : mn[q];
            mx[q] = hp[b * 6 + 3 + q] > mx[q] ? hp[b * 6 + 3 + q] : mx[q];
        }
    H->L = 0.0;
    for (int q = 0; q < d; q++) {
        H->lo[q] = mn[q];
        double e = mx[q] - mn[q];
        if (e > H->L) H->L = e;
    }

    // keys, stable sort by (key, original index)
    uint64_t *k_in = dalloc<uint64_t>(n);
    int32_t *i_in = dalloc<int32_t>(n);
    H->keys = dalloc<uint64_t>(n);
    H->order = dalloc<int32_t>(n);
    k_keys<<<grid_for(n, 256), 256, 0, s>>>(pin, n, d, ld, H->lo[0], H->lo[1], H->lo[2], H->L, H->kmax, k_in, i_in);
    HIPCHECK(hipGetLastError());
    radix_sort_pairs(k_in, i_in, H->keys, H->order, n, d * H->kmax, s);
    dfree(k_in);
    dfree(i_in);

    // depth: the first level with at most nu points in every cell; in the
    // general case at most nu points of P and at most nu of Q (Sec. 2.1),
    // found on each set's sorted keys
    int kap = 0;
    if (H->L > 0.0 && n > H->leaf) {
        int *dk = dalloc<int>(1);
        HIPCHECK(hipMemsetAsync(dk, 0, sizeof(int), s));
        if (split < 0) {
            k_depth<<<grid_for(n, 256), 256, 0, s>>>(H->keys, n, H->leaf, d, H->kmax, dk);
            HIPCHECK(hipGetLastError());
        } else {
            int32_t *pre = class_prefix(H, split);
            uint64_t *pk = dalloc<uint64_t>(split), *qk = dalloc<uint64_t>(n - split);
            k_split_sorted<<<grid_for(n, 256), 256, 0, s>>>(H->keys, H->order, n, split, pre, pk, qk, nullptr,
                                                             nullptr);
            HIPCHECK(hipGetLastError());
            if (split > H->leaf) k_depth<<<grid_for(split, 256), 256, 0, s>>>(pk, split, H->leaf, d, H->kmax, dk);
            if (n - split > H->leaf)
                k_depth<<<grid_for(n - split, 256), 256, 0, s>>>(qk, n - split, H->leaf, d, H->kmax, dk);
            HIPCHECK(hipGetLastError());
            HIPCHECK(hipStreamSynchronize(s));
            dfree(pre);
            dfree(pk);
            dfree(qk);
        }
        HIPCHECK(hipMemcpyAsync(&kap, dk, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        dfree(dk);
    }
    H->kappa = kap;

    H->pts64 = dalloc<double>(3 * n);
    HIPCHECK(hipMemsetAsync(H->pts64, 0, sizeof(double) * 3 * n, s));
    k_gather_pts<<<grid_for(n, 256), 256, 0, s>>>(pin, n, d, ld, H->order, H->pts64);
    HIPCHECK(hipGetLastError());

    // cells of every level
    H->lev.assign(kap + 1, Level());
    int32_t *flag = dalloc<int32_t>(n);
    int32_t *cinc = dalloc<int32_t>(n);
    int32_t *cprev = dalloc<int32_t>(n);
    for (int l = 0; l <= kap; l++) {
        Level &L = H->lev[l];
        L.h = ldexp(H->L, -l);
        int shift = d * (H->kmax - l);
        k_flags<<<grid_for(n, 256), 256, 0, s>>>(H->keys, n, shift, flag);
        HIPCHECK(hipGetLastError());
        scan<int32_t>(flag, cinc, n, true, s);
        int32_t nc = 0;
        HIPCHECK(hipMemcpy(&nc, cinc + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost));
        L.ncell = nc;
        L.first = dalloc<int32_t>(nc);
        L.count = dalloc<int32_t>(nc);
        L.key = dalloc<uint64_t>(nc);
        L.coord = dalloc<int32_t>(3 * (int64_t)nc);
        L.parent = dalloc<int32_t>(nc);
        L.child_first = dalloc<int32_t>(nc);
        L.child_count = dalloc<int32_t>(nc);
        HIPCHECK(hipMemsetAsync(L.coord, 0, sizeof(int32_t) * 3 * nc, s));
        HIPCHECK(hipMemsetAsync(L.child_first, 0, sizeof(int32_t) * nc, s));
        HIPCHECK(hipMemsetAsync(L.child_count, 0, sizeof(int32_t) * nc, s));
        k_cells<<<grid_for(n, 256), 256, 0, s>>>(H->keys, n, shift, flag, cinc, L.first, L.key);
        k_cell_info<<<grid_for(nc, 256), 256, 0, s>>>(nc, n, d, l, L.first, L.key, L.count, L.coord);
        k_parent<<<grid_for(nc, 256), 256, 0, s>>>(nc, L.first, l > 0 ? cprev : nullptr, L.parent);
        HIPCHECK(hipGetLastError());
        if (l > 0) {
            Level &P = H->lev[l - 1];
            k_child_first<<<grid_for(nc, 256), 256, 0, s>>>(nc, L.parent, P.child_first);
            k_child_count<<<grid_for(nc, 256), 256, 0, s>>>(nc, L.parent, P.child_first, P.child_count);
            HIPCHECK(hipGetLastError());
        }
        std::swap(cinc, cprev);
        HIPCHECK(hipStreamSynchronize(s));
    }
    dfree(flag);
    dfree(cinc);
    dfree(cprev);

    // lists
    int R = 1 + (int)ceil(sqrt((double)d * (double)H->eta_den / (double)H->eta_num));
    for (int l = 0; l <= kap; l++) {
        build_list(H, l, 0, R);
        build_list(H, l, 1, R);
    }
    // lmin: the coarsest level with a non-empty interaction list
    H->lmin = kap + 1;
    for (int l = 1; l <= kap; l++)
        if (H->lev[l].nil > 0) { H->lmin = l; break; }
}

void split_general(nnca_h2 *H, const double *Z, int64_t ldz, int64_t split)
{
    hipStream_t s = H->stream;
    const int64_t n = H->n, np = split, nq = n - split;
    const int d = H->dim;
    int32_t *pre = class_prefix(H, split);
    int32_t *porder = dalloc<int32_t>(np);
    H->qorder = dalloc<int32_t>(nq);
    k_split_sorted<<<grid_for(n, 256), 256, 0, s>>>(H->keys, H->order, n, split, pre, nullptr, nullptr, porder,
                                                     H->qorder);
    HIPCHECK(hipGetLastError());
    H->lev_o.assign(H->lev.size(), Level());
    for (size_t l = 0; l < H->lev.size(); l++) {
        Level &L = H->lev[l];
        Level &O = H->lev_o[l];
        const int64_t nc = L.ncell;
        int32_t *pf = dalloc<int32_t>(nc), *pc = dalloc<int32_t>(nc);
        int32_t *qf = dalloc<int32_t>(nc), *qc = dalloc<int32_t>(nc);
        k_split_ranges<<<grid_for(nc, 256), 256, 0, s>>>(nc, L.first, L.count, pre, pf, pc, qf, qc);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(s));
        dfree(L.first);
        dfree(L.count);
        L.first = pf;
        L.count = pc;
        O = L;   // the tree fields, shared
        O.shares_tree = true;
        O.first = qf;
        O.count = qc;
    }
    // the points of each set in its own tree order
    dfree(H->pts64);
    H->pts64 = nullptr;
    double *pp = dalloc<double>(3 * np), *qp = dalloc<double>(3 * nq);
    HIPCHECK(hipMemsetAsync(pp, 0, sizeof(double) * 3 * np, s));
    HIPCHECK(hipMemsetAsync(qp, 0, sizeof(double) * 3 * nq, s));
    k_gather_pts<<<grid_for(np, 256), 256, 0, s>>>(Z, np, d, ldz, porder, pp);
    k_gather_pts<<<grid_for(nq, 256), 256, 0, s>>>(Z + split, nq, d, ldz, H->qorder, qp);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(s));
    dfree(pre);
    dfree(H->order);
    H->order = porder;
    H->pts64 = pp;
    H->qpts64 = qp;
    H->n = np;
    H->nq = nq;
    H->general = true;
}

}  // namespace nnca
