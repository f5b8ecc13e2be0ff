// C ABI of the library (declared in include/nnca.h): argument checks, error
// translation, handle lifetime, parity exports.
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <new>
#include <utility>

#include "nnca_internal.h"

namespace nnca {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

void fail(nnca_status s, const std::string &msg) { throw Error{s, msg}; }

void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? NNCA_ERR_OUT_OF_MEMORY : NNCA_ERR_HIP,
             std::string(what) + ": " + hipGetErrorString(e));
    }
}

static thread_local const Allocator *tl_alloc = nullptr;

const Allocator *current_allocator() { return tl_alloc; }

AllocScope::AllocScope(const Allocator &a) : prev(tl_alloc) { tl_alloc = &a; }
AllocScope::~AllocScope() { tl_alloc = prev; }

void *dalloc_bytes(size_t bytes)
{
    void *p = nullptr;
    const Allocator *a = tl_alloc;
    if (a && a->alloc) {
        p = a->alloc(bytes, a->ctx);
        if (!p) fail(NNCA_ERR_OUT_OF_MEMORY, "the caller's allocator returned NULL for " + std::to_string(bytes) +
                                                 " bytes");
        return p;
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(NNCA_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return p;
}

// A caller's allocator may hand the memory to other work at once (a caching
// allocator), so the device is drained first, as hipFree does by itself.
void dfree(void *p)
{
    if (!p) return;
    const Allocator *a = tl_alloc;
    if (a && a->free) {
        (void)hipDeviceSynchronize();
        a->free(p, a->ctx);
        return;
    }
    (void)hipFree(p);
}

}  // namespace nnca

using namespace nnca;

template <typename F>
static nnca_status guarded(F &&f)
{
    try {
        f();
        return NNCA_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return NNCA_ERR_OUT_OF_MEMORY;
    } catch (...) {
        set_error("unexpected exception");
        return NNCA_ERR_INTERNAL;
    }
}

static void clear_profile(nnca_h2 *H)
{
    for (auto &r : H->prof) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    H->prof.clear();
}

void nnca::destroy_handle(nnca_h2 *H)
{
    if (!H) return;
    clear_profile(H);
    free_multi(H);
    free_grad(H);
    if (H->aux) {
        (void)hipStreamSynchronize(H->aux);
        (void)hipStreamDestroy(H->aux);
    }
    if (H->ev_fork) (void)hipEventDestroy(H->ev_fork);
    if (H->ev_join) (void)hipEventDestroy(H->ev_join);
    if (H->ev_leafk) (void)hipEventDestroy(H->ev_leafk);
    if (H->ev_done) (void)hipEventDestroy(H->ev_done);
    for (auto *lv : {&H->lev, &H->lev_o})
        for (auto &L : *lv) {
            if (!L.shares_tree) {
                void *ts[] = {L.key, L.coord, L.parent, L.child_first, L.child_count, L.nb_ptr, L.nb, L.il_ptr, L.il};
                for (void *p : ts) dfree(p);
            }
            void *ps[] = {L.first, L.count, L.m, L.tt_off, L.k, L.piv_ptr, L.piv_id, L.ipos, L.jid, L.rem_ptr,
                          L.rem_pos, L.crem_off, L.crem64, L.crem_t, L.piv_cell, L.rem_cell, L.pc64, L.pc32,
                          L.ilpre, L.ilsum, L.w64, L.u64, L.hcell, L.own_ptr, L.own_il, L.own_pre, L.own_sum,
                          L.own_slot, L.non_ptr, L.non_slot, L.sym_order, L.m2l_order, L.col64};   // col32 aliases col64
            for (void *p : ps) dfree(p);
        }
    void *ps[] = {H->pts64,    H->order,    H->keys,     H->nbpre,    H->nbsum,     H->xs64,
                  H->far64,    H->xhi,      H->xlo,      H->m2l_part, H->pown_ptr,  H->pown_nb,
                  H->pown_pre, H->pown_sum, H->pown_slot, H->pnon_ptr, H->pnon_slot, H->pcell,
                  H->pcol_hi,  H->pcol_lo,  H->prow,     H->near64,   H->rank,      H->qpts64,
                  H->qorder,   H->qrank,    H->nbpre_o,  H->nbsum_o};
    for (void *p : ps) dfree(p);
    delete H;
}

static bool uses_length_scale(int32_t kind)
{
    return kind == NNCA_K_GAUSS || kind == NNCA_K_LOG_REG || kind == NNCA_K_INV_REG || kind == NNCA_K_EXP_R;
}

static void check_kernel(int32_t kind, int32_t dim, double hparam)
{
    if (kind != NNCA_K_LOG_R && kind != NNCA_K_INV_R && kind != NNCA_K_GAUSS && kind != NNCA_K_LOG_REG &&
        kind != NNCA_K_INV_REG && kind != NNCA_K_EXP_R)
        fail(NNCA_ERR_INVALID_ARG, "unknown kernel kind");
    if ((kind == NNCA_K_LOG_R || kind == NNCA_K_LOG_REG) && dim != 2)
        fail(NNCA_ERR_NOT_SUPPORTED, "log kernels are provided in 2D only");
    if (uses_length_scale(kind) && !(hparam > 0.0 && std::isfinite(hparam)))
        fail(NNCA_ERR_INVALID_ARG, "the kernel's length scale must be positive and finite");
    if ((kind == NNCA_K_LOG_REG) && !(hparam < 1.0))
        fail(NNCA_ERR_INVALID_ARG, "the regularised log kernel needs a < 1 (log a must be negative)");
}

static const Level &level_of(nnca_handle h, int32_t level)
{
    if (!h) fail(NNCA_ERR_INVALID_ARG, "handle is NULL");
    if (level < 0 || level > h->kappa) fail(NNCA_ERR_INVALID_ARG, "level out of range");
    return h->lev[level];
}

template <typename S, typename D>
static void d2h_convert(const S *dev, int64_t cnt, D *host)
{
    std::vector<S> tmp(cnt > 0 ? cnt : 1);
    if (cnt > 0) HIPCHECK(hipMemcpy(tmp.data(), dev, sizeof(S) * cnt, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < cnt; i++) host[i] = (D)tmp[i];
}

// Checks shared by the matvec entry points (nnca_matvec, its adjoint and the
// allocation-free variant).
void nnca::check_matvec_args(nnca_handle h, const void *X, const void *Y, int64_t nrhs, int64_t ldx, int64_t ldy,
                             int32_t dtype, int32_t precision, bool adjoint)
{
    if (!h) fail(NNCA_ERR_INVALID_ARG, "handle is NULL");
    if (!X || !Y) fail(NNCA_ERR_INVALID_ARG, "X or Y is NULL");
    if (nrhs < 1) fail(NNCA_ERR_INVALID_ARG, "nrhs < 1");
    // rows of X and Y: n for P = Q; for P != Q the product maps Q to P and
    // its transpose P to Q
    const int64_t nx = h->general ? (adjoint ? h->n : h->nq) : h->n;
    const int64_t ny = h->general ? (adjoint ? h->nq : h->n) : h->n;
    if (ldx < nx || ldy < ny) fail(NNCA_ERR_INVALID_ARG, "leading dimension < rows");
    if (dtype != NNCA_F32 && dtype != NNCA_F64) fail(NNCA_ERR_INVALID_ARG, "bad dtype");
    if (precision != NNCA_PREC_FP64 && precision != NNCA_PREC_MIXED) fail(NNCA_ERR_INVALID_ARG, "bad precision");
    const int64_t es = dtype == NNCA_F32 ? 4 : 8;
    const char *xb = (const char *)X, *xe = xb + ((nrhs - 1) * ldx + nx) * es;
    const char *yb = (const char *)Y, *ye = yb + ((nrhs - 1) * ldy + ny) * es;
    if (xb < ye && yb < xe) fail(NNCA_ERR_INVALID_ARG, "X and Y overlap");
}

// entry points that cover the symmetric case only
static void require_square(nnca_handle h, const char *what)
{
    if (h && h->general) fail(NNCA_ERR_NOT_SUPPORTED, std::string(what) + " covers P = Q only (a handle of nnca_build)");
}

// dense m x k operator C of one cell (the identity rows at the pivots)
static void export_operator(const Level &L, int64_t cell, double *C, int64_t cap, int64_t *m, int64_t *k)
{
    {
        if (cell < 0 || cell >= L.ncell) fail(NNCA_ERR_INVALID_ARG, "cell out of range");
        int64_t mm = L.h_m[cell], kk = L.h_k[cell];
        if (m) *m = mm;
        if (k) *k = kk;
        if (!C) return;
        if (cap < mm * kk) fail(NNCA_ERR_INVALID_ARG, "C too small");
        int32_t pp[2], rp[2];
        int64_t co[2];
        HIPCHECK(hipMemcpy(pp, L.piv_ptr + cell, sizeof(pp), hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(rp, L.rem_ptr + cell, sizeof(rp), hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(co, L.crem_off + cell, sizeof(co), hipMemcpyDeviceToHost));
        std::vector<int32_t> ip(kk > 0 ? kk : 1), rpos(rp[1] - rp[0] > 0 ? rp[1] - rp[0] : 1);
        std::vector<double> cr(co[1] - co[0] > 0 ? co[1] - co[0] : 1);
        if (kk) HIPCHECK(hipMemcpy(ip.data(), L.ipos + pp[0], sizeof(int32_t) * kk, hipMemcpyDeviceToHost));
        if (rp[1] > rp[0])
            HIPCHECK(hipMemcpy(rpos.data(), L.rem_pos + rp[0], sizeof(int32_t) * (rp[1] - rp[0]), hipMemcpyDeviceToHost));
        if (co[1] > co[0])
            HIPCHECK(hipMemcpy(cr.data(), L.crem64 + co[0], sizeof(double) * (co[1] - co[0]), hipMemcpyDeviceToHost));
        std::memset(C, 0, sizeof(double) * mm * kk);
        for (int64_t q = 0; q < kk; q++) C[(int64_t)ip[q] * kk + q] = 1.0;
        for (int64_t r = 0; r < rp[1] - rp[0]; r++)
            for (int64_t q = 0; q < kk; q++) C[(int64_t)rpos[r] * kk + q] = cr[r * kk + q];
    }
}

// the level of one half: 0 incoming, 1 outgoing (the same level when P = Q)
static const Level &half_level(nnca_handle h, int32_t level, int32_t half)
{
    const Level &L = level_of(h, level);
    if (half != 0 && half != 1) fail(NNCA_ERR_INVALID_ARG, "half must be 0 or 1");
    if (!L.has_piv) fail(NNCA_ERR_INVALID_ARG, "level carries no pivots");
    return half == 1 && h->general ? h->lev_o[level] : L;
}

// Calls on one handle share its workspace: each waits for the end of the
// previous one (recorded on that call's stream), whatever stream it names.
void nnca::order_call_begin(nnca_handle h, hipStream_t s) { HIPCHECK(hipStreamWaitEvent(s, h->ev_done, 0)); }
void nnca::order_call_end(nnca_handle h, hipStream_t s) { HIPCHECK(hipEventRecord(h->ev_done, s)); }

extern "C" {

// A handle with its options set, not yet built: checks every argument that
// is not a point array.
static nnca_h2 *new_handle(int64_t n, int32_t dim, int32_t kernel_kind, double length_scale, double tol,
                           int32_t leaf_size, const nnca_build_options *opts, void *stream)
{
    if (dim != 2 && dim != 3) fail(NNCA_ERR_INVALID_ARG, "dim must be 2 or 3");
    if (leaf_size < 1) fail(NNCA_ERR_INVALID_ARG, "leaf_size < 1");
    if (!(tol >= 0.0) || !std::isfinite(tol)) fail(NNCA_ERR_INVALID_ARG, "tol must be finite and >= 0");
    check_kernel(kernel_kind, dim, length_scale);
    nnca_build_options o{};
    o.struct_size = sizeof(o);
    o.exhausted_policy = 1;
    if (opts) {
        // callers built against the first version of the struct end at
        // `reserved`; the fields after it keep their defaults
        const size_t v1 = offsetof(nnca_build_options, max_rhs);
        if (opts->struct_size != v1 && opts->struct_size < sizeof(nnca_build_options))
            fail(NNCA_ERR_INVALID_ARG, "bad struct_size");
        std::memcpy(&o, opts, opts->struct_size < sizeof(o) ? opts->struct_size : sizeof(o));
        o.struct_size = sizeof(o);
    }
    if ((o.alloc == nullptr) != (o.free == nullptr))
        fail(NNCA_ERR_INVALID_ARG, "alloc and free must both be set or both be NULL");
    if (o.max_rhs < 0) fail(NNCA_ERR_INVALID_ARG, "max_rhs < 0");
    if ((o.eta2_num == 0) != (o.eta2_den == 0) || o.eta2_num < 0 || o.eta2_den < 0)
        fail(NNCA_ERR_INVALID_ARG, "eta2 must be a positive fraction or 0/0");
    if (o.exhausted_policy != 0 && o.exhausted_policy != 1) fail(NNCA_ERR_INVALID_ARG, "bad exhausted_policy");
    if (o.rank_reserve < 0) fail(NNCA_ERR_INVALID_ARG, "rank_reserve < 0");
    nnca_h2 *H = new nnca_h2();
    H->n = n;
    H->dim = dim;
    H->kind = kernel_kind;
    H->hparam = uses_length_scale(kernel_kind) ? length_scale : 1.0;
    H->tol = tol;
    H->leaf = leaf_size;
    H->eta_num = o.eta2_num ? o.eta2_num : dim;
    H->eta_den = o.eta2_num ? o.eta2_den : 1;
    H->policy = o.exhausted_policy;
    H->ws_budget = o.workspace_bytes;
    H->rank_reserve = o.rank_reserve > 0 ? o.rank_reserve : 256;
    H->stream = (hipStream_t)stream;
    H->alloc.alloc = o.alloc;
    H->alloc.free = o.free;
    H->alloc.ctx = o.alloc_ctx;
    H->max_rhs = o.max_rhs == 0 ? 16 : (o.max_rhs > 64 ? 64 : o.max_rhs);
    return H;
}

nnca_status nnca_build(const double *points, int64_t n, int32_t dim, int64_t ld, int32_t points_on_device,
                       int32_t kernel_kind, double length_scale, double tol, int32_t leaf_size,
                       const nnca_build_options *opts, void *stream, nnca_handle *out)
{
    return guarded([&] {
        if (!out) fail(NNCA_ERR_INVALID_ARG, "out is NULL");
        if (!points) fail(NNCA_ERR_INVALID_ARG, "points is NULL");
        if (n < 1 || n > (int64_t)INT32_MAX / 2) fail(NNCA_ERR_INVALID_ARG, "n out of range");
        if (ld < n) fail(NNCA_ERR_INVALID_ARG, "ld < n");
        auto t0 = std::chrono::steady_clock::now();
        nnca_h2 *H = new_handle(n, dim, kernel_kind, length_scale, tol, leaf_size, opts, stream);
        AllocScope as(H->alloc);
        try {
            double *pin = nullptr;
            int64_t pld = ld;
            if (points_on_device) {
                pin = const_cast<double *>(points);
            } else {
                pin = dalloc<double>((size_t)dim * n);
                HIPCHECK(hipMemcpy2DAsync(pin, sizeof(double) * n, points, sizeof(double) * ld, sizeof(double) * n,
                                          dim, hipMemcpyHostToDevice, H->stream));
                pld = n;
            }
            try {
                build_tree(H, pin, pld);
            } catch (...) {
                if (!points_on_device) dfree(pin);
                throw;
            }
            if (!points_on_device) {
                HIPCHECK(hipStreamSynchronize(H->stream));
                dfree(pin);
            }
            {
                HIPCHECK(hipStreamSynchronize(H->stream));
                const auto ta = std::chrono::steady_clock::now();
                build_pivots(H);
                HIPCHECK(hipStreamSynchronize(H->stream));
                H->aca_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - ta).count();
            }
            prepare_apply(H);
            HIPCHECK(hipEventCreateWithFlags(&H->ev_done, hipEventDisableTiming));
            HIPCHECK(hipStreamSynchronize(H->stream));
        } catch (...) {
            (void)hipStreamSynchronize(H->stream);
            destroy_handle(H);
            throw;
        }
        H->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = H;
    });
}

nnca_status nnca_build_general(const double *targets, int64_t np, int64_t ldp, const double *sources, int64_t nq,
                               int64_t ldq, int32_t dim, int32_t points_on_device, int32_t kernel_kind,
                               double length_scale, double tol, int32_t leaf_size, const nnca_build_options *opts,
                               void *stream, nnca_handle *out)
{
    return guarded([&] {
        if (!out) fail(NNCA_ERR_INVALID_ARG, "out is NULL");
        if (!targets || !sources) fail(NNCA_ERR_INVALID_ARG, "targets or sources is NULL");
        if (np < 1 || nq < 1 || np + nq > (int64_t)INT32_MAX / 2) fail(NNCA_ERR_INVALID_ARG, "np or nq out of range");
        if (ldp < np || ldq < nq) fail(NNCA_ERR_INVALID_ARG, "leading dimension < point count");
        auto t0 = std::chrono::steady_clock::now();
        const int64_t n = np + nq;
        nnca_h2 *H = new_handle(n, dim, kernel_kind, length_scale, tol, leaf_size, opts, stream);
        AllocScope as(H->alloc);
        try {
            // the union Z = [P, Q] as one dim x (np + nq) array on the device
            double *Z = dalloc<double>((size_t)dim * n);
            try {
                const hipMemcpyKind kd = points_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
                HIPCHECK(hipMemcpy2DAsync(Z, sizeof(double) * n, targets, sizeof(double) * ldp, sizeof(double) * np,
                                          dim, kd, H->stream));
                HIPCHECK(hipMemcpy2DAsync(Z + np, sizeof(double) * n, sources, sizeof(double) * ldq,
                                          sizeof(double) * nq, dim, kd, H->stream));
                build_tree(H, Z, n, np);
                split_general(H, Z, n, np);
            } catch (...) {
                (void)hipStreamSynchronize(H->stream);
                dfree(Z);
                throw;
            }
            HIPCHECK(hipStreamSynchronize(H->stream));
            dfree(Z);
            {
                HIPCHECK(hipStreamSynchronize(H->stream));
                const auto ta = std::chrono::steady_clock::now();
                build_pivots(H);
                HIPCHECK(hipStreamSynchronize(H->stream));
                H->aca_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - ta).count();
            }
            prepare_general(H);
            HIPCHECK(hipEventCreateWithFlags(&H->ev_done, hipEventDisableTiming));
            HIPCHECK(hipStreamSynchronize(H->stream));
        } catch (...) {
            (void)hipStreamSynchronize(H->stream);
            destroy_handle(H);
            throw;
        }
        H->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = H;
    });
}

static nnca_status matvec_common(nnca_handle h, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy,
                                 int32_t dtype, int32_t precision, bool adjoint, void *stream)
{
    return guarded([&] {
        check_matvec_args(h, X, Y, nrhs, ldx, ldy, dtype, precision, adjoint);
        AllocScope as(h->alloc);
        const hipStream_t s = (hipStream_t)stream;
        order_call_begin(h, s);
        if (h->general) run_matvec_general(h, X, Y, nrhs, ldx, ldy, dtype, precision, adjoint, s);
        else run_matvec(h, X, Y, nrhs, ldx, ldy, dtype, precision, s);
        order_call_end(h, s);
    });
}

nnca_status nnca_matvec(nnca_handle h, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy,
                        int32_t dtype, int32_t precision, void *stream)
{
    return matvec_common(h, X, Y, nrhs, ldx, ldy, dtype, precision, false, stream);
}

// In the symmetric case of Sec. 5 (P = Q, K(x,y) = K(y,x), V_B = U_B,
// T_{B B_c} = C_{B_c B}^T) the transposed passes coincide with the forward
// ones: P2M^T = L2P, M2M^T = L2L, and every block S_{B,B'}^T = S_{B',B} with
// B' in IL(B) <=> B in IL(B'), near blocks likewise.  The adjoint therefore
// runs the same kernels.  In the general case it runs them with the two
// halves exchanged.
nnca_status nnca_matvec_adjoint(nnca_handle h, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy,
                                int32_t dtype, int32_t precision, void *stream)
{
    return matvec_common(h, X, Y, nrhs, ldx, ldy, dtype, precision, true, stream);
}

nnca_status nnca_set_apply_flags(nnca_handle h, int32_t flags)
{
    return guarded([&] {
        if (!h) fail(NNCA_ERR_INVALID_ARG, "handle is NULL");
        if (flags & ~NNCA_APPLY_NO_SYMMETRIC) fail(NNCA_ERR_INVALID_ARG, "unknown apply flags");
        h->apply_flags = flags;
    });
}

nnca_status nnca_matvec_backward(nnca_handle h, const double *X, const double *G, int64_t nrhs, int64_t ldx,
                                 int64_t ldg, int32_t precision, double *DX, int64_t lddx, double *dLdh,
                                 void *stream)
{
    return guarded([&] {
        if (!h) fail(NNCA_ERR_INVALID_ARG, "handle is NULL");
        require_square(h, "nnca_matvec_backward");
        if (!G) fail(NNCA_ERR_INVALID_ARG, "G is NULL");
        if (!DX && !dLdh) fail(NNCA_ERR_INVALID_ARG, "neither DX nor dLdh requested");
        if (dLdh && !X) fail(NNCA_ERR_INVALID_ARG, "X is NULL");
        if (nrhs < 1) fail(NNCA_ERR_INVALID_ARG, "nrhs < 1");
        if (ldg < h->n || (X && ldx < h->n) || (DX && lddx < h->n))
            fail(NNCA_ERR_INVALID_ARG, "leading dimension < n");
        if (precision != NNCA_PREC_FP64 && precision != NNCA_PREC_MIXED) fail(NNCA_ERR_INVALID_ARG, "bad precision");
        if (dLdh && h->kind != NNCA_K_GAUSS)
            fail(NNCA_ERR_NOT_SUPPORTED, "the length-scale derivative is defined for the Gaussian kernel only");
        auto span = [&](const double *p, int64_t ld) {
            return std::make_pair((const char *)p, (const char *)(p + (nrhs - 1) * ld + h->n));
        };
        if (DX) {
            auto d = span(DX, lddx), g = span(G, ldg);
            if (d.first < g.second && g.first < d.second) fail(NNCA_ERR_INVALID_ARG, "DX and G overlap");
            if (X) {
                auto x = span(X, ldx);
                if (d.first < x.second && x.first < d.second) fail(NNCA_ERR_INVALID_ARG, "DX and X overlap");
            }
            if (dLdh) {
                const char *q = (const char *)dLdh;
                if (d.first < q + sizeof(double) && q < d.second) fail(NNCA_ERR_INVALID_ARG, "DX and dLdh overlap");
            }
        }
        AllocScope as(h->alloc);
        const hipStream_t s = (hipStream_t)stream;
        order_call_begin(h, s);
        run_backward(h, X, G, nrhs, ldx, ldg, precision, DX, lddx, dLdh, s);
        order_call_end(h, s);
    });
}

nnca_status nnca_batch_create(const nnca_handle *handles, int32_t count, int32_t flags, nnca_batch_handle *out)
{
    return guarded([&] {
        if (!handles || !out) fail(NNCA_ERR_INVALID_ARG, "NULL argument");
        if (count < 1) fail(NNCA_ERR_INVALID_ARG, "count < 1");
        if (flags & ~(NNCA_BATCH_GRAPH | NNCA_BATCH_AUTOTUNE)) fail(NNCA_ERR_INVALID_ARG, "unknown flags");
        for (int32_t b = 0; b < count; b++) {
            if (!handles[b]) fail(NNCA_ERR_INVALID_ARG, "a handle is NULL");
            require_square(handles[b], "nnca_batch_create");
        }
        AllocScope as(handles[0]->alloc);
        *out = create_batch(handles, count, flags);
    });
}

nnca_status nnca_batch_query(nnca_batch_handle b, int32_t *count, int64_t *rows, int64_t *offsets)
{
    return guarded([&] {
        if (!b) fail(NNCA_ERR_INVALID_ARG, "batch is NULL");
        if (count) *count = batch_count(b);
        if (rows) *rows = batch_rows(b);
        if (offsets) std::memcpy(offsets, batch_offsets(b), sizeof(int64_t) * (batch_count(b) + 1));
    });
}

nnca_status nnca_batch_matvec(nnca_batch_handle b, const double *X, double *Y, int64_t nrhs, int64_t ldx,
                              int64_t ldy, int32_t precision, void *stream)
{
    return guarded([&] {
        if (!b) fail(NNCA_ERR_INVALID_ARG, "batch is NULL");
        if (!X || !Y) fail(NNCA_ERR_INVALID_ARG, "X or Y is NULL");
        if (nrhs < 1) fail(NNCA_ERR_INVALID_ARG, "nrhs < 1");
        const int64_t n = batch_rows(b);
        if (ldx < n || ldy < n) fail(NNCA_ERR_INVALID_ARG, "leading dimension < total rows");
        if (precision != NNCA_PREC_FP64 && precision != NNCA_PREC_MIXED) fail(NNCA_ERR_INVALID_ARG, "bad precision");
        const char *xb = (const char *)X, *xe = (const char *)(X + (nrhs - 1) * ldx + n);
        const char *yb = (const char *)Y, *ye = (const char *)(Y + (nrhs - 1) * ldy + n);
        if (xb < ye && yb < xe) fail(NNCA_ERR_INVALID_ARG, "X and Y overlap");
        AllocScope as(*batch_allocator(b));
        run_batch(b, X, Y, nrhs, ldx, ldy, precision, (hipStream_t)stream);
    });
}

nnca_status nnca_batch_destroy(nnca_batch_handle b)
{
    return guarded([&] {
        if (!b) return;
        const Allocator a = *batch_allocator(b);
        AllocScope as(a);
        destroy_batch(b);
    });
}

nnca_status nnca_direct(const double *points, int64_t n, int32_t dim, int64_t ld, int32_t kernel_kind,
                        double length_scale, const double *X, double *Y, int64_t nrhs, int64_t ldx, int64_t ldy,
                        void *stream)
{
    return guarded([&] {
        if (!points || !X || !Y) fail(NNCA_ERR_INVALID_ARG, "NULL pointer");
        if (n < 1 || (dim != 2 && dim != 3) || ld < n || nrhs < 1 || ldx < n || ldy < n)
            fail(NNCA_ERR_INVALID_ARG, "bad size");
        check_kernel(kernel_kind, dim, length_scale);
        run_direct(points, n, dim, ld, kernel_kind, uses_length_scale(kernel_kind) ? length_scale : 1.0, X, Y, nrhs,
                   ldx, ldy, (hipStream_t)stream);
    });
}

nnca_status nnca_query(nnca_handle h, nnca_info *info)
{
    return guarded([&] {
        if (!h || !info) fail(NNCA_ERR_INVALID_ARG, "NULL argument");
        std::memset(info, 0, sizeof(*info));
        info->n = h->n;
        info->dim = h->dim;
        info->kappa = h->kappa;
        info->lmin = h->lmin;
        info->leaf_size = h->leaf;
        info->kernel_kind = h->kind;
        info->length_scale = h->hparam;
        info->tol = h->tol;
        for (int q = 0; q < 3; q++) info->lo[q] = h->lo[q];
        info->side = h->L;
        for (int l = 0; l <= h->kappa && l < NNCA_MAX_LEVELS; l++) {
            const Level &L = h->lev[l];
            info->ncell[l] = L.ncell;
            info->npiv[l] = L.has_piv ? L.npiv : 0;
            info->nlist[l][0] = L.nnb;
            info->nlist[l][1] = L.nil;
            info->max_rank[l] = L.has_piv ? L.max_k : 0;
            info->m2l_level[l] = L.has_piv ? L.m2l_inter : 0;
        }
        info->transfer_entries = h->transfer_entries;
        info->m2l_interactions = h->m2l_inter;
        info->p2p_interactions = h->p2p_inter;
        info->build_seconds = h->build_seconds;
        info->mixed_fp32_levels = h->fp32_levels;
        info->mixed_near_symmetric = h->p2p_sym ? 1 : 0;
    });
}

nnca_status nnca_query_build(nnca_handle h, double *out, int32_t count)
{
    return guarded([&] {
        if (!h || !out || count < 1) fail(NNCA_ERR_INVALID_ARG, "NULL argument or count < 1");
        const double v[3] = {h->build_seconds, h->aca_seconds, h->aca_panel_bytes};
        for (int32_t q = 0; q < count && q < 3; q++) out[q] = v[q];
    });
}

nnca_status nnca_query_shape(nnca_handle h, int64_t *rows, int64_t *cols, int32_t *general)
{
    return guarded([&] {
        if (!h) fail(NNCA_ERR_INVALID_ARG, "handle is NULL");
        if (rows) *rows = h->n;
        if (cols) *cols = h->general ? h->nq : h->n;
        if (general) *general = h->general ? 1 : 0;
    });
}

nnca_status nnca_export_half(nnca_handle h, int32_t level, int32_t half, int64_t *ptr, int64_t *rows,
                             int64_t *cols)
{
    return guarded([&] {
        const Level &L = half_level(h, level, half);
        // rows index the half's own set, columns the other set
        const bool q_rows = h->general && half == 1, q_cols = h->general && half == 0;
        auto order_of = [&](bool q) {
            std::vector<int32_t> o(q ? h->nq : h->n);
            HIPCHECK(hipMemcpy(o.data(), q ? h->qorder : h->order, sizeof(int32_t) * o.size(), hipMemcpyDeviceToHost));
            return o;
        };
        if (ptr) d2h_convert(L.piv_ptr, L.ncell + 1, ptr);
        std::vector<int32_t> tmp(L.npiv > 0 ? L.npiv : 1);
        if (rows) {
            const std::vector<int32_t> o = order_of(q_rows);
            if (L.npiv) HIPCHECK(hipMemcpy(tmp.data(), L.piv_id, sizeof(int32_t) * L.npiv, hipMemcpyDeviceToHost));
            for (int64_t q = 0; q < L.npiv; q++) rows[q] = o[tmp[q]];
        }
        if (cols) {
            const std::vector<int32_t> o = order_of(q_cols);
            if (L.npiv) HIPCHECK(hipMemcpy(tmp.data(), L.jid, sizeof(int32_t) * L.npiv, hipMemcpyDeviceToHost));
            for (int64_t q = 0; q < L.npiv; q++) cols[q] = tmp[q] < 0 ? -1 : o[tmp[q]];
        }
    });
}

nnca_status nnca_export_order(nnca_handle h, int64_t *order)
{
    return guarded([&] {
        if (!h || !order) fail(NNCA_ERR_INVALID_ARG, "NULL argument");
        d2h_convert(h->order, h->n, order);
    });
}

nnca_status nnca_export_cells(nnca_handle h, int32_t level, uint64_t *key, int64_t *first, int64_t *count)
{
    return guarded([&] {
        const Level &L = level_of(h, level);
        if (key) HIPCHECK(hipMemcpy(key, L.key, sizeof(uint64_t) * L.ncell, hipMemcpyDeviceToHost));
        if (first) d2h_convert(L.first, L.ncell, first);
        if (count) d2h_convert(L.count, L.ncell, count);
    });
}

nnca_status nnca_export_lists(nnca_handle h, int32_t level, int32_t which, int64_t *ptr, int64_t *idx)
{
    return guarded([&] {
        const Level &L = level_of(h, level);
        if (which != 0 && which != 1) fail(NNCA_ERR_INVALID_ARG, "which must be 0 or 1");
        if (!ptr || !idx) fail(NNCA_ERR_INVALID_ARG, "NULL argument");
        d2h_convert(which ? L.il_ptr : L.nb_ptr, L.ncell + 1, ptr);
        d2h_convert(which ? L.il : L.nb, which ? L.nil : L.nnb, idx);
    });
}

nnca_status nnca_export_pivots(nnca_handle h, int32_t level, int64_t *ptr, int64_t *rows, int64_t *cols)
{
    return guarded([&] {
        const Level &L = level_of(h, level);
        if (!L.has_piv) fail(NNCA_ERR_INVALID_ARG, "level carries no pivots");
        std::vector<int32_t> order(h->n);
        HIPCHECK(hipMemcpy(order.data(), h->order, sizeof(int32_t) * h->n, hipMemcpyDeviceToHost));
        if (ptr) d2h_convert(L.piv_ptr, L.ncell + 1, ptr);
        std::vector<int32_t> tmp(L.npiv > 0 ? L.npiv : 1);
        if (rows) {
            if (L.npiv) HIPCHECK(hipMemcpy(tmp.data(), L.piv_id, sizeof(int32_t) * L.npiv, hipMemcpyDeviceToHost));
            for (int64_t q = 0; q < L.npiv; q++) rows[q] = order[tmp[q]];
        }
        if (cols) {
            if (L.npiv) HIPCHECK(hipMemcpy(tmp.data(), L.jid, sizeof(int32_t) * L.npiv, hipMemcpyDeviceToHost));
            for (int64_t q = 0; q < L.npiv; q++) cols[q] = tmp[q] < 0 ? -1 : order[tmp[q]];
        }
    });
}

nnca_status nnca_export_operator(nnca_handle h, int32_t level, int64_t cell, double *C, int64_t cap, int64_t *m,
                                 int64_t *k)
{
    return guarded([&] {
        const Level &L = level_of(h, level);
        if (!L.has_piv) fail(NNCA_ERR_INVALID_ARG, "level carries no pivots");
        export_operator(L, cell, C, cap, m, k);
    });
}

nnca_status nnca_export_half_operator(nnca_handle h, int32_t level, int32_t half, int64_t cell, double *C,
                                      int64_t cap, int64_t *m, int64_t *k)
{
    return guarded([&] { export_operator(half_level(h, level, half), cell, C, cap, m, k); });
}

nnca_status nnca_debug_kernel_eval(int32_t kernel_kind, double length_scale, int32_t dim, const double *a,
                                   const double *b, int64_t count, double *out)
{
    return guarded([&] {
        if (!a || !b || !out || count < 1 || (dim != 2 && dim != 3)) fail(NNCA_ERR_INVALID_ARG, "bad argument");
        check_kernel(kernel_kind, dim, length_scale);
        debug_kernel_eval(kernel_kind, uses_length_scale(kernel_kind) ? length_scale : 1.0, dim, a, b, count, out,
                          nullptr);
    });
}

nnca_status nnca_gmres(nnca_handle h, double alpha, double beta, const double *F, double *X, double tol,
                       int32_t max_iter, int32_t restart, int32_t precision, int32_t *iters, double *relres,
                       void *stream)
{
    return guarded([&] {
        if (!h) fail(NNCA_ERR_INVALID_ARG, "handle is NULL");
        require_square(h, "nnca_gmres");
        if (!F || !X) fail(NNCA_ERR_INVALID_ARG, "F or X is NULL");
        if (F == X) fail(NNCA_ERR_INVALID_ARG, "F and X are the same buffer");
        {
            const char *fb = (const char *)F, *fe = fb + sizeof(double) * h->n;
            const char *xb = (const char *)X, *xe = xb + sizeof(double) * h->n;
            if (fb < xe && xb < fe) fail(NNCA_ERR_INVALID_ARG, "F and X overlap");
        }
        if (!(tol >= 0.0) || !std::isfinite(alpha) || !std::isfinite(beta))
            fail(NNCA_ERR_INVALID_ARG, "tol must be >= 0 and alpha, beta finite");
        if (max_iter < 0 || restart < 1 || restart > 1000) fail(NNCA_ERR_INVALID_ARG, "bad max_iter or restart");
        if (precision != NNCA_PREC_FP64 && precision != NNCA_PREC_MIXED) fail(NNCA_ERR_INVALID_ARG, "bad precision");
        AllocScope as(h->alloc);
        const hipStream_t s = (hipStream_t)stream;
        order_call_begin(h, s);
        run_gmres(h, alpha, beta, F, X, tol, max_iter, restart, precision, iters, relres, s);
        order_call_end(h, s);
    });
}

static void no_overlap(const double *a, int64_t na, const double *b, int64_t nb, const char *what)
{
    const char *ab = (const char *)a, *ae = ab + sizeof(double) * na;
    const char *bb = (const char *)b, *be = bb + sizeof(double) * nb;
    if (ab < be && bb < ae) fail(NNCA_ERR_INVALID_ARG, what);
}

nnca_status nnca_svm_train(nnca_handle h, const double *y, double *alpha, double lambda, double beta, double eta,
                           double tol, int32_t max_iter, int32_t precision, int32_t *iters, double *bias,
                           double *eta_used, void *stream)
{
    return guarded([&] {
        if (!h) fail(NNCA_ERR_INVALID_ARG, "handle is NULL");
        require_square(h, "nnca_svm_train");
        if (!y || !alpha) fail(NNCA_ERR_INVALID_ARG, "y or alpha is NULL");
        no_overlap(y, h->n, alpha, h->n, "y and alpha overlap");
        if (!(lambda > 0.0) || !std::isfinite(lambda)) fail(NNCA_ERR_INVALID_ARG, "lambda must be finite and > 0");
        if (!(beta >= 0.0) || !std::isfinite(beta)) fail(NNCA_ERR_INVALID_ARG, "beta must be finite and >= 0");
        if (!std::isfinite(eta) || !(tol >= 0.0)) fail(NNCA_ERR_INVALID_ARG, "eta must be finite and tol >= 0");
        if (max_iter < 0) fail(NNCA_ERR_INVALID_ARG, "max_iter < 0");
        if (precision != NNCA_PREC_FP64 && precision != NNCA_PREC_MIXED) fail(NNCA_ERR_INVALID_ARG, "bad precision");
        AllocScope as(h->alloc);
        const hipStream_t s = (hipStream_t)stream;
        order_call_begin(h, s);
        run_svm_train(h, y, alpha, lambda, beta, eta, tol, max_iter, precision, iters, bias, eta_used, s);
        order_call_end(h, s);
    });
}

nnca_status nnca_svm_decision(nnca_handle h, const double *y, const double *alpha, double bias, double *f,
                              int32_t precision, void *stream)
{
    return guarded([&] {
        if (!h) fail(NNCA_ERR_INVALID_ARG, "handle is NULL");
        if (!y || !alpha || !f) fail(NNCA_ERR_INVALID_ARG, "y, alpha or f is NULL");
        const int64_t nq = h->general ? h->nq : h->n, np = h->n;
        no_overlap(f, np, y, nq, "f and y overlap");
        no_overlap(f, np, alpha, nq, "f and alpha overlap");
        if (!std::isfinite(bias)) fail(NNCA_ERR_INVALID_ARG, "bias must be finite");
        if (precision != NNCA_PREC_FP64 && precision != NNCA_PREC_MIXED) fail(NNCA_ERR_INVALID_ARG, "bad precision");
        AllocScope as(h->alloc);
        const hipStream_t s = (hipStream_t)stream;
        order_call_begin(h, s);
        run_svm_decision(h, y, alpha, bias, f, precision, s);
        order_call_end(h, s);
    });
}

nnca_status nnca_probe_rates(double *out, int32_t count, void *stream)
{
    return guarded([&] {
        if (!out || count < 1) fail(NNCA_ERR_INVALID_ARG, "out is NULL or count < 1");
        probe_rates(out, count, (hipStream_t)stream);
    });
}

nnca_status nnca_profile_enable(nnca_handle h, int32_t enable)
{
    return guarded([&] {
        if (!h) fail(NNCA_ERR_INVALID_ARG, "handle is NULL");
        HIPCHECK(hipStreamSynchronize(h->stream));
        clear_profile(h);
        h->prof_mask = enable;
    });
}

nnca_status nnca_profile_read(nnca_handle h, int64_t *count, int32_t *pass, int32_t *level, double *ms, int64_t cap)
{
    return guarded([&] {
        if (!h || !count) fail(NNCA_ERR_INVALID_ARG, "NULL argument");
        int64_t nrec = (int64_t)h->prof.size();
        for (int64_t q = 0; q < nrec && q < cap; q++) {
            auto &r = h->prof[q];
            HIPCHECK(hipEventSynchronize(r.b));
            float t = 0.f;
            HIPCHECK(hipEventElapsedTime(&t, r.a, r.b));
            if (pass) pass[q] = r.pass;
            if (level) level[q] = r.level;
            if (ms) ms[q] = t;
        }
        *count = nrec;
        clear_profile(h);
    });
}

nnca_status nnca_destroy(nnca_handle h)
{
    return guarded([&] {
        if (h) {
            (void)hipStreamSynchronize(h->stream);
            if (h->ev_done) (void)hipEventSynchronize(h->ev_done);
            const Allocator a = h->alloc;
            AllocScope as(a);
            destroy_handle(h);
        }
    });
}

const char *nnca_status_string(nnca_status s)
{
    switch (s) {
    case NNCA_OK: return "ok";
    case NNCA_ERR_INVALID_ARG: return "invalid argument";
    case NNCA_ERR_OUT_OF_MEMORY: return "out of memory";
    case NNCA_ERR_HIP: return "HIP error";
    case NNCA_ERR_NOT_SUPPORTED: return "not supported";
    case NNCA_ERR_NUMERICAL: return "numerical failure";
    case NNCA_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char *nnca_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
