// Uneven batch: many independent problems applied by one set of launches.
//
// The handles' apply data are merged into one forest handle.  Tree levels are
// aligned by their distance from the leaves: slot s of the forest holds level
// kappa_b - s of every problem b that has pivots there, so the upward pass
// runs slot 0, 1, ... and the downward pass the reverse, each slot one launch
// over the cells of all problems, and the transverse and near-field passes
// (independent across cells) likewise.  Every cell, pivot, list entry, point
// and operator index is rebased into the concatenated arrays; problems never
// reference each other's cells, so the forest applies the block-diagonal
// operator diag(A~_1, ..., A~_B).  The cell side of the FP32 transverse
// shift is stored per cell.  The apply kernels are the single handle's.
//
// With graph mode on, the first call with a given set of arguments runs once
// eagerly (allocating workspaces and, with autotuning on, timing the split
// factors of every transverse-pass launch), then captures the whole matvec
// into a HIP graph on the batch's own stream; later calls with the same
// arguments replay the graph.
#include <algorithm>
#include <cstring>

#include "nnca_internal.h"

namespace nnca {

namespace {

__global__ void k_copy_add32(int64_t cnt, const int32_t *src, int32_t add, int32_t *dst, int keep_negative)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    int32_t v = src[i];
    dst[i] = (keep_negative && v < 0) ? v : v + add;
}

__global__ void k_copy_add64(int64_t cnt, const int64_t *src, int64_t add, int64_t *dst)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < cnt) dst[i] = src[i] + add;
}

__global__ void k_fill_f32(int64_t cnt, float v, float *dst)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < cnt) dst[i] = v;
}

struct Merger {
    hipStream_t s;
    void add32(int32_t *dst, const int32_t *src, int64_t cnt, int64_t add, bool keep_neg = false)
    {
        if (cnt <= 0) return;
        if (add > INT32_MAX || add < INT32_MIN) fail(NNCA_ERR_NOT_SUPPORTED, "batch exceeds 32-bit indices");
        k_copy_add32<<<grid_for(cnt, 256), 256, 0, s>>>(cnt, src, (int32_t)add, dst, keep_neg ? 1 : 0);
        HIPCHECK(hipGetLastError());
    }
    void add64(int64_t *dst, const int64_t *src, int64_t cnt, int64_t add)
    {
        if (cnt <= 0) return;
        k_copy_add64<<<grid_for(cnt, 256), 256, 0, s>>>(cnt, src, add, dst);
        HIPCHECK(hipGetLastError());
    }
    template <typename T>
    void copy(T *dst, const T *src, int64_t cnt)
    {
        if (cnt > 0) HIPCHECK(hipMemcpyAsync(dst, src, sizeof(T) * cnt, hipMemcpyDeviceToDevice, s));
    }
};

}  // namespace

}  // namespace nnca

struct nnca_batch {
    nnca_h2 *M = nullptr;
    int32_t count = 0;
    std::vector<int64_t> off;   // count + 1 row offsets of the problems
    hipStream_t gs = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    bool use_graph = false;
    struct Key {
        const double *X = nullptr;
        double *Y = nullptr;
        int64_t nrhs = 0, ldx = 0, ldy = 0;
        int32_t prec = -1;
        bool operator==(const Key &o) const
        {
            return X == o.X && Y == o.Y && nrhs == o.nrhs && ldx == o.ldx && ldy == o.ldy && prec == o.prec;
        }
    } key;
    bool have_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace nnca {

void destroy_batch(nnca_batch *B)
{
    if (!B) return;
    if (B->gs) (void)hipStreamSynchronize(B->gs);
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    if (B->M) destroy_handle(B->M);
    if (B->ev_in) (void)hipEventDestroy(B->ev_in);
    if (B->ev_out) (void)hipEventDestroy(B->ev_out);
    if (B->gs) (void)hipStreamDestroy(B->gs);
    delete B;
}

nnca_batch *create_batch(nnca_h2 *const *hs, int32_t count, int32_t flags)
{
    const nnca_h2 &H0 = *hs[0];
    for (int32_t b = 0; b < count; b++) {
        const nnca_h2 &H = *hs[b];
        if (H.dim != H0.dim || H.kind != H0.kind || H.hparam != H0.hparam)
            fail(NNCA_ERR_INVALID_ARG, "batched problems must share dimension, kernel and length scale");
        if (H.kappa < H.lmin)
            fail(NNCA_ERR_NOT_SUPPORTED, "a batched problem without a far field (all cells adjacent)");
    }
    nnca_batch *B = new nnca_batch();
    try {
        B->count = count;
        B->use_graph = (flags & NNCA_BATCH_GRAPH) != 0;
        HIPCHECK(hipStreamCreateWithFlags(&B->gs, hipStreamNonBlocking));
        HIPCHECK(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
        HIPCHECK(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
        hipStream_t s = B->gs;
        // the handles' own streams may still carry work
        for (int32_t b = 0; b < count; b++) HIPCHECK(hipStreamSynchronize(hs[b]->stream));

        nnca_h2 *M = new nnca_h2();
        B->M = M;
        M->dim = H0.dim;
        M->kind = H0.kind;
        M->hparam = H0.hparam;
        M->stream = s;
        M->autotune = (flags & NNCA_BATCH_AUTOTUNE) != 0;
        M->alloc = H0.alloc;   // the batch's memory comes from the first handle's allocator
        M->max_rhs = 1;
        for (int32_t b = 0; b < count; b++) M->max_rhs = std::max(M->max_rhs, hs[b]->max_rhs);
        B->off.assign(count + 1, 0);
        int S = 0;
        for (int32_t b = 0; b < count; b++) {
            B->off[b + 1] = B->off[b] + hs[b]->n;
            S = std::max(S, hs[b]->kappa - hs[b]->lmin + 1);
        }
        const int64_t N = B->off[count];
        if (N > INT32_MAX / 2) fail(NNCA_ERR_NOT_SUPPORTED, "batch exceeds 32-bit indices");
        M->n = N;
        M->kappa = S - 1;
        M->lmin = 0;
        M->lev.resize(S);
        Merger mg{s};

        // points, tree order, near-field prefixes
        M->pts64 = dalloc<double>(3 * N);
        M->order = dalloc<int32_t>(N);
        for (int32_t b = 0; b < count; b++) {
            const nnca_h2 &H = *hs[b];
            for (int q = 0; q < 3; q++) mg.copy(M->pts64 + q * N + B->off[b], H.pts64 + q * H.n, H.n);
            mg.add32(M->order + B->off[b], H.order, H.n, B->off[b]);
        }

        // level slots, slot s at M->lev[S - 1 - s]
        std::vector<int64_t> prev_piv_off(count, 0);   // pivot offsets of slot s - 1 per problem
        for (int sl = 0; sl < S; sl++) {
            Level &D = M->lev[S - 1 - sl];
            struct Part {
                const Level *L;
                int32_t b;
                int64_t cell, piv, rem, crem, il, nb;
            };
            std::vector<Part> parts;
            std::vector<int64_t> piv_off(count, -1);
            int64_t nc = 0, np = 0, nr = 0, ncr = 0, nil = 0, nnb = 0;
            for (int32_t b = 0; b < count; b++) {
                const nnca_h2 &H = *hs[b];
                const int l = H.kappa - sl;
                if (l < H.lmin) continue;
                const Level &L = H.lev[l];
                parts.push_back({&L, b, nc, np, nr, ncr, nil, nnb});
                piv_off[b] = np;
                nc += L.ncell;
                np += L.npiv;
                nr += L.nrem;
                ncr += L.ncrem;
                nil += L.nil;
                if (sl == 0) nnb += L.nnb;
                D.max_k = std::max(D.max_k, L.max_k);
                D.max_nrem = std::max(D.max_nrem, L.max_nrem);
                D.max_ilsum = std::max(D.max_ilsum, L.max_ilsum);
                D.m2l_inter += L.m2l_inter;
                D.h_k.insert(D.h_k.end(), L.h_k.begin(), L.h_k.end());
                D.h_m.insert(D.h_m.end(), L.h_m.begin(), L.h_m.end());
            }
            if (std::max({nc, np, nr, ncr, nil, nnb}) > INT32_MAX / 2)
                fail(NNCA_ERR_NOT_SUPPORTED, "batch exceeds 32-bit indices");
            D.ncell = nc;
            D.npiv = np;
            D.nrem = nr;
            D.ncrem = ncr;
            D.nil = nil;
            D.nnb = nnb;
            D.has_piv = true;
            D.h = 0.0;
            D.coord = dalloc<int32_t>(3 * nc);
            D.hcell = dalloc<float>(nc);
            D.il_ptr = dalloc<int32_t>(nc + 1);
            D.il = dalloc<int32_t>(nil);
            D.m = dalloc<int32_t>(nc);
            D.tt_off = dalloc<int32_t>(nc);
            D.k = dalloc<int32_t>(nc);
            D.piv_ptr = dalloc<int32_t>(nc + 1);
            D.ipos = dalloc<int32_t>(np);
            D.rem_ptr = dalloc<int32_t>(nc + 1);
            D.rem_pos = dalloc<int32_t>(nr);
            D.crem_off = dalloc<int64_t>(nc + 1);
            D.crem64 = dalloc<double>(ncr);
            D.crem_t = dalloc<double>(ncr);
            D.piv_cell = dalloc<int32_t>(np);
            D.rem_cell = dalloc<int32_t>(nr);
            D.pc64 = dalloc<double>(3 * np);
            D.pc32 = dalloc<float>(3 * np);
            D.ilpre = dalloc<int32_t>(nil);
            D.ilsum = dalloc<int32_t>(nc);
            D.w64 = dalloc<double>(np);
            D.u64 = dalloc<double>(np);
            if (sl == 0) {
                D.first = dalloc<int32_t>(nc);
                D.count = dalloc<int32_t>(nc);
                D.nb_ptr = dalloc<int32_t>(nc + 1);
                D.nb = dalloc<int32_t>(nnb);
                M->nbpre = dalloc<int32_t>(nnb);
                M->nbsum = dalloc<int32_t>(nc);
            }
            for (const Part &p : parts) {
                const Level &L = *p.L;
                const nnca_h2 &H = *hs[p.b];
                const int64_t c = L.ncell;
                for (int q = 0; q < 3; q++) {
                    if (q < H.dim) mg.copy(D.coord + q * nc + p.cell, L.coord + q * c, c);
                    mg.copy(D.pc64 + q * np + p.piv, L.pc64 + q * L.npiv, L.npiv);
                    mg.copy(D.pc32 + q * np + p.piv, L.pc32 + q * L.npiv, L.npiv);
                }
                k_fill_f32<<<grid_for(c, 256), 256, 0, s>>>(c, (float)L.h, D.hcell + p.cell);
                HIPCHECK(hipGetLastError());
                mg.add32(D.il_ptr + p.cell, L.il_ptr, c + 1, p.il);
                mg.add32(D.il + p.il, L.il, L.nil, p.cell);
                mg.copy(D.m + p.cell, L.m, c);
                mg.add32(D.tt_off + p.cell, L.tt_off, c, sl == 0 ? B->off[p.b] : prev_piv_off[p.b]);
                mg.copy(D.k + p.cell, L.k, c);
                mg.add32(D.piv_ptr + p.cell, L.piv_ptr, c + 1, p.piv);
                mg.copy(D.ipos + p.piv, L.ipos, L.npiv);
                mg.add32(D.rem_ptr + p.cell, L.rem_ptr, c + 1, p.rem);
                mg.copy(D.rem_pos + p.rem, L.rem_pos, L.nrem);
                mg.add64(D.crem_off + p.cell, L.crem_off, c + 1, p.crem);
                mg.copy(D.crem64 + p.crem, L.crem64, L.ncrem);
                mg.copy(D.crem_t + p.crem, L.crem_t, L.ncrem);
                mg.add32(D.piv_cell + p.piv, L.piv_cell, L.npiv, p.cell);
                mg.add32(D.rem_cell + p.rem, L.rem_cell, L.nrem, p.cell);
                mg.copy(D.ilpre + p.il, L.ilpre, L.nil);
                mg.copy(D.ilsum + p.cell, L.ilsum, c);
                if (sl == 0) {
                    mg.add32(D.first + p.cell, L.first, c, B->off[p.b]);
                    mg.copy(D.count + p.cell, L.count, c);
                    mg.add32(D.nb_ptr + p.cell, L.nb_ptr, c + 1, p.nb);
                    mg.add32(D.nb + p.nb, L.nb, L.nnb, p.cell);
                    mg.copy(M->nbpre + p.nb, H.nbpre, L.nnb);
                    mg.copy(M->nbsum + p.cell, H.nbsum, c);
                    M->max_leaf = std::max(M->max_leaf, H.max_leaf);
                }
            }
            for (int32_t b = 0; b < count; b++) prev_piv_off[b] = piv_off[b];
            M->m2l_inter += D.m2l_inter;
            M->transfer_entries += D.ncrem;
        }
        for (int32_t b = 0; b < count; b++) M->p2p_inter += hs[b]->p2p_inter;
        HIPCHECK(hipStreamSynchronize(s));
        M->fp32_levels = mixed_fp32_levels(M->kind);
        for (int l = 0; l <= M->kappa; l++) prepare_symmetric(M, M->lev[l], l <= M->kappa - M->fp32_levels);
        HIPCHECK(hipStreamCreateWithFlags(&M->aux, hipStreamNonBlocking));
        HIPCHECK(hipEventCreateWithFlags(&M->ev_fork, hipEventDisableTiming));
        HIPCHECK(hipEventCreateWithFlags(&M->ev_join, hipEventDisableTiming));
        HIPCHECK(hipEventCreateWithFlags(&M->ev_leafk, hipEventDisableTiming));
        M->xs64 = dalloc<double>(N);
        M->far64 = dalloc<double>(N);
        prepare_output(M, s);
        M->xhi = dalloc<float>(N);
        M->xlo = dalloc<float>(N);
        prepare_workspace(M);
        HIPCHECK(hipStreamSynchronize(s));
    } catch (...) {
        destroy_batch(B);
        throw;
    }
    return B;
}

void run_batch(nnca_batch *B, const double *X, double *Y, int64_t nrhs, int64_t ldx, int64_t ldy, int precision,
               hipStream_t cs)
{
    HIPCHECK(hipEventRecord(B->ev_in, cs));
    HIPCHECK(hipStreamWaitEvent(B->gs, B->ev_in, 0));
    if (!B->use_graph) {
        run_matvec(B->M, X, Y, nrhs, ldx, ldy, NNCA_F64, precision, B->gs);
    } else {
        nnca_batch::Key k;
        k.X = X;
        k.Y = Y;
        k.nrhs = nrhs;
        k.ldx = ldx;
        k.ldy = ldy;
        k.prec = precision;
        if (!B->have_graph || !(k == B->key)) {
            if (B->exec) HIPCHECK(hipGraphExecDestroy(B->exec));
            if (B->graph) HIPCHECK(hipGraphDestroy(B->graph));
            B->exec = nullptr;
            B->graph = nullptr;
            B->have_graph = false;
            // eager run: workspaces and tuned split factors exist before capture
            run_matvec(B->M, X, Y, nrhs, ldx, ldy, NNCA_F64, precision, B->gs);
            HIPCHECK(hipStreamSynchronize(B->gs));
            HIPCHECK(hipStreamBeginCapture(B->gs, hipStreamCaptureModeThreadLocal));
            try {
                run_matvec(B->M, X, Y, nrhs, ldx, ldy, NNCA_F64, precision, B->gs);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(B->gs, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            HIPCHECK(hipStreamEndCapture(B->gs, &B->graph));
            HIPCHECK(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
            B->key = k;
            B->have_graph = true;
        }
        HIPCHECK(hipGraphLaunch(B->exec, B->gs));
    }
    HIPCHECK(hipEventRecord(B->ev_out, B->gs));
    HIPCHECK(hipStreamWaitEvent(cs, B->ev_out, 0));
}

int64_t batch_rows(const nnca_batch *B) { return B->off[B->count]; }
const Allocator *batch_allocator(const nnca_batch *B) { return &B->M->alloc; }
int32_t batch_count(const nnca_batch *B) { return B->count; }
const int64_t *batch_offsets(const nnca_batch *B) { return B->off.data(); }

}  // namespace nnca
