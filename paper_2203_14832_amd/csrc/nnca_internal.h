// Internal declarations of the gfx950 NNCA library: the handle, the per-level
// device layout and the launchers that each translation unit provides.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "nnca.h"

namespace nnca {

// Thrown inside the library and turned into an nnca_status at the ABI.
struct Error {
    nnca_status status;
    std::string msg;
};

void set_error(const std::string &msg);
[[noreturn]] void fail(nnca_status s, const std::string &msg);
void hip_check(hipError_t e, const char *what);
#define HIPCHECK(x) ::nnca::hip_check((x), #x)

// Device allocator of a handle (the caller's, or hipMalloc / hipFree when
// both functions are NULL).  Every ABI call that may allocate or free
// installs its handle's allocator for the calling thread (AllocScope); dalloc
// and dfree use the installed one.
struct Allocator {
    nnca_alloc_fn alloc = nullptr;
    nnca_free_fn free = nullptr;
    void *ctx = nullptr;
};
const Allocator *current_allocator();
struct AllocScope {
    const Allocator *prev;
    explicit AllocScope(const Allocator &a);
    ~AllocScope();
};
void *dalloc_bytes(size_t bytes);

// Device allocation owned by the library (freed with the handle).
template <typename T>
T *dalloc(size_t count)
{
    if (count == 0) count = 1;
    return static_cast<T *>(dalloc_bytes(count * sizeof(T)));
}
void dfree(void *p);

// One level of the uniform 2^d tree and, from lmin to kappa, its pivots,
// transfer operators and apply buffers.  All pointers are device memory.
// Cells are the non-empty cells of the level in ascending Morton order;
// points are addressed by their position in tree order ("sorted ids").
struct Level {
    int64_t ncell = 0;
    double h = 0.0;                  // cell side
    uint64_t *key = nullptr;         // Morton prefix of each cell
    int32_t *coord = nullptr;        // integer coordinates, SoA: coord[q * ncell + c]
    int32_t *first = nullptr;        // tree-order range of the cell's points
    int32_t *count = nullptr;
    int32_t *parent = nullptr;       // cell index one level up (-1 at the root)
    int32_t *child_first = nullptr;  // children: [child_first, child_first + child_count)
    int32_t *child_count = nullptr;
    int32_t *nb_ptr = nullptr, *nb = nullptr;  // N(B), CSR, ascending
    int32_t *il_ptr = nullptr, *il = nullptr;  // IL(B), CSR, ascending
    int64_t nnb = 0, nil = 0;

    // pivots: levels lmin..kappa
    bool has_piv = false;
    int64_t npiv = 0;                // sum of ranks
    int32_t max_k = 0;
    int32_t max_nrem = 0;            // most non-pivot rows of one cell
    int32_t *m = nullptr;            // |t~^{B,i}|
    int32_t *tt_off = nullptr;       // t~ as a range: leaf -> tree order, else -> piv_id of level+1
    int32_t *k = nullptr;            // rank k_B = |t^{B,i}|
    int32_t *piv_ptr = nullptr;      // ncell + 1
    int32_t *piv_id = nullptr;       // t^{B,i}: sorted ids, ACA selection order
    int32_t *ipos = nullptr;         // position of each pivot inside t~
    int32_t *jid = nullptr;          // s^{B,i}: sorted ids (-1 for a cell kept whole)
    int32_t *rem_ptr = nullptr;      // ncell + 1: rows of t~ that are not pivots
    int32_t *rem_pos = nullptr;      //   their positions inside t~, ascending
    int64_t *crem_off = nullptr;     // ncell + 1: offsets of each cell's block in crem
    int64_t ncrem = 0;
    double *crem64 = nullptr;        // non-identity rows of C_B, (m - k) x k row-major
    double *crem_t = nullptr;        //   the same blocks transposed, k x (m - k)
    int64_t nrem = 0;                // rows of t~ that are not pivots, over the level
    int32_t *piv_cell = nullptr;     // owning cell of every pivot
    int32_t *rem_cell = nullptr;     // owning cell of every non-pivot row
    double *pc64 = nullptr;          // pivot coordinates, SoA 3 x npiv (global)
    float *pc32 = nullptr;           // pivot coordinates relative to the cell centre
    int32_t *ilpre = nullptr;        // per IL entry: sources before it in the cell's list
    int32_t *ilsum = nullptr;        // per cell: M2L sources
    std::vector<int32_t> h_k, h_m;   // host copies
    int32_t max_ilsum = 0;
    int64_t m2l_inter = 0;           // sum over IL pairs of k_B k_B' at this level
    float *hcell = nullptr;          // per-cell side, set when a level holds cells of several problems

    // symmetric transverse pass (mixed form): each unordered pair of
    // interacting cells is evaluated once, by its owner; the owner's row sums
    // go to its local vector, its column sums to a slot of colbuf that the
    // partner adds afterwards
    bool sym = false;
    int32_t *own_ptr = nullptr, *own_il = nullptr, *own_pre = nullptr, *own_sum = nullptr;
    int32_t *own_slot = nullptr;     // per owned entry: colbuf offset of its first source minus own_pre
    int32_t *non_ptr = nullptr, *non_slot = nullptr;   // per cell: slots of the pairs it does not own
    int32_t *sym_order = nullptr;    // launch order: 8 runs (one per XCD) of sym_slots cells, -1 = empty,
    int64_t sym_slots = 0, sym_slots_hi = 0;   // then 8 runs of sym_slots_hi cells of rank > 80 (if split)
    int32_t *m2l_order = nullptr;    // launch order of the plain transverse pass: 8 runs of m2l_slots cells
    int64_t m2l_slots = 0;
    float *col32 = nullptr;          // column slots, FP32 (FP32 form) or
    double *col64 = nullptr;         //   FP64 (FP64-refined form)
    int64_t ncol = 0;
    int32_t max_own = 0;

    // apply state (one right-hand side at a time): multipole / local vectors
    double *w64 = nullptr, *u64 = nullptr;

    // general case: the outgoing half's levels share the tree fields (key,
    // coord, parent, children, lists) of the incoming half's levels
    bool shares_tree = false;
};

struct ChunkInfo;

}  // namespace nnca

struct nnca_h2 {
    int64_t n = 0;
    int32_t dim = 3, kind = NNCA_K_INV_R, leaf = 64;
    double hparam = 1.0, tol = 0.0;
    int64_t eta_num = 3, eta_den = 1;
    int32_t policy = 1;
    int64_t ws_budget = 0;
    int32_t rank_reserve = 256;
    int32_t apply_flags = 0;      // NNCA_APPLY_* bits
    nnca::Allocator alloc;        // device memory of the handle
    int32_t max_rhs = 16;         // columns of the many-column workspace (1: none)
    hipEvent_t ev_done = nullptr; // end of the last matvec (orders calls across streams)
    int32_t fp32_levels = 2;      // mixed matvec: finest levels whose transverse pass runs in FP32
    int32_t kmax = 20, kappa = 0, lmin = 1;
    double lo[3] = {0, 0, 0}, L = 0.0;
    hipStream_t stream = nullptr;
    hipStream_t aux = nullptr;               // second stream of the matvec (near field)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_leafk = nullptr;           // after the leaf level's transverse kernel
    double build_seconds = 0.0;
    double aca_seconds = 0.0;     // the pivot traversal (ACA and transfer operators) of the build
    double aca_panel_bytes = 0.0; // its algorithmic panel reads: sum over ACA cells of k (k - 1) n 8 bytes

    // General case P != Q (Sec. 2.1, 2.3): n is |P| (the rows), nq = |Q| (the
    // columns).  lev holds the incoming half of every cell (targets: first /
    // count are ranges of P in P's tree order; pivots t^{B,i}, operators U_B /
    // C_{B_c B}), lev_o the outgoing half (sources: ranges of Q in Q's tree
    // order; pivots s^{B,o}, operators V_B / T_{B B_c}^T).  With P = Q
    // (general == false) lev_o is empty and lev serves both halves.
    bool general = false;
    int64_t nq = 0;
    std::vector<nnca::Level> lev_o;
    double *qpts64 = nullptr;     // 3 x nq, Q's tree order
    int32_t *qorder = nullptr;    // Q's tree position -> index into Q
    int32_t *qrank = nullptr;     // inverse of qorder
    int32_t *nbpre_o = nullptr;   // leaf level, transposed product: per N entry, targets before it
    int32_t *nbsum_o = nullptr;   //   and per cell the near-field targets
    int64_t io_cap = 0;           // entries of xs64, far64, near64, xhi, xlo

    double *pts64 = nullptr;      // 3 x n, tree order
    int32_t *order = nullptr;     // tree position -> original index
    uint64_t *keys = nullptr;     // finest Morton key per tree position
    std::vector<nnca::Level> lev;

    int32_t *nbpre = nullptr;     // leaf level: per N entry, sources before it
    int32_t *nbsum = nullptr;     // leaf level: near-field sources per cell
    int32_t max_leaf = 0;
    int64_t p2p_split = 0;        // leaf cell where half of the near-field work is done

    // matvec workspace
    double *xs64 = nullptr, *far64 = nullptr;
    double *near64 = nullptr;     // near-field sums in tree order (overlapped schedule)
    int32_t *rank = nullptr;      // original index -> tree position (inverse of order)
    float *xhi = nullptr, *xlo = nullptr;
    // symmetric near field of the mixed matvec (leaf level): per cell the
    // owned neighbour entries (cell, first source, column slot of source 0),
    // the owned source count, the slots of the pairs owned by neighbours;
    // FP32 column slots (x_hi and x_lo parts), FP64 row sums (2 x n), the
    // leaf cell of every point
    bool p2p_sym = false;
    int32_t *pown_ptr = nullptr, *pown_nb = nullptr, *pown_pre = nullptr, *pown_sum = nullptr;
    int32_t *pown_slot = nullptr, *pnon_ptr = nullptr, *pnon_slot = nullptr, *pcell = nullptr;
    float *pcol_hi = nullptr, *pcol_lo = nullptr;
    double *prow = nullptr;
    int64_t pcol_n = 0;           // entries of pcol_hi and of pcol_lo
    double *m2l_part = nullptr;   // partial M2L vectors of split launches
    int64_t m2l_part_cap = 0;

    // workspace of the many-column matvec: rows in tree order, columns
    // innermost, padded to rp columns
    struct Multi {
        int rp = 0;
        double *xs = nullptr, *far = nullptr, *part = nullptr;
        int64_t part_cap = 0;
        float *xhi = nullptr, *xlo = nullptr;
        std::vector<double *> w, u;   // per level
        std::vector<float *> w32;     // per level: FP32 copy of w for the FP32 transverse pass
        int R = 0;                    // columns of the block in flight
    } multi;
    // transverse-pass choices per level picked by timing (autotune on): 2 P +
    // TSEL (split factor, tile shape), keyed by column-block width and
    // precision
    bool autotune = false;
    std::map<int, std::vector<int32_t>> m2l_tuned;
    int64_t m2l_inter = 0, p2p_inter = 0, transfer_entries = 0;

    // state of the length-scale derivative (set up on first use; pivots frozen)
    struct Grad {
        bool ready = false;
        std::vector<int64_t *> lu_off;   // per level: ncell + 1 offsets into lu
        std::vector<double *> lu;        // per level: L U = K(I, J) of every ACA cell, column-major
        std::vector<double *> gw, gu;    // per level: multipole / local vectors of the cotangent
        std::vector<double *> zx, zg;    // per level: K(I, J)^{-1} u of x and of the cotangent
        std::vector<int32_t *> items;    // per level: (cell, first row) of every row block
        std::vector<int64_t> nitems;
        std::vector<int64_t> term_off;   // per level: first row-block term; the dot parts follow
        double *gs = nullptr;            // cotangent in tree order
        double *yd = nullptr;            // derivative-kernel product, original order
        double *terms = nullptr;
        int64_t nterms = 0, lu_entries = 0;
        int32_t *flag = nullptr;
    } grad;

    // per-launch HIP-event timing of the matvec passes (off by default)
    struct ProfRec {
        int32_t pass, level;
        hipEvent_t a, b;
    };
    int32_t prof_mask = 0;        // bit p: record launches of pass p
    std::vector<ProfRec> prof;
};

namespace nnca {

// tree.hip.  With split >= 0 the points are the union of P (indices <
// split) and Q, and the depth counts each set on its own.
void build_tree(nnca_h2 *H, const double *pts_dev, int64_t ld, int64_t split = -1);
// after build_tree over the union: the general layout (lev / lev_o ranges,
// pts64 / qpts64, order / qorder); H->n becomes |P|
void split_general(nnca_h2 *H, const double *Z, int64_t ldz, int64_t split);
// aca.hip
void build_pivots(nnca_h2 *H);
void debug_kernel_eval(int kind, double hparam, int dim, const double *a, const double *b,
                       int64_t count, double *out, hipStream_t s);
// apply.hip
void prepare_apply(nnca_h2 *H);
void prepare_general(nnca_h2 *H);
// general case: Y = A~ X (X: nq rows, Y: n rows) or, with adjoint, A~^T X
void run_matvec_general(nnca_h2 *H, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy, int dtype,
                        int precision, bool adjoint, hipStream_t s);
// X, Y of element type dtype (NNCA_F32 / NNCA_F64)
void run_matvec(nnca_h2 *H, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy, int dtype,
                int precision, hipStream_t s);
void run_matvec_multi(nnca_h2 *H, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy, int dtype,
                      int precision, hipStream_t s);
// one column at a time (the one-column passes), whatever nrhs
void run_matvec_columns(nnca_h2 *H, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy, int dtype,
                        int precision, hipStream_t s);
// workspace of the matvec, allocated once (build, batch creation): split
// partial vectors of the one-column transverse pass and the many-column
// buffers for H->max_rhs columns
void prepare_workspace(nnca_h2 *H);
void alloc_multi(nnca_h2 *H, int RP);
void free_multi(nnca_h2 *H);
void gather_input(nnca_h2 *H, const double *x, int precision, hipStream_t s);
void prepare_symmetric(nnca_h2 *H, Level &L, bool fp64_slots);
void prepare_output(nnca_h2 *H, hipStream_t s);
int mixed_fp32_levels(int kind);
void column_passes(nnca_h2 *H, int precision, int kind, bool do_up, bool do_p2p, double *y, hipStream_t s);
// grad.hip
void run_backward(nnca_h2 *H, const double *X, const double *G, int64_t nrhs, int64_t ldx, int64_t ldg,
                  int precision, double *DX, int64_t lddx, double *dldh, hipStream_t s);
void free_grad(nnca_h2 *H);
// api.hip
void destroy_handle(nnca_h2 *H);
void check_matvec_args(nnca_h2 *h, const void *X, const void *Y, int64_t nrhs, int64_t ldx, int64_t ldy,
                       int32_t dtype, int32_t precision, bool adjoint = false);
void order_call_begin(nnca_h2 *h, hipStream_t s);
void order_call_end(nnca_h2 *h, hipStream_t s);
// batch.hip
nnca_batch *create_batch(nnca_h2 *const *hs, int32_t count, int32_t flags);
void destroy_batch(nnca_batch *B);
void run_batch(nnca_batch *B, const double *X, double *Y, int64_t nrhs, int64_t ldx, int64_t ldy, int precision,
               hipStream_t cs);
int64_t batch_rows(const nnca_batch *B);
const Allocator *batch_allocator(const nnca_batch *B);
int32_t batch_count(const nnca_batch *B);
const int64_t *batch_offsets(const nnca_batch *B);
enum { PASS_GATHER = 0, PASS_UP = 1, PASS_M2L = 2, PASS_DOWN = 3, PASS_P2P = 4, PASS_M2L_COMBINE = 5 };
// gmres.hip: restarted GMRES(restart) for (alpha I + beta A~) x = f
void run_gmres(nnca_h2 *H, double alpha, double beta, const double *F, double *X, double tol, int32_t max_iter,
               int32_t restart, int precision, int32_t *iters, double *relres, hipStream_t s);
// svm.hip: projected gradient ascent on the penalised SVM dual (eta <= 0:
// 1 / (|K~|_2 + beta n) by the power method), then the bias; the decision
// function f = K~ (y .* alpha) + bias
void run_svm_train(nnca_h2 *H, const double *y, double *alpha, double lambda, double beta, double eta, double tol,
                   int32_t max_iter, int precision, int32_t *iters, double *bias, double *eta_used,
                   hipStream_t s);
void run_svm_decision(nnca_h2 *H, const double *y, const double *alpha, double bias, double *f, int precision,
                      hipStream_t s);
// probe.hip: out[0..count) of {HBM copy bytes/s, FP32 FMA lane-ops/s,
// v_rsq_f32 lane-ops/s, pairs/s of the symmetric pass's inner loop with r^2
// on the vector ALUs, the same with r^2 on the matrix cores}
void probe_rates(double *out, int32_t count, hipStream_t s);
void run_direct(const double *pts, int64_t n, int dim, int64_t ld, int kind, double hparam,
                const double *X, double *Y, int64_t nrhs, int64_t ldx, int64_t ldy, hipStream_t s);

// event pair around one launch when the handle is profiling
struct Span {
    nnca_h2 *H;
    hipStream_t s;
    bool on;
    nnca_h2::ProfRec r;
    Span(nnca_h2 *H_, hipStream_t s_, int pass, int level) : H(H_), s(s_), on(((H_->prof_mask >> pass) & 1) != 0)
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

inline int grid_for(int64_t work, int block)
{
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 1048576) g = 1048576;
    return (int)g;
}

}  // namespace nnca
