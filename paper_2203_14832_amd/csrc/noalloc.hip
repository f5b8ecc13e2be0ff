// Allocation-free matvec: nnca_matvec_noalloc runs the one-column passes of
// nnca_matvec with every per-call buffer (the input in tree order and its
// FP32 split, the multipole and local vectors of every level, the column
// slots of the symmetric passes, the split partial vectors, the near-field
// and far-field sums) carved out of one static device array instead of the
// handle's workspace.  The kernels are nnca_matvec's; they receive the
// array's device address like any other buffer.
#include <mutex>

#include "nnca_internal.h"

namespace nnca {

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
constexpr size_t SCRATCH_ALIGN = 256;
constexpr int MAX_DEVICES = 64;

// One copy per GPU the library runs on, held until the process ends.  Host
// code never uses this name as an address: it asks the runtime for the
// device address (scratch_base) and passes that to the kernels.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mtx;
void *g_base[MAX_DEVICES] = {};

// device address of the current device's array, looked up once per device
void *scratch_base()
{
    int dev = -1;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) fail(NNCA_ERR_NOT_SUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_mtx);
    if (!g_base[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(NNCA_ERR_HIP, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
        }
        g_base[dev] = p;
    }
    return g_base[dev];
}

// The per-call buffers of the one-column matvec: where the handle keeps each
// pointer and how many bytes it needs (fixed capacity: nothing is allocated
// on the host either).
struct Slot {
    void **field;
    size_t bytes;
};
constexpr int MAX_SLOTS = 9 + 3 * NNCA_MAX_LEVELS;
struct Slots {
    Slot s[MAX_SLOTS];
    int n = 0;
    void add(void **field, size_t bytes)
    {
        if (n == MAX_SLOTS) fail(NNCA_ERR_INTERNAL, "too many scratch slots");
        s[n++] = {field, bytes};
    }
};

void per_call_buffers(nnca_h2 *H, Slots &v)
{
    const size_t n = (size_t)H->n;
    v.add((void **)&H->xs64, n * sizeof(double));
    v.add((void **)&H->far64, n * sizeof(double));
    v.add((void **)&H->near64, n * sizeof(double));
    v.add((void **)&H->xhi, n * sizeof(float));
    v.add((void **)&H->xlo, n * sizeof(float));
    if (H->p2p_sym) {
        v.add((void **)&H->prow, 2 * n * sizeof(double));
        v.add((void **)&H->pcol_hi, (size_t)H->pcol_n * sizeof(float));
        v.add((void **)&H->pcol_lo, (size_t)H->pcol_n * sizeof(float));
    }
    if (H->m2l_part_cap > 0) v.add((void **)&H->m2l_part, (size_t)H->m2l_part_cap * sizeof(double));
    for (int l = H->lmin; l <= H->kappa; l++) {
        Level &L = H->lev[l];
        if (!L.has_piv) continue;
        const size_t np = (size_t)(L.npiv > 0 ? L.npiv : 1);
        v.add((void **)&L.w64, np * sizeof(double));
        v.add((void **)&L.u64, np * sizeof(double));
        if (L.sym) v.add((void **)&L.col64, (size_t)(L.ncol > 0 ? L.ncol : 1) * sizeof(double));
    }
}

size_t aligned(size_t b) { return (b + SCRATCH_ALIGN - 1) / SCRATCH_ALIGN * SCRATCH_ALIGN; }

// Points the handle's per-call buffers at consecutive slices of the scratch
// array for the lifetime of the object, then puts the handle's own back
// (host pointers only: work already launched keeps the slices it was given).
struct ScratchView {
    nnca_h2 *H;
    const Slots &slots;
    void *saved[MAX_SLOTS];
    float *saved32[NNCA_MAX_LEVELS];
    int32_t saved_prof;
    ScratchView(nnca_h2 *H_, char *base, const Slots &s) : H(H_), slots(s), saved_prof(H_->prof_mask)
    {
        size_t off = 0;
        for (int i = 0; i < slots.n; i++) {
            saved[i] = *slots.s[i].field;
            *slots.s[i].field = base + off;
            off += aligned(slots.s[i].bytes);
        }
        for (size_t l = 0; l < H->lev.size(); l++) {
            Level &L = H->lev[l];
            saved32[l] = L.col32;
            if (L.sym) L.col32 = reinterpret_cast<float *>(L.col64);   // the FP32 form's view of the slots
        }
        H->prof_mask = 0;   // no event records (they would create events)
    }
    ~ScratchView()
    {
        for (int i = 0; i < slots.n; i++) *slots.s[i].field = saved[i];
        for (size_t l = 0; l < H->lev.size(); l++) H->lev[l].col32 = saved32[l];
        H->prof_mask = saved_prof;
    }
};

}  // namespace

}  // namespace nnca

using namespace nnca;

extern "C" nnca_status nnca_matvec_noalloc(nnca_handle h, const void *X, void *Y, int64_t nrhs, int64_t ldx,
                                           int64_t ldy, int32_t dtype, int32_t precision, void *stream)
{
    try {
        check_matvec_args(h, X, Y, nrhs, ldx, ldy, dtype, precision);
        if (h->general) fail(NNCA_ERR_NOT_SUPPORTED, "nnca_matvec_noalloc covers P = Q only (a handle of nnca_build)");
        if (h->lev.size() > (size_t)NNCA_MAX_LEVELS) fail(NNCA_ERR_INTERNAL, "too many levels");
        Slots slots;
        per_call_buffers(h, slots);
        size_t need = 0;
        for (int i = 0; i < slots.n; i++) need += aligned(slots.s[i].bytes);
        if (need > SCRATCH_BYTES)
            fail(NNCA_ERR_NOT_SUPPORTED, "the matvec needs " + std::to_string(need) + " bytes of workspace; the "
                                         "static scratch holds " + std::to_string(SCRATCH_BYTES) +
                                         " (use nnca_matvec)");
        char *base = static_cast<char *>(scratch_base());
        const hipStream_t s = (hipStream_t)stream;
        ScratchView view(h, base, slots);
        order_call_begin(h, s);
        run_matvec_columns(h, X, Y, nrhs, ldx, ldy, dtype, precision, s);
        order_call_end(h, s);
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
