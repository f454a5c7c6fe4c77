// C ABI of the DAO library (include/dao.h): context, device buffers, launch
// sequences and the column-generation driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <type_traits>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dao.h"
#include "dao_common.h"
#include "kernels.h"
#include "kernels_ap.h"
#include "kernels_coop.h"
#include "layout.h"

using namespace dao;

namespace {

thread_local std::string g_create_error;

constexpr size_t STAGE_LIMIT = 48 * 1024;   // largest vector staged in LDS per block
constexpr int MAX_BATCH = 64;                // solves of one batched master launch
constexpr int ELEM_BLOCKS_MAX = 2048;
constexpr int REDUCE_BLOCKS_MAX = 512;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct dao_ctx {
    dao_options opt{};
    int dtype = DAO_F32;
    size_t tsize = 4;
    hipStream_t stream = nullptr;
    std::string err;

    // sizes and host geometry
    int64_t V = 0, N = 0, nnz = 0, Vnz = 0, Vpad = 0, nslices = 0;
    int32_t B = 0, R = 0, maxRB = 0, ncls = 0;
    uint32_t sell_entries = 0;
    double F_const = 0.0;
    std::vector<int32_t> rows_per_beam, row_len, beam_row0;

    // device memory
    std::vector<DevBuf> bufs;
    int64_t device_bytes = 0;
    uint32_t* slice_ptr = nullptr;
    int32_t* slice_w = nullptr;
    void* sell_val = nullptr;
    uint16_t* sell_col = nullptr;
    int32_t* perm = nullptr;
    int32_t* csc_ptr = nullptr;
    int32_t* csc_row = nullptr;
    void* csc_val = nullptr;
    void* sell_lo = nullptr;           // FP16 residuals of the 16-bit formats (with d_residual)
    void* csc_lo = nullptr;
    float* col_scale = nullptr;        // per-beamlet scale of the 16-bit formats
    uint8_t* cls_int = nullptr;
    uint8_t* cls_ext = nullptr;
    ObjClass* classes = nullptr;
    int32_t *row_start_d = nullptr, *row_len_d = nullptr, *beam_row0_d = nullptr;
    int32_t *blt_beam_d = nullptr, *blt_row_d = nullptr, *blt_pos_d = nullptr;
    // master vectors
    double* d = nullptr;       // [Vpad] master dose
    void* q = nullptr;         // [Vpad] ctx type
    void* u = nullptr;         // [Vpad] ctx type
    double* u64 = nullptr;     // [Vpad]
    void* ug = nullptr;        // [Vpad] scratch for dao_gradient
    void* vscratch = nullptr;  // [V] ctx type, allocated on first product timing
    void* dk = nullptr;        // [Vpad * KS] ctx type: aperture dose matrix (aperture master)
    void* ind = nullptr;       // [N] ctx type: 0/1 beamlet indicator of one aperture
    double* parts2 = nullptr;  // [ap_blocks * (KS + 1)] update records of the aperture master
    ProfCounters* pc = nullptr;
    CoopSync* coop = nullptr;          // grid-reduction scratch of the persistent master
    double* coop_recs = nullptr;       // [2][coop_grid][RECW]
    double* coop_bpart = nullptr;      // streaming form's per-batch grad_y partials (Vpad / 32 * KS)
    int coop_grid = 0;                 // co-resident workgroups (0: persistent master unavailable)
    int ncu = 0;                       // compute units of the device
    int coop_lds_max = 0;              // dynamic LDS the on-chip variant may use (0: never)
    void* batch_args = nullptr;        // [MAX_BATCH] CoopArgs of a batched master launch
    int32_t* batch_gstart = nullptr;   // [MAX_BATCH + 1] first workgroup of each solve
    void* batch_host = nullptr;        // pinned staging of both
    bool batch_ok = false;             // the batched master launch is available
    ProfCounters* pc_h = nullptr;      // pinned
    int prof_kernel = -1;              // aperture-master kernel timed with events (-1: none)
    int last_form = -1;                // form of the last master solve (dao_info_t.last_master_form)
    double prof_phase_us[PROF_PHASES] = {};   // persistent master split of the last window
    int device = 0;                    // HIP device of the context
    int dose_var = 0;                  // k_dose variant (0 staged, 1 staged + deep loads, 2 global x + deep)
    int32_t* slice_order[2] = {nullptr, nullptr};   // dose variants 7 / 8: balanced slice lists
    int slice_rounds[2] = {0, 0};
    int gradT_pf = 4;                  // k_gradT entries in flight per thread (4, 8 or 16)
    int last_steps = 0;                // steps of the previous master solve (chunk size guess)
    // column-generation loop state of the last (or restored) solve, for resume
    double loop_rc1 = NAN;             // reduced cost of round 1 (NaN: none yet)
    double loop_eps = 0.0;             // current master tolerance factor
    int loop_tighten = 0;              // tightenings so far
    int last_stop = 0;                 // stop reason of the last master solve (MasterState.stop_reason)
    std::vector<hipEvent_t> prof_events;
    hipGraphExec_t price_exec[2] = {nullptr, nullptr};   // captured pricing sequence (without / with residual)
    hipStream_t cap_stream = nullptr;  // capture only (the null stream cannot be captured); replays use `stream`
    size_t prof_used = 0;
    void* g = nullptr;         // [N] ctx type
    double* g64 = nullptr;     // [N]
    void* dx = nullptr;        // [N] ctx type
    double* x64 = nullptr;     // [N]
    // pool
    int K = 0;
    int32_t* ap_beam = nullptr;
    int16_t* ap_lv = nullptr;
    double* y = nullptr;
    double* p = nullptr;
    CgMem* cgm = nullptr;             // conjugate-direction memory of the master
    bool dk16 = false;                // D_K stored in FP16 (values over dk_scale)
    bool lo_now = false;              // selective residual: products use the FP16 residual now
    bool final_phase = false;         // selective residual: the plan's final rounds have begun
    int32_t reprices = 0;             // selective residual: near-tie decisions priced again with it
    double* gabs64 = nullptr;         // [N] D^T |grad F| (rounding bound of the prices)
    double* uabs64 = nullptr;         // [Vpad] |grad F|
    double dk_scale = 1.0;            // D_K = dk_scale * stored value
    double dk16_scale = 1.0;          // dk_scale while D_K is stored in FP16
    bool dk16_base = false;           // the storage a plan starts with (dk_format, resolved at creation)
    double* tau_int = nullptr;        // per-voxel threshold shifts, internal rows (null: none)
    double* tau_ext = nullptr;        // the same in caller order
    unsigned char* scratch_dev = nullptr;   // this device's copy of the static pricing scratch
    double* gradk = nullptr;
    std::vector<int32_t> pool_beam;
    std::vector<int16_t> pool_lv;
    // state and scratch
    MasterState* ms = nullptr;
    MasterState* ms_h = nullptr;      // pinned
    PriceResult* pr = nullptr;
    PriceResult* pr_h = nullptr;      // pinned
    RowRec* rowrec = nullptr;
    Rec* parts = nullptr;
    Rec* upd_parts = nullptr;
    int64_t nparts = 0;
    Arrival* arr = nullptr;
    double* scalar = nullptr;
    double* scalar_h = nullptr;       // pinned
    int16_t* lv_stage_h = nullptr;    // pinned

    ~dao_ctx() {
        for (auto& b : bufs) if (b.p) (void)hipFree(b.p);
        if (ms_h) (void)hipHostFree(ms_h);
        if (pr_h) (void)hipHostFree(pr_h);
        if (scalar_h) (void)hipHostFree(scalar_h);
        if (lv_stage_h) (void)hipHostFree(lv_stage_h);
        if (pc_h) (void)hipHostFree(pc_h);
        if (batch_host) (void)hipHostFree(batch_host);
        for (auto e : prof_events) (void)hipEventDestroy(e);
        for (auto g : price_exec)
            if (g) (void)hipGraphExecDestroy(g);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }

    dao_status fail(dao_status s, std::string m) {
        err = std::move(m);
        return s;
    }

    int64_t elem_blocks(int64_t n) const {
        return std::max<int64_t>(1, std::min<int64_t>(ELEM_BLOCKS_MAX, (n + BLOCK - 1) / BLOCK));
    }
    // kernels that end in arrive_and_reduce: every workgroup's arrival takes
    // an agent-scope fence, whose cost grows with the workgroup count, so
    // these take at most REDUCE_BLOCKS_MAX workgroups of 4+ rows per thread
    int64_t reduce_blocks(int64_t n) const {
        return std::max<int64_t>(1, std::min<int64_t>(REDUCE_BLOCKS_MAX, (n + 4 * BLOCK - 1) / (4 * BLOCK)));
    }
    int64_t slab_blocks() const { return std::max<int64_t>(1, (nslices + SPB - 1) / SPB); }
    int64_t ap_blocks() const { return std::max<int64_t>(1, std::min<int64_t>(512, (Vpad + 255) / 256)); }
    bool ap_master() const { return opt.master == DAO_MASTER_APERTURE; }
    bool coop_master() const { return ap_master() && opt.persistent && coop_grid > 0; }
    int64_t price_blocks() const { return std::max<int64_t>(1, (R + BLOCK / WAVE - 1) / (BLOCK / WAVE)); }
    bool stage_x() const { return size_t(N) * tsize <= STAGE_LIMIT; }
    bool stage_x64() const { return size_t(N) * 8 <= STAGE_LIMIT; }
    size_t dir_lds() const {
        return ((size_t(N) * tsize + 15) & ~size_t(15)) + size_t(opt.max_apertures) * maxRB * 4;
    }
    bool stage_dir() const { return dir_lds() <= STAGE_LIMIT; }
};

#define HIPCHK(ctx, call)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return (ctx)->fail(DAO_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define LAUNCHCHK(ctx)                                                                        \
    do {                                                                                      \
        hipError_t e_ = hipGetLastError();                                                    \
        if (e_ != hipSuccess)                                                                 \
            return (ctx)->fail(DAO_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

namespace {

template <class P>
dao_status dev_alloc(dao_ctx* c, P** out, size_t bytes) {
    void* p = nullptr;
    bytes = std::max<size_t>(bytes, 16);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return c->fail(DAO_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    c->bufs.push_back(DevBuf{p, bytes});
    c->device_bytes += int64_t(bytes);
    *out = static_cast<P*>(p);
    return DAO_OK;
}

template <class P>
dao_status upload(dao_ctx* c, P** out, const void* host, size_t bytes) {
    dao_status s = dev_alloc(c, out, bytes);
    if (s != DAO_OK) return s;
    if (bytes) HIPCHK(c, hipMemcpyAsync(*out, host, bytes, hipMemcpyHostToDevice, c->stream));
    return DAO_OK;
}

template <class T>
std::vector<T> convert(const std::vector<double>& v) {
    std::vector<T> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = T(v[i]);
    return o;
}

// Device footprint predicted from the layout (checked against mem_cap before allocating).
int64_t predicted_bytes(const HostLayout& L, size_t ts, int kmax, const dao_options& opt) {
    const int64_t vs = opt.d_format != DAO_DFMT_NATIVE ? 2 + (opt.d_residual ? 2 : 0) : int64_t(ts);
    int64_t b = 0;
    b += (L.nslices + 1) * 4 + L.nslices * 4 + int64_t(L.slice_ptr.back()) * (vs + 2) + L.Vpad * 4;
    b += (L.N + 1) * 4 + L.nnz * (4 + vs) + (opt.d_format != DAO_DFMT_NATIVE ? L.N * 4 : 0);
    b += L.Vpad + L.V + int64_t(L.classes.size()) * sizeof(ObjClass) + int64_t(L.tau_int.size() + L.tau_ext.size()) * 8;
    b += int64_t(L.R) * 8 + (L.B + 1) * 4 + L.N * 12;
    b += L.Vpad * (8 + 3 * ts + 8) + L.N * (ts + 8 + ts + 8);
    b += int64_t(kmax) * (4 + 2 * 2 * L.max_rows_per_beam + 24);
    // FP16 D_K: 2 bytes, unless the selective residual keeps an FP32-sized
    // buffer; the automatic choice is counted at the native size (a bound)
    const int64_t dkb = (opt.dk_format == DAO_DFMT_F16 && ts == 4 && opt.d_residual != 2) ? 2 : int64_t(ts);
    b += int64_t(L.Vpad) * KS * dkb + L.N * ts + 512 * (KS + 1) * 8;
    b += int64_t(L.Vpad) / 32 * KS * 8;   // the persistent master's per-batch partials
    b += 2 * 8 * (L.nslices + 4096) * 4;   // the forward product's slice lists (a generous bound)
    b += sizeof(MasterState) + sizeof(PriceResult) + L.R * sizeof(RowRec) + 2 * ELEM_BLOCKS_MAX * sizeof(Rec) +
         sizeof(Arrival);
    return b;
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
template <class T>
SellView<T> sell_view(dao_ctx* c) {
    return SellView<T>{c->slice_ptr, c->slice_w, static_cast<const T*>(c->sell_val), c->sell_col,
                       c->nslices, static_cast<const __half*>(c->sell_lo)};
}

// Calls f(ValueTag<VT, LO>{}) with the device type of D's stored values and
// whether the FP16 residual is used (16-bit formats exist for FP32 only).
template <class V, bool L>
struct ValueTag {
    using VT = V;
    static constexpr bool LO = L;
};
template <class T, class F>
void with_values(const dao_ctx* c, F&& f) {
    if constexpr (std::is_same<T, float>::value) {
        // the FP16 residual: always (d_residual 1) or while the selective
        // policy asks for it (d_residual 2)
        const bool lo = c->opt.d_residual == 1 || (c->opt.d_residual == 2 && c->lo_now);
        if (c->opt.d_format == DAO_DFMT_F16) {
            if (lo)
                f(ValueTag<__half, true>{});
            else
                f(ValueTag<__half, false>{});
            return;
        }
        if (c->opt.d_format == DAO_DFMT_BF16) {
            if (lo)
                f(ValueTag<__hip_bfloat16, true>{});
            else
                f(ValueTag<__hip_bfloat16, false>{});
            return;
        }
    }
    f(ValueTag<T, false>{});
}

// d_out (T, caller order) = D x (x: T, caller order) through k_dose, in
// variant `var` (-1: the context's tuned one).  Every variant adds the same
// products in the same order.  Variant 2 reads x from device memory and
// exists for native values only (a 16-bit format folds its scale into the
// staged copy); variant 3 gives each workgroup twice the slices (each
// wavefront two chunks of its row).
// Grid of the whole-rows forward product with per_cu workgroups per compute unit.
inline int64_t rows_grid(const dao_ctx* c, int per_cu) {
    const int64_t need = (c->nslices + ROWS_THREADS / WAVE - 1) / (ROWS_THREADS / WAVE);
    return std::max<int64_t>(1, std::min<int64_t>(need, int64_t(std::max(1, c->ncu)) * per_cu));
}

template <class T>
void launch_dose(dao_ctx* c, const T* x, T* d_out, int var = -1) {
    if (var < 0) var = c->dose_var;
    with_values<T>(c, [&](auto tag) {
        using VT = typename decltype(tag)::VT;
        constexpr bool LO = decltype(tag)::LO;
        const bool stage = c->stage_x() && !(var == 2 && c->opt.d_format == DAO_DFMT_NATIVE);
        const size_t lds = stage ? c->N * sizeof(T) : 0;
        if (var == 0)
            k_dose<T, VT, LO, 0><<<c->slab_blocks(), SLAB_THREADS, lds, c->stream>>>(
                sell_view<VT>(c), c->perm, c->Vpad, x, int(c->N), stage, c->col_scale, d_out);
        else if (var == 3)
            k_dose<T, VT, LO, 0, 2 * SPB><<<(c->nslices + 2 * SPB - 1) / (2 * SPB), SLAB_THREADS, lds, c->stream>>>(
                sell_view<VT>(c), c->perm, c->Vpad, x, int(c->N), stage, c->col_scale, d_out);
        else if (var >= 7 && stage && c->slice_order[var - 7]) {
            // whole rows per lane, 2 or 4 workgroups per CU, balanced slice lists
            const int i = var - 7;
            k_dose_rows<T, VT, LO, 8, true><<<rows_grid(c, i == 0 ? 2 : 4), ROWS_THREADS, lds, c->stream>>>(
                sell_view<VT>(c), c->perm, c->Vpad, x, int(c->N), c->col_scale, d_out, c->slice_order[i],
                c->slice_rounds[i]);
        }
        else if (var >= 4 && var <= 6 && stage) {
            // whole rows per lane on a grid of 1, 2 or 4 workgroups per CU
            const int per_cu = var == 4 ? 1 : var == 5 ? 2 : 4;
            k_dose_rows<T, VT, LO><<<rows_grid(c, per_cu), ROWS_THREADS, lds, c->stream>>>(
                sell_view<VT>(c), c->perm, c->Vpad, x, int(c->N), c->col_scale, d_out);
        }
        else
            k_dose<T, VT, LO, 8><<<c->slab_blocks(), SLAB_THREADS, lds, c->stream>>>(
                sell_view<VT>(c), c->perm, c->Vpad, x, int(c->N), stage, c->col_scale, d_out);
    });
}

// g = D^T u (internal row order in, beamlet order out) through k_gradT with
// pf entries per thread in flight (-1: the context's tuned depth); the sums
// do not depend on pf.
template <class T, class UT, class Acc, class GT>
void launch_gradT(dao_ctx* c, const UT* u, GT* g, int pf = -1) {
    if (pf < 0) pf = c->gradT_pf;
    with_values<T>(c, [&](auto tag) {
        using VT = typename decltype(tag)::VT;
        constexpr bool LO = decltype(tag)::LO;
        const VT* cv = static_cast<const VT*>(c->csc_val);
        const __half* cl = static_cast<const __half*>(c->csc_lo);
        if (pf >= 16)
            k_gradT<VT, UT, Acc, GT, false, LO, 16><<<c->N, BLOCK, 0, c->stream>>>(
                c->csc_ptr, c->csc_row, cv, cl, u, g, nullptr, c->col_scale);
        else if (pf >= 8)
            k_gradT<VT, UT, Acc, GT, false, LO, 8><<<c->N, BLOCK, 0, c->stream>>>(
                c->csc_ptr, c->csc_row, cv, cl, u, g, nullptr, c->col_scale);
        else
            k_gradT<VT, UT, Acc, GT, false, LO, 4><<<c->N, BLOCK, 0, c->stream>>>(
                c->csc_ptr, c->csc_row, cv, cl, u, g, nullptr, c->col_scale);
    });
}

// Picks the fastest k_dose variant and k_gradT depth for this matrix by
// timing each a few times on the context's stream (inputs are zeros; every
// variant computes the same sums, so the choice changes time only).  The
// forward product's output takes a transient buffer of n_vox values.
template <class T>
dao_status tune_products(dao_ctx* c) {
    void* out = nullptr;
    HIPCHK(c, hipMalloc(&out, std::max<int64_t>(1, c->V) * sizeof(T)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    dao_status s = DAO_OK;
    auto fail = [&](hipError_t e) {
        s = c->fail(DAO_EDEVICE, std::string("product tuning: ") + hipGetErrorString(e));
    };
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he == hipSuccess) he = hipMemsetAsync(c->u, 0, c->Vpad * sizeof(T), c->stream);
    const bool native = c->opt.d_format == DAO_DFMT_NATIVE;
    const int pfs[3] = {4, 8, 16};
    constexpr int NDV = 9;   // forward variants: 0-3 slab forms, 4-8 whole rows per lane
    double best_d[NDV], best_g[3] = {1e30, 1e30, 1e30};
    for (double& b : best_d) b = 1e30;
    constexpr int REPS = 3, LAUNCHES = 8;
    auto time_one = [&](auto&& launch) -> double {
        launch();
        if (he == hipSuccess) he = hipEventRecord(e0, c->stream);
        for (int i = 0; i < LAUNCHES; ++i) launch();
        if (he == hipSuccess) he = hipEventRecord(e1, c->stream);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        return double(ms);
    };
    for (int r = 0; r < REPS && he == hipSuccess; ++r) {
        for (int v = 0; v < NDV; ++v)
            if ((native || v != 2) && (v < 4 || c->stage_x()))
                best_d[v] = std::min(best_d[v], time_one([&] {
                launch_dose<T>(c, static_cast<const T*>(c->dx), static_cast<T*>(out), v);
            }));
        for (int v = 0; v < 3; ++v)
            best_g[v] = std::min(best_g[v], time_one([&] {
                launch_gradT<T, T, T, T>(c, static_cast<const T*>(c->u), static_cast<T*>(c->g), pfs[v]);
            }));
    }
    if (he == hipSuccess) he = hipGetLastError();
    if (he != hipSuccess) fail(he);
    if (s == DAO_OK) {
        // a variant replaces the plain one only when clearly faster (2 %)
        c->dose_var = 0;
        for (int v = 1; v < NDV; ++v)
            if (best_d[v] < 0.98 * best_d[c->dose_var]) c->dose_var = v;
        int bg = 0;
        for (int v = 1; v < 3; ++v)
            if (best_g[v] < 0.98 * best_g[bg]) bg = v;
        c->gradT_pf = pfs[bg];
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(out);
    return s;
}

// Scratch of dao_price_noalloc: the per-row records, the result and the
// arrival counters of one pricing launch, for up to NOALLOC_MAX_ROWS MLC
// rows.  One copy per device (static device memory, held until the process
// ends); every call on a device shares it.  Host code never passes the
// array's name to a kernel: its device address is looked up once per device
// (hipGetSymbolAddress) and kept in g_scratch_addr.
constexpr size_t align256(size_t n) { return (n + 255) & ~size_t(255); }
constexpr int NOALLOC_MAX_ROWS = 4096;
constexpr size_t NOALLOC_ROWS_OFF = 0;
constexpr size_t NOALLOC_PR_OFF = align256(size_t(NOALLOC_MAX_ROWS) * sizeof(RowRec));
constexpr size_t NOALLOC_ARR_OFF = align256(NOALLOC_PR_OFF + sizeof(PriceResult));
constexpr size_t NOALLOC_BYTES = align256(NOALLOC_ARR_OFF + sizeof(Arrival));
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_addr;   // device -> address of its scratch copy

// Device address of the current device's scratch copy (looked up on first use).
dao_status scratch_address(unsigned char** out, std::string* err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = "hipGetDevice failed";
        return DAO_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return DAO_EDEVICE;
        }
        it = g_scratch_addr.emplace(dev, static_cast<unsigned char*>(ptr)).first;
    }
    *out = it->second;
    return DAO_OK;
}

PoolView pool_view(dao_ctx* c) {
    return PoolView{c->ap_beam, c->ap_lv, c->maxRB, c->blt_beam_d, c->blt_row_d, c->blt_pos_d,
                    c->beam_row0_d, c->row_start_d, int32_t(c->N)};
}

template <class T>
dao_status enqueue_cycle(dao_ctx* c) {
    const PoolView P = pool_view(c);
    const SellView<T> S = sell_view<T>(c);
    const size_t cls_b = sizeof(ObjClass) * c->ncls;
    const int nupd = int(c->slab_blocks());
    k_dir<T><<<1, 1024, c->stage_dir() ? c->dir_lds() : 0, c->stream>>>(
        P, static_cast<const T*>(c->g), c->y, c->p, c->gradk, static_cast<T*>(c->dx), c->ms, c->cgm, c->upd_parts,
        nupd, c->stage_dir());
    k_qstep<T><<<c->slab_blocks(), SLAB_THREADS, cls_b + (c->stage_x() ? c->N * sizeof(T) : 0), c->stream>>>(
        S, c->Vpad, static_cast<const T*>(c->dx), int(c->N), c->stage_x(), c->d, c->cls_int, c->classes,
        c->ncls, static_cast<T*>(c->q), c->parts, c->arr, c->ms, P, c->y, c->p, c->x64);
    for (int i = 0; i < c->opt.ls_slots; ++i)
        k_lseval<<<c->reduce_blocks(c->Vpad), BLOCK, 0, c->stream>>>(
            c->d, c->q, sizeof(T) == 8, c->cls_int, c->Vpad, c->classes, c->ncls, c->parts, c->arr, c->ms, P,
            c->y, c->p, c->x64);
    k_update<T><<<c->slab_blocks(), SLAB_THREADS, cls_b + (c->stage_x64() ? c->N * 8 : 0), c->stream>>>(
        S, c->Vpad, c->x64, int(c->N), c->stage_x64(), c->d, static_cast<const T*>(c->q), c->cls_int,
        c->classes, c->ncls, c->tau_int, static_cast<T*>(c->u), c->upd_parts, c->ms);
    k_gradT<T, T, T, T, true><<<c->N, BLOCK, 0, c->stream>>>(c->csc_ptr, c->csc_row,
                                                             static_cast<const T*>(c->csc_val), nullptr,
                                                             static_cast<const T*>(c->u),
                                                             static_cast<T*>(c->g), c->ms, nullptr);
    LAUNCHCHK(c);
    return DAO_OK;
}

// Event pair around one launch of the profiled kernel (when enabled).
dao_status prof_mark(dao_ctx* c, int kernel, bool before) {
    if (c->prof_kernel != kernel) return DAO_OK;
    if (c->prof_used == c->prof_events.size()) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c->prof_events.push_back(e);
    }
    (void)before;
    HIPCHK(c, hipEventRecord(c->prof_events[c->prof_used++], c->stream));
    return DAO_OK;
}

template <class T, class DT>
dao_status enqueue_cycle_ap_dt(dao_ctx* c) {
    if (c->Vpad % Batch<DT>::ROWS != 0) return c->fail(DAO_ESTATE, "padded rows not a multiple of the D_K batch");
    const int nb = int(c->ap_blocks());
    const DT* dk = static_cast<const DT*>(c->dk);
    const double dks = c->dk_scale;
    dao_status s;
#define MARK(k, b)                      \
    do {                                \
        s = prof_mark(c, k, b);         \
        if (s != DAO_OK) return s;      \
    } while (0)
    MARK(0, true);
    k_upd_ap<T, DT><<<nb, BLOCK, 0, c->stream>>>(dk, dks, c->Vpad, c->d, static_cast<const T*>(c->q), c->cls_int,
                                              c->classes, c->ncls, c->y, c->parts2, c->ms, c->pc, c->Vnz,
                                              c->tau_int);
    MARK(0, false);
    MARK(3, true);
    k_dir_ap<<<1, 1024, 0, c->stream>>>(c->parts2, nb, c->y, c->p, c->gradk, c->ms, c->cgm, c->pc);
    MARK(3, false);
    MARK(1, true);
    k_qstep_ap<T, DT><<<nb, BLOCK, 0, c->stream>>>(dk, dks, c->Vpad, c->d, c->cls_int, c->classes, c->ncls,
                                                static_cast<T*>(c->q), c->parts, c->arr, c->ms, c->y, c->p,
                                                c->pc, c->Vnz);
    MARK(1, false);
    for (int i = 0; i < c->opt.ls_slots; ++i) {
        MARK(2, true);
        k_lseval_ap<T><<<c->reduce_blocks(c->Vpad), BLOCK, 0, c->stream>>>(
            c->d, static_cast<const T*>(c->q), c->cls_int, c->Vpad, c->classes, c->ncls, c->parts, c->arr,
            c->ms, c->y, c->p, c->pc, c->Vnz);
        MARK(2, false);
    }
#undef MARK
    LAUNCHCHK(c);
    return DAO_OK;
}

template <class T>
dao_status enqueue_cycle_ap(dao_ctx* c) {
    if constexpr (std::is_same<T, float>::value)
        if (c->dk16) return enqueue_cycle_ap_dt<T, __half>(c);
    return enqueue_cycle_ap_dt<T, T>(c);
}

// Whether the persistent master keeps D_K on chip in the context type for a
// pool of K apertures (the same test its launch makes).
template <class T>
bool dk_on_chip(const dao_ctx* c, int K) {
    if (c->opt.persistent != 2 || c->coop_grid <= 0) return false;
    const int nc = (K + DKG<T>::EPL - 1) / DKG<T>::EPL;
    const int64_t rows = coop_batches_per_group<T>(c->Vpad, c->coop_grid) * Batch<T>::ROWS;
    return coop_lds_bytes<T>(rows, nc) <= size_t(c->coop_lds_max);
}

// Column k of the aperture dose matrix: D times the 0/1 indicator of aperture k.
// With dk_format DAO_DFMT_AUTO a plan starts with D_K in FP32 and moves it to
// FP16 (its columns rebuilt once) before the first column that would make the
// pool too large for the on-chip master form.
template <class T>
dao_status build_dk_column(dao_ctx* c, int k) {
    if (!c->ap_master()) return DAO_OK;
    if constexpr (std::is_same<T, float>::value) {
        if (c->opt.dk_format == DAO_DFMT_AUTO && !c->dk16 && !c->final_phase && !dk_on_chip<T>(c, k + 1)) {
            c->dk16 = true;
            c->dk_scale = c->dk16_scale;
            HIPCHK(c, hipMemsetAsync(c->dk, 0, size_t(c->Vpad) * KS * sizeof(T), c->stream));
            for (int j = 0; j < k; ++j) {
                const dao_status s = build_dk_column<T>(c, j);
                if (s != DAO_OK) return s;
            }
        }
    }
    k_ap_indicator<T><<<(c->N + BLOCK - 1) / BLOCK, BLOCK, 0, c->stream>>>(pool_view(c), k, static_cast<T*>(c->ind));
    with_values<T>(c, [&](auto tag) {
        using VT = typename decltype(tag)::VT;
        constexpr bool LO = decltype(tag)::LO;
        const size_t lds = c->stage_x() ? c->N * sizeof(T) : 0;
        if constexpr (std::is_same<T, float>::value) {
            if (c->dk16) {
                k_dk_column<T, VT, LO, __half><<<c->slab_blocks(), SLAB_THREADS, lds, c->stream>>>(
                    sell_view<VT>(c), c->Vpad, static_cast<const T*>(c->ind), int(c->N), c->stage_x(),
                    c->col_scale, k, static_cast<__half*>(c->dk), 1.0 / c->dk_scale);
                return;
            }
        }
        k_dk_column<T, VT, LO, T><<<c->slab_blocks(), SLAB_THREADS, lds, c->stream>>>(
            sell_view<VT>(c), c->Vpad, static_cast<const T*>(c->ind), int(c->N), c->stage_x(), c->col_scale, k,
            static_cast<T*>(c->dk), 1.0);
    });
    LAUNCHCHK(c);
    return DAO_OK;
}

// One cooperative launch runs the whole master solve.
template <class T, class DT>
dao_status run_master_coop_dt(dao_ctx* c, double tol, int max_steps) {
    if (c->Vpad % Batch<DT>::ROWS != 0) return c->fail(DAO_ESTATE, "padded rows not a multiple of the D_K batch");
    k_master_init_ap<<<1, 1, 0, c->stream>>>(c->ms, c->K, tol, max_steps);
    LAUNCHCHK(c);
    HIPCHK(c, hipMemsetAsync(c->coop, 0, sizeof(CoopSync), c->stream));
    CoopArgs<T> A{c->dk, c->dk_scale, c->Vpad, c->Vnz, c->d, static_cast<T*>(c->q), c->cls_int,
                  c->classes, c->ncls, c->y, c->p, c->gradk, c->cgm, c->tau_int, c->ms, c->coop_recs,
                  c->coop_bpart, c->coop, c->pc, c->prof_kernel == 4 ? 1 : 0};
    void* args[] = {&A};
    const bool prof = c->prof_kernel == 4;
    if (prof) {
        dao_status s = prof_mark(c, 4, true);
        if (s != DAO_OK) return s;
    }
    // the form: the workgroup's rows on chip when they fit, else d, q and
    // the classes on chip with D_K streamed, else everything streamed
    // (persistent 1 always streams everything)
    const int nc = (c->K + DKG<DT>::EPL - 1) / DKG<DT>::EPL;
    const int64_t rows = coop_batches_per_group<DT>(c->Vpad, c->coop_grid) * Batch<DT>::ROWS;
    const size_t lds = coop_lds_bytes<T>(rows, nc), lds_h = coop_hybrid_lds<T, DT>(rows);
    const bool chip_ok = c->opt.persistent == 2 && c->coop_lds_max > 0;
    if (chip_ok && lds <= size_t(c->coop_lds_max)) {
        HIPCHK(c, hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_master_coop<T, DT, COOP_CHIP>),
                                             dim3(c->coop_grid), dim3(COOP_THREADS), args, lds, c->stream));
        c->last_form = 2;
    } else if (chip_ok && lds_h <= size_t(c->coop_lds_max)) {
        HIPCHK(c, hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_master_coop<T, DT, COOP_HYBRID>),
                                             dim3(c->coop_grid), dim3(COOP_THREADS), args, lds_h, c->stream));
        c->last_form = 5;
    } else {
        HIPCHK(c, hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_master_coop<T, DT, COOP_STREAM>),
                                             dim3(c->coop_grid), dim3(COOP_THREADS), args, coop_stream_lds<DT>(),
                                             c->stream));
        c->last_form = 1;
    }
    if (prof) {
        dao_status s = prof_mark(c, 4, false);
        if (s != DAO_OK) return s;
    }
    HIPCHK(c, hipMemcpyAsync(c->ms_h, c->ms, sizeof(MasterState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->ms_h->stop_reason == 4 || !c->ms_h->done)
        return c->fail(DAO_EDEVICE, "persistent master: grid reduction timed out");
    c->last_steps = c->ms_h->steps;
    c->last_stop = c->ms_h->stop_reason;
    return DAO_OK;
}

template <class T>
dao_status run_master_coop(dao_ctx* c, double tol, int max_steps) {
    if constexpr (std::is_same<T, float>::value)
        if (c->dk16) return run_master_coop_dt<T, __half>(c, tol, max_steps);
    return run_master_coop_dt<T, T>(c, tol, max_steps);
}

template <class T>
dao_status run_master(dao_ctx* c, double tol, int max_steps) {
    if (c->coop_master()) return run_master_coop<T>(c, tol, max_steps);
    if (c->ap_master())
        k_master_init_ap<<<1, 1, 0, c->stream>>>(c->ms, c->K, tol, max_steps);
    else
        k_master_init<<<1, 1, 0, c->stream>>>(c->ms, c->K, tol, max_steps);
    LAUNCHCHK(c);
    // every cycle either finishes a step or advances a line search by
    // ls_slots evaluations; bound the cycles so a stuck state cannot spin
    const int64_t max_cycles =
        int64_t(max_steps + 1) * (LS_MAX_ITER / std::max(1, c->opt.ls_slots) + 2) + 16;
    int64_t cycles = 0;
    // the previous solve's step count predicts this one (rounds of one plan
    // grow slowly); after that first guess, grow geometrically
    int chunk = std::max(2, std::min(max_steps + 1, int(0.9 * c->last_steps)));
    for (;;) {
        for (int i = 0; i < chunk; ++i) {
            dao_status s = c->ap_master() ? enqueue_cycle_ap<T>(c) : enqueue_cycle<T>(c);
            if (s != DAO_OK) return s;
        }
        cycles += chunk;
        HIPCHK(c, hipMemcpyAsync(c->ms_h, c->ms, sizeof(MasterState), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (c->ms_h->done) break;
        if (cycles > max_cycles) return c->fail(DAO_EDEVICE, "master state machine made no progress");
        chunk = std::max(4, std::min(32, (max_steps - c->ms_h->steps) / 4 + 4));
    }
    c->last_steps = c->ms_h->steps;
    c->last_stop = c->ms_h->stop_reason;
    c->last_form = 0;
    return DAO_OK;
}

// u, u64 and F from the master dose; g (ctx type) from u.
template <class T>
dao_status refresh_gradient(dao_ctx* c) {
    k_objective_int<T><<<c->reduce_blocks(c->Vpad), BLOCK, 0, c->stream>>>(
        c->d, c->cls_int, c->Vpad, c->classes, c->ncls, static_cast<T*>(c->u), c->u64, c->parts, c->arr, c->ms);
    launch_gradT<T, T, T, T>(c, static_cast<const T*>(c->u), static_cast<T*>(c->g));
    LAUNCHCHK(c);
    return DAO_OK;
}

PriceGeom price_geom(dao_ctx* c) {
    return PriceGeom{c->row_start_d, c->row_len_d, c->beam_row0_d, c->R, c->B};
}

// One pricing launch with the given scratch (row records, result, arrival
// counters), then the result to the host.
dao_status price_with(dao_ctx* c, const double* g, RowRec* rows, PriceResult* pr, Arrival* arr, int32_t* beam,
                      int16_t* leaves, double* rc, double* gap) {
    k_price<<<c->price_blocks(), BLOCK, 0, c->stream>>>(price_geom(c), g, rows, pr, arr);
    LAUNCHCHK(c);
    HIPCHK(c, hipMemcpyAsync(c->pr_h, pr, sizeof(PriceResult), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (beam) *beam = c->pr_h->beam;
    if (leaves) std::memcpy(leaves, c->pr_h->leaves, sizeof(int16_t) * 2 * c->pr_h->n_rows);
    if (rc) *rc = c->pr_h->rc;
    if (gap) *gap = c->pr_h->gap;
    return DAO_OK;
}

dao_status price_on(dao_ctx* c, const double* g, int32_t* beam, int16_t* leaves, double* rc,
                    double* gap) {
    return price_with(c, g, c->rowrec, c->pr, c->arr, beam, leaves, rc, gap);
}

// The master dose recomputed from the intensities in FP64 (x = A y, then
// d = D x with FP64 products and sums), replacing the master's incremental
// dose.
template <class T>
dao_status refresh_dose_exact(dao_ctx* c) {
    k_pool_x<<<(c->N + BLOCK - 1) / BLOCK, BLOCK, 0, c->stream>>>(pool_view(c), c->K, c->y, c->x64);
    with_values<T>(c, [&](auto tag) {
        using VT = typename decltype(tag)::VT;
        constexpr bool LO = decltype(tag)::LO;
        k_dose_exact<VT, LO><<<c->slab_blocks(), SLAB_THREADS, c->stage_x64() ? c->N * 8 : 0, c->stream>>>(
            sell_view<VT>(c), c->Vpad, c->x64, int(c->N), c->stage_x64(), c->col_scale, c->tau_int, c->d);
    });
    LAUNCHCHK(c);
    return DAO_OK;
}

// u, u64, F and g (ctx type) after the master dose changed outside a master
// solve.
template <class T>
dao_status refresh_objective(dao_ctx* c) {
    k_objective_int<T><<<c->reduce_blocks(c->Vpad), BLOCK, 0, c->stream>>>(
        c->d, c->cls_int, c->Vpad, c->classes, c->ncls, static_cast<T*>(c->u), c->u64, c->parts, c->arr, c->ms);
    if (!c->ap_master()) launch_gradT<T, T, T, T>(c, static_cast<const T*>(c->u), static_cast<T*>(c->g));
    LAUNCHCHK(c);
    return DAO_OK;
}

// The pricing launches after x = A y: d = D x in FP64, grad F and F, the
// FP64 prices, the pricing scan and the result's copy to the host.  Every
// argument is fixed per context (and per residual setting), so the sequence
// can be captured once as a graph.
template <class T>
dao_status enqueue_price_tail(dao_ctx* c) {
    with_values<T>(c, [&](auto tag) {
        using VT = typename decltype(tag)::VT;
        constexpr bool LO = decltype(tag)::LO;
        k_dose_exact<VT, LO><<<c->slab_blocks(), SLAB_THREADS, c->stage_x64() ? c->N * 8 : 0, c->stream>>>(
            sell_view<VT>(c), c->Vpad, c->x64, int(c->N), c->stage_x64(), c->col_scale, c->tau_int, c->d);
    });
    dao_status s = refresh_objective<T>(c);
    if (s != DAO_OK) return s;
    launch_gradT<T, double, double, double>(c, c->u64, c->g64);
    k_price<<<c->price_blocks(), BLOCK, 0, c->stream>>>(price_geom(c), c->g64, c->rowrec, c->pr, c->arr);
    LAUNCHCHK(c);
    HIPCHK(c, hipMemcpyAsync(c->pr_h, c->pr, sizeof(PriceResult), hipMemcpyDeviceToHost, c->stream));
    return DAO_OK;
}

// FP64 prices at the current intensities: the dose is first recomputed as
// D (A y) in FP64, then g64 = D^T grad F(d) with FP64 sums.  With
// dao_options.graphs the launches after x = A y replay a graph captured on
// the context stream at first use (one per residual setting).
template <class T>
dao_status price_current(dao_ctx* c, int32_t* beam, int16_t* leaves, double* rc, double* gap) {
    k_pool_x<<<(c->N + BLOCK - 1) / BLOCK, BLOCK, 0, c->stream>>>(pool_view(c), c->K, c->y, c->x64);
    LAUNCHCHK(c);
    dao_status s = DAO_OK;
    if (c->opt.graphs) {
        const int gi = (c->opt.d_residual == 1 || (c->opt.d_residual == 2 && c->lo_now)) ? 1 : 0;
        if (!c->price_exec[gi]) {
            // recorded on a stream of the context's own: nothing runs during
            // the capture, and the caller's stream may be the null stream
            if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
            HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            const hipStream_t run_stream = c->stream;
            c->stream = c->cap_stream;
            s = enqueue_price_tail<T>(c);
            c->stream = run_stream;
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
            if (s != DAO_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return s;
            }
            HIPCHK(c, e);
            const hipError_t ei = hipGraphInstantiate(&c->price_exec[gi], graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIPCHK(c, ei);
        }
        HIPCHK(c, hipGraphLaunch(c->price_exec[gi], c->stream));
    } else {
        s = enqueue_price_tail<T>(c);
        if (s != DAO_OK) return s;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (beam) *beam = c->pr_h->beam;
    if (leaves) std::memcpy(leaves, c->pr_h->leaves, sizeof(int16_t) * 2 * c->pr_h->n_rows);
    if (rc) *rc = c->pr_h->rc;
    if (gap) *gap = c->pr_h->gap;
    return DAO_OK;
}

template <class T>
dao_status reset_state(dao_ctx* c) {
    const int64_t eb = c->elem_blocks(c->Vpad);
    // a new pool starts in the fast form of the selective residual and in
    // the starting storage of D_K
    const bool dk_prev = c->dk16;
    c->lo_now = false;
    c->final_phase = false;
    c->reprices = 0;
    c->dk16 = c->dk16_base;
    c->dk_scale = c->dk16 ? c->dk16_scale : 1.0;
    // columns of one storage are about to be written over those of the
    // other (the selective residual's final phase, the automatic storage's
    // switch; both keep an FP32-sized buffer): clear it, so that no slot
    // beyond the pool holds a stale value (the products multiply every slot
    // of a row's last vector by 0)
    if (c->ap_master() && c->dk16 != dk_prev)
        HIPCHK(c, hipMemsetAsync(c->dk, 0, size_t(c->Vpad) * KS * sizeof(T), c->stream));
    // zero dose; the master keeps d - tau
    k_neg_or_zero<<<eb, BLOCK, 0, c->stream>>>(c->tau_int, c->Vpad, c->d);
    k_fill<double><<<1, BLOCK, 0, c->stream>>>(c->y, c->opt.max_apertures, 0.0);
    k_clear_steps<<<1, 1, 0, c->stream>>>(c->ms);
    LAUNCHCHK(c);
    c->K = 0;
    c->pool_beam.clear();
    c->pool_lv.clear();
    return refresh_gradient<T>(c);
}

dao_status check_aperture(dao_ctx* c, int32_t beam, const int16_t* leaves) {
    if (beam < 0 || beam >= c->B) return c->fail(DAO_EINVAL, "aperture beam out of range");
    if (!leaves) return c->fail(DAO_EINVAL, "null leaves");
    for (int r = c->beam_row0[beam]; r < c->beam_row0[beam + 1]; ++r) {
        const int lr = r - c->beam_row0[beam];
        const int L = leaves[2 * lr], Rr = leaves[2 * lr + 1];
        if (L < 0 || Rr > c->row_len[r] || L > Rr || (L == Rr && L != 0))
            return c->fail(DAO_EINVAL, "malformed leaf pair in row " + std::to_string(lr));
    }
    return DAO_OK;
}

void mirror_add(dao_ctx* c, int32_t beam, const int16_t* leaves) {
    c->pool_beam.push_back(beam);
    const int nr = c->rows_per_beam[beam];
    for (int i = 0; i < c->maxRB; ++i) {
        c->pool_lv.push_back(i < nr ? leaves[2 * i] : int16_t(0));
        c->pool_lv.push_back(i < nr ? leaves[2 * i + 1] : int16_t(0));
    }
}

bool in_pool(dao_ctx* c, int32_t beam, const int16_t* leaves) {
    const int nr = c->rows_per_beam[beam];
    for (size_t k = 0; k < c->pool_beam.size(); ++k) {
        if (c->pool_beam[k] != beam) continue;
        const int16_t* lv = &c->pool_lv[k * 2 * c->maxRB];
        if (std::equal(lv, lv + 2 * nr, leaves)) return true;
    }
    return false;
}

// Grid and on-chip LDS budget of the persistent master for D_K storage DT
// (one co-resident workgroup per compute unit).  Sets coop_grid (0: the
// device cannot run it), coop_lds_max and batch_ok.
template <class T, class DT>
hipError_t setup_coop(dao_ctx* c, int dev, int coop, int ncu) {
    int occ = 0;
    c->coop_lds_max = 0;
    c->batch_ok = false;
    c->coop_grid = 0;
    // the streaming form's dynamic LDS (the q pass's row partials)
    constexpr int slds = int(coop_stream_lds<DT>());
    for (const void* fn : {reinterpret_cast<const void*>(&k_master_coop<T, DT, COOP_STREAM>),
                           reinterpret_cast<const void*>(&k_master_batch<T, DT, COOP_STREAM>)}) {
        const hipError_t ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, slds);
        if (ea != hipSuccess) {
            (void)hipGetLastError();
            return hipSuccess;   // no persistent master on this device
        }
    }
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &occ, reinterpret_cast<const void*>(&k_master_coop<T, DT, COOP_STREAM>), COOP_THREADS, slds);
    if (e != hipSuccess) return e;
    if (coop && occ > 0 && ncu > 0) {
        c->coop_grid = std::min(ncu, MAX_COOP_GRID);   // one co-resident workgroup per compute unit
        // on-chip variant: as much dynamic LDS as the device grants one
        // workgroup beyond the kernel's static LDS, if one per CU still fits
        int lds_max = 0;
        e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess) return e;
        // the kernels' own static LDS (the largest of the single and the
        // batched launch in the two forms with rows on chip), rounded up to 1 KB
        int stat = 0;
        for (const void* fn : {reinterpret_cast<const void*>(&k_master_coop<T, DT, COOP_CHIP>),
                               reinterpret_cast<const void*>(&k_master_batch<T, DT, COOP_CHIP>),
                               reinterpret_cast<const void*>(&k_master_coop<T, DT, COOP_HYBRID>),
                               reinterpret_cast<const void*>(&k_master_batch<T, DT, COOP_HYBRID>)}) {
            hipFuncAttributes fa{};
            if (hipFuncGetAttributes(&fa, fn) == hipSuccess) stat = std::max(stat, int(fa.sharedSizeBytes));
            else stat = std::max(stat, 32 * 1024);
        }
        const int want = lds_max - ((stat + 1023) / 1024) * 1024;
        if (want > 0 &&
            hipFuncSetAttribute(reinterpret_cast<const void*>(&k_master_coop<T, DT, COOP_CHIP>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, want) == hipSuccess &&
            hipFuncSetAttribute(reinterpret_cast<const void*>(&k_master_coop<T, DT, COOP_HYBRID>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, want) == hipSuccess) {
            int occ2 = 0, occ5 = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &occ2, reinterpret_cast<const void*>(&k_master_coop<T, DT, COOP_CHIP>), COOP_THREADS, want) ==
                    hipSuccess &&
                occ2 >= 1 &&
                hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &occ5, reinterpret_cast<const void*>(&k_master_coop<T, DT, COOP_HYBRID>), COOP_THREADS, want) ==
                    hipSuccess &&
                occ5 >= 1)
                c->coop_lds_max = want;
        }
        (void)hipGetLastError();
        // the batched launch: same resources, both variants
        int occ3 = 0, occ4 = 0;
        c->batch_ok =
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ3, reinterpret_cast<const void*>(&k_master_batch<T, DT, COOP_STREAM>), COOP_THREADS,
                coop_stream_lds<DT>()) == hipSuccess &&
            occ3 >= 1;
        int occ6 = 0;
        if (c->batch_ok && c->coop_lds_max > 0 &&
            !(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_master_batch<T, DT, COOP_CHIP>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, c->coop_lds_max) == hipSuccess &&
              hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &occ4, reinterpret_cast<const void*>(&k_master_batch<T, DT, COOP_CHIP>), COOP_THREADS,
                  c->coop_lds_max) == hipSuccess &&
              occ4 >= 1 &&
              hipFuncSetAttribute(reinterpret_cast<const void*>(&k_master_batch<T, DT, COOP_HYBRID>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, c->coop_lds_max) == hipSuccess &&
              hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &occ6, reinterpret_cast<const void*>(&k_master_batch<T, DT, COOP_HYBRID>), COOP_THREADS,
                  c->coop_lds_max) == hipSuccess &&
              occ6 >= 1))
            c->batch_ok = false;
        (void)hipGetLastError();
    }
    return hipSuccess;
}

// f(a, b) over [0, n) split into contiguous ranges of at least `grain`
// items, on up to 16 host threads (the 16-bit encode of a large matrix).
template <class F>
void parallel_ranges(int64_t n, int64_t grain, F&& f) {
    const int64_t hc = std::max<int64_t>(1, int64_t(std::thread::hardware_concurrency()));
    const int64_t nt = std::min<int64_t>({16, hc, std::max<int64_t>(1, n / std::max<int64_t>(1, grain))});
    if (nt <= 1) {
        f(int64_t(0), n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t per = (n + nt - 1) / nt;
    for (int64_t a = 0; a < n; a += per) {
        const int64_t b = std::min(n, a + per);
        th.emplace_back([&f, a, b] { f(a, b); });
    }
    for (auto& t : th) t.join();
}

template <class T>
dao_status create_typed(dao_ctx* c, const HostLayout& L) {
    dao_status s;
#define TRY(x)            \
    do {                  \
        s = (x);          \
        if (s != DAO_OK) return s; \
    } while (0)
    const size_t ts = sizeof(T);
    TRY(upload(c, &c->slice_ptr, L.slice_ptr.data(), L.slice_ptr.size() * 4));
    TRY(upload(c, &c->slice_w, L.slice_w.data(), L.slice_w.size() * 4));
    const int fmt = c->opt.d_format;
    if (fmt == DAO_DFMT_NATIVE) {
        std::vector<T> v = convert<T>(L.sell_val);
        TRY(upload(c, &c->sell_val, v.data(), v.size() * ts));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        // 16-bit value / per-beamlet scale (+ FP16 residual)
        const bool res = c->opt.d_residual != 0;
        std::vector<uint16_t> hi(L.sell_val.size()), lo(res ? L.sell_val.size() : 0);
        parallel_ranges(int64_t(hi.size()), int64_t(1) << 18, [&](int64_t a, int64_t b) {
            for (int64_t e = a; e < b; ++e)
                encode_value(fmt, L.sell_val[e] / double(L.col_scale[L.sell_col[e]]), &hi[e], res ? &lo[e] : nullptr);
        });
        TRY(upload(c, &c->sell_val, hi.data(), hi.size() * 2));
        if (res) TRY(upload(c, &c->sell_lo, lo.data(), lo.size() * 2));
        TRY(upload(c, &c->col_scale, L.col_scale.data(), L.col_scale.size() * 4));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    TRY(upload(c, &c->sell_col, L.sell_col.data(), L.sell_col.size() * 2));
    TRY(upload(c, &c->perm, L.perm.data(), L.perm.size() * 4));
    TRY(upload(c, &c->csc_ptr, L.csc_ptr.data(), L.csc_ptr.size() * 4));
    TRY(upload(c, &c->csc_row, L.csc_row.data(), L.csc_row.size() * 4));
    if (fmt == DAO_DFMT_NATIVE) {
        std::vector<T> v = convert<T>(L.csc_val);
        TRY(upload(c, &c->csc_val, v.data(), v.size() * ts));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        const bool res = c->opt.d_residual != 0;
        std::vector<uint16_t> hi(L.csc_val.size()), lo(res ? L.csc_val.size() : 0);
        parallel_ranges(L.N, 32, [&](int64_t a, int64_t b) {
            for (int64_t i = a; i < b; ++i)
                for (int32_t e = L.csc_ptr[i]; e < L.csc_ptr[i + 1]; ++e)
                    encode_value(fmt, L.csc_val[e] / double(L.col_scale[i]), &hi[e], res ? &lo[e] : nullptr);
        });
        TRY(upload(c, &c->csc_val, hi.data(), hi.size() * 2));
        if (res) TRY(upload(c, &c->csc_lo, lo.data(), lo.size() * 2));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    TRY(upload(c, &c->cls_int, L.cls_int.data(), L.cls_int.size()));
    TRY(upload(c, &c->cls_ext, L.cls_ext.data(), L.cls_ext.size()));
    TRY(upload(c, &c->classes, L.classes.data(), L.classes.size() * sizeof(ObjClass)));
    if (!L.tau_int.empty()) {
        TRY(upload(c, &c->tau_int, L.tau_int.data(), L.tau_int.size() * 8));
        TRY(upload(c, &c->tau_ext, L.tau_ext.data(), L.tau_ext.size() * 8));
    }
    TRY(upload(c, &c->row_start_d, L.row_start.data(), L.row_start.size() * 4));
    TRY(upload(c, &c->row_len_d, L.row_len.data(), L.row_len.size() * 4));
    TRY(upload(c, &c->beam_row0_d, L.beam_row0.data(), L.beam_row0.size() * 4));
    TRY(upload(c, &c->blt_beam_d, L.blt_beam.data(), L.blt_beam.size() * 4));
    TRY(upload(c, &c->blt_row_d, L.blt_row.data(), L.blt_row.size() * 4));
    TRY(upload(c, &c->blt_pos_d, L.blt_pos.data(), L.blt_pos.size() * 4));
    TRY(dev_alloc(c, &c->d, c->Vpad * 8));
    TRY(dev_alloc(c, &c->q, c->Vpad * ts));
    TRY(dev_alloc(c, &c->u, c->Vpad * ts));
    TRY(dev_alloc(c, &c->u64, c->Vpad * 8));
    if (c->opt.d_residual == 2) {
        TRY(dev_alloc(c, &c->gabs64, c->N * 8));
        TRY(dev_alloc(c, &c->uabs64, c->Vpad * 8));
    }
    TRY(dev_alloc(c, &c->ug, c->Vpad * ts));
    TRY(dev_alloc(c, &c->g, c->N * ts));
    TRY(dev_alloc(c, &c->g64, c->N * 8));
    TRY(dev_alloc(c, &c->dx, c->N * ts));
    TRY(dev_alloc(c, &c->x64, c->N * 8));
    const int km = c->opt.max_apertures;
    TRY(dev_alloc(c, &c->ap_beam, km * 4));
    TRY(dev_alloc(c, &c->ap_lv, size_t(km) * c->maxRB * 2 * 2));
    TRY(dev_alloc(c, &c->y, km * 8));
    TRY(dev_alloc(c, &c->p, km * 8));
    TRY(dev_alloc(c, &c->cgm, sizeof(CgMem)));
    TRY(dev_alloc(c, &c->gradk, km * 8));
    TRY(dev_alloc(c, &c->ms, sizeof(MasterState)));
    TRY(dev_alloc(c, &c->pr, sizeof(PriceResult)));
    TRY(dev_alloc(c, &c->rowrec, std::max<int64_t>(1, c->R) * sizeof(RowRec)));
    {
        // this device's copy of the static scratch of dao_price_noalloc
        std::string e;
        if (scratch_address(&c->scratch_dev, &e) != DAO_OK) return c->fail(DAO_EDEVICE, e);
    }
    c->nparts = std::max<int64_t>({c->slab_blocks(), c->elem_blocks(c->Vpad), c->elem_blocks(c->V)});
    TRY(dev_alloc(c, &c->parts, c->nparts * sizeof(Rec)));
    TRY(dev_alloc(c, &c->upd_parts, c->slab_blocks() * sizeof(Rec)));
    TRY(dev_alloc(c, &c->arr, sizeof(Arrival)));
    TRY(dev_alloc(c, &c->pc, sizeof(ProfCounters)));
    // storage of D_K: FP16 on request, or (DAO_DFMT_AUTO) where the master
    // cannot keep it on chip
    constexpr bool f32 = std::is_same<T, float>::value;
    c->dk16 = f32 && c->ap_master() && c->opt.dk_format == DAO_DFMT_F16;
    // DAO_DFMT_AUTO: without the persistent launch the per-phase kernels
    // always stream D_K, so FP16 from the start; otherwise a plan starts in
    // FP32 and moves to FP16 when the pool outgrows the on-chip form
    const bool dk_auto = f32 && c->ap_master() && c->opt.dk_format == DAO_DFMT_AUTO;
    if (dk_auto && !c->opt.persistent) c->dk16 = true;
    if (c->ap_master() && c->opt.persistent) {
        int dev = 0, coop = 0, ncu = 0;
        HIPCHK(c, hipGetDevice(&dev));
        c->device = dev;
        HIPCHK(c, hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
        HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        if constexpr (f32) {
            if ((c->dk16 && c->opt.d_residual == 2) || dk_auto) {
                // both storages run: keep the smaller on-chip budget
                HIPCHK(c, (setup_coop<T, T>(c, dev, coop, ncu)));
                const int lds_f = c->coop_lds_max;
                const bool ok_f = c->batch_ok;
                HIPCHK(c, (setup_coop<T, __half>(c, dev, coop, ncu)));
                c->coop_lds_max = std::min(c->coop_lds_max, lds_f);
                c->batch_ok = c->batch_ok && ok_f;
            } else if (c->dk16) {
                HIPCHK(c, (setup_coop<T, __half>(c, dev, coop, ncu)));
            } else {
                HIPCHK(c, (setup_coop<T, T>(c, dev, coop, ncu)));
            }
        } else {
            HIPCHK(c, (setup_coop<T, T>(c, dev, coop, ncu)));
        }
        if (c->coop_grid > 0) {
            (void)hipGetLastError();
            TRY(dev_alloc(c, &c->coop, sizeof(CoopSync)));
            TRY(dev_alloc(c, &c->coop_recs, 2 * size_t(c->coop_grid) * RECW * sizeof(double)));
            // batches of at least 32 rows
            TRY(dev_alloc(c, &c->coop_bpart, size_t(c->Vpad / 32) * KS * sizeof(double)));
        }
    }
    // FP16 storage of D_K: values over the largest entry of D (every D_K
    // entry is a sum of D entries, so the stored values stay well inside
    // FP16's range)
    c->dk16_base = c->dk16;
    if (c->dk16 || dk_auto) {
        float mx = 0.0f;
        for (float v : L.col_scale) mx = std::max(mx, v);
        c->dk16_scale = mx > 0.0f ? double(mx) : 1.0;
    }
    c->dk_scale = c->dk16 ? c->dk16_scale : 1.0;
    // bytes per stored D_K value; the selective residual switches D_K to FP32
    // for the final rounds, so its buffer holds FP32 values
    const size_t dkb = (c->dk16 && c->opt.d_residual != 2 && !(dk_auto && c->opt.persistent)) ? sizeof(__half) : ts;
    if (c->ap_master()) {
        // D_K is stored in blocks of one batch of rows; the padded row count
        // (whole slices) is a whole number of blocks in every storage type
        static_assert(SLICE % Batch<float>::ROWS == 0 && SLICE % Batch<double>::ROWS == 0 &&
                          SLICE % Batch<__half>::ROWS == 0,
                      "D_K blocks tile the padded rows");
        TRY(dev_alloc(c, &c->dk, size_t(c->Vpad) * KS * dkb));
        TRY(dev_alloc(c, &c->ind, c->N * ts));
        TRY(dev_alloc(c, &c->parts2, c->ap_blocks() * (KS + 1) * sizeof(double)));
    }
    TRY(dev_alloc(c, &c->scalar, 16));
#undef TRY
    HIPCHK(c, hipHostMalloc((void**)&c->ms_h, sizeof(MasterState), hipHostMallocDefault));
    HIPCHK(c, hipHostMalloc((void**)&c->pr_h, sizeof(PriceResult), hipHostMallocDefault));
    HIPCHK(c, hipHostMalloc((void**)&c->scalar_h, 16, hipHostMallocDefault));
    HIPCHK(c, hipHostMalloc((void**)&c->lv_stage_h, size_t(c->maxRB) * 4 + 16, hipHostMallocDefault));
    HIPCHK(c, hipHostMalloc((void**)&c->pc_h, sizeof(ProfCounters), hipHostMallocDefault));
    HIPCHK(c, hipMemsetAsync(c->pc, 0, sizeof(ProfCounters), c->stream));
    std::memset(c->ms_h, 0, sizeof(MasterState));
    c->ms_h->done = 1;
    c->ms_h->refresh_every = c->opt.refresh_every;
    c->ms_h->conj = c->opt.direction == DAO_DIR_CONJUGATE ? 1 : 0;
    c->ms_h->F_const = c->F_const;
    HIPCHK(c, hipMemcpyAsync(c->ms, c->ms_h, sizeof(MasterState), hipMemcpyHostToDevice, c->stream));
    std::memset(c->pr_h, 0, sizeof(PriceResult));
    HIPCHK(c, hipMemcpyAsync(c->pr, c->pr_h, sizeof(PriceResult), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->arr, 0, sizeof(Arrival), c->stream));
    if (c->ap_master()) HIPCHK(c, hipMemsetAsync(c->dk, 0, size_t(c->Vpad) * KS * dkb, c->stream));
    HIPCHK(c, hipMemsetAsync(c->ap_lv, 0, size_t(km) * c->maxRB * 4, c->stream));
    HIPCHK(c, hipMemsetAsync(c->ap_beam, 0, km * 4, c->stream));
    HIPCHK(c, hipMemsetAsync(c->p, 0, km * 8, c->stream));
    HIPCHK(c, hipMemsetAsync(c->q, 0, c->Vpad * ts, c->stream));
    HIPCHK(c, hipMemsetAsync(c->dx, 0, c->N * ts, c->stream));
    {
        int dev = 0;
        HIPCHK(c, hipGetDevice(&dev));
        HIPCHK(c, hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, dev));
    }
    // balanced slice lists of the whole-rows forward product (variants 7 and 8:
    // 2 and 4 workgroups per CU), for this device's compute units
    if (c->stage_x() && c->nslices > 0) {
        for (int i = 0; i < 2; ++i) {
            std::vector<int32_t> order;
            int rounds = 0;
            balanced_slice_order(L.slice_w, rows_grid(c, i == 0 ? 2 : 4) * (ROWS_THREADS / WAVE), order, rounds);
            const dao_status su = upload(c, &c->slice_order[i], order.data(), order.size() * 4);
            if (su != DAO_OK) return su;
            c->slice_rounds[i] = rounds;
        }
    }
    c->dose_var = c->opt.dose_variant;
    if (c->dose_var >= 4 && !c->stage_x()) c->dose_var = 0;   // the row form stages x
    c->gradT_pf = c->opt.gradient_depth;
    if (c->opt.product_tune) {
        s = tune_products<T>(c);
        if (s != DAO_OK) return s;
    }
    s = reset_state<T>(c);
    if (s != DAO_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DAO_OK;
}

template <class T>
dao_status dose_typed(dao_ctx* c, const void* x, void* d) {
    k_fill<T><<<c->elem_blocks(c->V), BLOCK, 0, c->stream>>>(static_cast<T*>(d), c->V, T(0));
    launch_dose<T>(c, static_cast<const T*>(x), static_cast<T*>(d));
    LAUNCHCHK(c);
    return DAO_OK;
}

template <class T>
dao_status gradient_typed(dao_ctx* c, const void* d, void* g, double* F) {
    const T* dd = static_cast<const T*>(d);
    k_objective_ext<T><<<c->reduce_blocks(c->V), BLOCK, 0, c->stream>>>(dd, c->cls_ext, c->V, c->classes, c->ncls,
                                                                         c->tau_ext, c->parts, c->arr, c->scalar);
    k_gather_grad<T><<<c->elem_blocks(c->Vpad), BLOCK, 0, c->stream>>>(dd, c->perm, c->cls_int, c->Vpad,
                                                                        c->classes, c->tau_int,
                                                                        static_cast<T*>(c->ug));
    launch_gradT<T, T, T, T>(c, static_cast<const T*>(c->ug), static_cast<T*>(g));
    LAUNCHCHK(c);
    HIPCHK(c, hipMemcpyAsync(c->scalar_h, c->scalar, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (F) *F = c->scalar_h[0];
    return DAO_OK;
}

// Mean device time of `iters` back-to-back launches of one product kernel,
// measured with HIP events on the context stream.  Inputs are the master's
// current vectors; outputs go to scratch buffers.
template <class T>
dao_status time_product_typed(dao_ctx* c, int kernel, int iters, double* us, bool warm = true) {
    if (!c->vscratch) {   // k_dose scatters to caller order: V entries
        dao_status s = dev_alloc(c, &c->vscratch, size_t(c->V) * sizeof(T));
        if (s != DAO_OK) return s;
    }
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    auto launch = [&]() {
        if (kernel == 0)
            launch_dose<T>(c, static_cast<const T*>(c->dx), static_cast<T*>(c->vscratch));
        else
            launch_gradT<T, T, T, T>(c, static_cast<const T*>(c->u), static_cast<T*>(c->dx));
    };
    if (warm) launch();
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int i = 0; i < iters; ++i) launch();
    HIPCHK(c, hipEventRecord(e1, c->stream));
    LAUNCHCHK(c);
    HIPCHK(c, hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *us = 1e3 * double(ms) / iters;
    return DAO_OK;
}

// Reads the whole scrub buffer (clean lines displace D and the vectors from
// the caches without leaving dirty lines for the timed launch to write
// back).  The store only keeps the loads alive: it happens when a thread's
// XOR of its words equals `never`, which the caller picks so that it does
// not, and it would only change the scrub buffer.
__global__ void k_scrub(uint4* __restrict__ p, int64_t n, uint32_t never) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    uint32_t x = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint4 v = p[i];
        x ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (x == never && x != 0u) p[0] = make_uint4(x, x, x, x);
}

// Cold-cache timing: scrub, then one timed product, per iteration.
template <class T>
dao_status time_product_cold_typed(dao_ctx* c, int kernel, int iters, void* scrub, int64_t scrub_bytes,
                                   double* us) {
    double tot = 0.0;
    for (int i = 0; i < iters; ++i) {
        k_scrub<<<2048, BLOCK, 0, c->stream>>>(static_cast<uint4*>(scrub), scrub_bytes / 16, 0x9E3779B9u + uint32_t(i));
        LAUNCHCHK(c);
        double one = 0.0;
        dao_status s = time_product_typed<T>(c, kernel, 1, &one, false);
        if (s != DAO_OK) return s;
        tot += one;
    }
    *us = tot / iters;
    return DAO_OK;
}

template <class T>
dao_status master_solve_typed(dao_ctx* c, double tol, int max_steps, int32_t* steps, double* kkt,
                              double* F) {
    dao_status s = run_master<T>(c, tol, max_steps);
    if (s != DAO_OK) return s;
    if (steps) *steps = c->ms_h->steps;
    if (kkt) *kkt = c->ms_h->kkt;
    if (F) *F = c->ms_h->F;
    return c->ms_h->stop_reason == 2 ? DAO_ENOTCONV : DAO_OK;
}

// Restore a pool, its intensities and the loop state: the columns of D_K are
// rebuilt, the dose is D (A y) in FP64 and the objective, grad F and prices
// follow from it.
template <class T>
dao_status set_state_typed(dao_ctx* c, const dao_state_info* info, const int32_t* beams, const int16_t* leaves,
                           const double* y) {
    dao_status s = reset_state<T>(c);
    if (s != DAO_OK) return s;
    const int n = info->n;
    for (int k = 0; k < n; ++k) {
        const int16_t* lv = leaves + size_t(k) * 2 * c->maxRB;
        const int nr = c->rows_per_beam[beams[k]];
        for (int i = 0; i < c->maxRB; ++i) {
            c->lv_stage_h[2 * i] = i < nr ? lv[2 * i] : int16_t(0);
            c->lv_stage_h[2 * i + 1] = i < nr ? lv[2 * i + 1] : int16_t(0);
        }
        HIPCHK(c, hipMemcpyAsync(c->ap_lv + size_t(k) * c->maxRB * 2, c->lv_stage_h, size_t(c->maxRB) * 4,
                                 hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(c->ap_beam + k, beams + k, 4, hipMemcpyHostToDevice, c->stream));
        // the staging buffer is reused by the next aperture
        HIPCHK(c, hipStreamSynchronize(c->stream));
        s = build_dk_column<T>(c, k);
        if (s != DAO_OK) return s;
        mirror_add(c, beams[k], lv);
        c->K = k + 1;
    }
    if (n > 0) HIPCHK(c, hipMemcpyAsync(c->y, y, size_t(n) * 8, hipMemcpyHostToDevice, c->stream));
    k_set_history<<<1, 1, 0, c->stream>>>(c->ms, info->last_step, info->prev_step);
    LAUNCHCHK(c);
    s = refresh_dose_exact<T>(c);
    if (s != DAO_OK) return s;
    s = refresh_objective<T>(c);
    if (s != DAO_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->loop_rc1 = info->rc1;
    c->loop_eps = info->eps;
    c->loop_tighten = info->tighten;
    return DAO_OK;
}

// Append an aperture given on the host (leaves of its beam's rows) with y = 0.
// Selective residual (d_residual 2).  The final rounds of a plan run with
// the FP16 residual in every product and with D_K in FP32: the columns built
// so far are rebuilt that way once, when the final phase begins.
template <class T>
dao_status enter_final_phase(dao_ctx* c) {
    c->final_phase = true;
    c->lo_now = true;
    if (c->dk16) {
        c->dk16 = false;
        c->dk_scale = 1.0;   // FP32 columns hold D_K itself
        HIPCHK(c, hipMemsetAsync(c->dk, 0, size_t(c->Vpad) * KS * sizeof(T), c->stream));
        for (int k = 0; k < c->K; ++k) {
            const dao_status s = build_dk_column<T>(c, k);
            if (s != DAO_OK) return s;
        }
    }
    return DAO_OK;
}

// Before the final phase, pricing runs on the 16-bit values alone.  Each of
// its prices w_i = sum_j D_ij pi_j is then off by at most u sum_j D_ij |pi_j|
// (u = 2^-11 for FP16, 2^-8 for BF16: the relative rounding of a stored
// value), so a reduced cost is off by at most u sum_{i in A} (D^T |pi|)_i,
// doubled for the rounding the dose carries into pi.  A decision whose gap
// is below twice that bound is priced again with the residual.
template <class T>
dao_status price_selective(dao_ctx* c, int32_t* beam, int16_t* leaves, double* rc, double* gap) {
    dao_status s = price_current<T>(c, beam, leaves, rc, gap);
    if (s != DAO_OK || c->opt.d_residual != 2 || c->lo_now) return s;
    k_abs_copy<<<c->elem_blocks(c->Vpad), BLOCK, 0, c->stream>>>(c->u64, c->Vpad, c->uabs64);
    launch_gradT<T, double, double, double>(c, c->uabs64, c->gabs64);
    LAUNCHCHK(c);
    std::vector<double> ga(size_t(c->N));
    HIPCHK(c, hipMemcpyAsync(ga.data(), c->gabs64, size_t(c->N) * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int start = 0;
    for (int r = 0; r < c->beam_row0[*beam]; ++r) start += c->row_len[r];
    double sum = 0.0;
    for (int r = c->beam_row0[*beam]; r < c->beam_row0[*beam + 1]; ++r) {
        const int lr = r - c->beam_row0[*beam];
        for (int pos = leaves[2 * lr]; pos < leaves[2 * lr + 1]; ++pos) sum += ga[size_t(start + pos)];
        start += c->row_len[r];
    }
    const double u = c->opt.d_format == DAO_DFMT_BF16 ? 0x1p-8 : 0x1p-11;
    if (!(*gap > 4.0 * u * sum)) {
        c->lo_now = true;
        s = price_current<T>(c, beam, leaves, rc, gap);
        c->lo_now = false;
        ++c->reprices;
    }
    return s;
}

dao_status add_aperture_host(dao_ctx* c, int32_t beam, const int16_t* leaves) {
    dao_status s;
    if (c->K >= c->opt.max_apertures) return c->fail(DAO_ESTATE, "pool capacity reached");
    const int nr = c->rows_per_beam[beam];
    for (int i = 0; i < c->maxRB; ++i) {
        c->lv_stage_h[2 * i] = i < nr ? leaves[2 * i] : int16_t(0);
        c->lv_stage_h[2 * i + 1] = i < nr ? leaves[2 * i + 1] : int16_t(0);
    }
    HIPCHK(c, hipMemcpyAsync(c->ap_lv + size_t(c->K) * c->maxRB * 2, c->lv_stage_h,
                             size_t(c->maxRB) * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->ap_beam + c->K, &beam, 4, hipMemcpyHostToDevice, c->stream));
    k_fill<double><<<1, 64, 0, c->stream>>>(c->y + c->K, 1, 0.0);
    LAUNCHCHK(c);
    s = c->dtype == DAO_F64 ? build_dk_column<double>(c, c->K) : build_dk_column<float>(c, c->K);
    if (s != DAO_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    mirror_add(c, beam, leaves);
    c->K += 1;
    return DAO_OK;
}


// Several apertures per round: after the entering aperture, the beams ranked
// 2..m by value (ties to the lowest beam) add their own best apertures, each
// if its value is below -tau, it is not pooled yet and the budget allows.
// The beam values are summed from the pricing launch's row records in the
// kernel's own order, so the ranking sees the same values as the argmin.
template <class T>
dao_status add_ranked_apertures(dao_ctx* c, int m, int n_ap, double tau, int* added) {
    *added = 0;
    std::vector<RowRec> rows(size_t(c->R));
    HIPCHK(c, hipMemcpyAsync(rows.data(), c->rowrec, size_t(c->R) * sizeof(RowRec), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<std::pair<double, int>> order;
    for (int b = 0; b < c->B; ++b) {
        double sb = 0.0;
        for (int rr = c->beam_row0[b]; rr < c->beam_row0[b + 1]; ++rr) sb += rows[size_t(rr)].v;
        order.push_back({sb, b});
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<double, int>& x, const std::pair<double, int>& y) {
                         return x.first < y.first || (x.first == y.first && x.second < y.second);
                     });
    std::vector<int16_t> lv(size_t(2 * c->maxRB), 0);
    for (int i = 1; i < std::min(m, int(order.size())); ++i) {
        if (c->K >= n_ap || !(order[size_t(i)].first < -tau)) break;
        const int b = order[size_t(i)].second;
        for (int rr = c->beam_row0[b]; rr < c->beam_row0[b + 1]; ++rr) {
            lv[size_t(2 * (rr - c->beam_row0[b]))] = int16_t(rows[size_t(rr)].L);
            lv[size_t(2 * (rr - c->beam_row0[b]) + 1)] = int16_t(rows[size_t(rr)].R);
        }
        if (in_pool(c, b, lv.data())) continue;
        const dao_status s = add_aperture_host(c, b, lv.data());
        if (s != DAO_OK) return s;
        ++*added;
    }
    return DAO_OK;
}

// One column-generation solve, split into the steps around its master
// solves so that several solves can share one master launch per round.
using clk = std::chrono::steady_clock;
inline double since(clk::time_point t0) { return std::chrono::duration<double>(clk::now() - t0).count(); }

struct PlanRun {
    dao_ctx* c = nullptr;
    int32_t n_ap = 0;
    dao_plan* out = nullptr;
    double eps = 0.0, rc1 = NAN, tol = 0.0;
    int tighten = 0, rounds = 0, capped = 0;
    int32_t stop = DAO_OK;
    int64_t steps0 = 0, ls0 = 0;
    double t_price = 0.0, t_master = 0.0;
    bool finished = false, added = false;
    int32_t beam = 0;
    double rc = 0.0, gap = 0.0;
    std::vector<int16_t> lv;
    clk::time_point tm;
};

// A fresh solve starts from an empty pool; a resumed one from the context's
// current pool, intensities and loop state (dao_set_state or an earlier
// solve), numbering its rounds on from the pool size.
template <class T>
dao_status plan_start(PlanRun& r, bool resume = false) {
    dao_ctx* c = r.c;
    if (resume) {
        r.eps = c->loop_eps > 0.0 ? c->loop_eps : c->opt.eps;
        r.rc1 = c->loop_rc1;
        r.tighten = c->loop_tighten;
    } else {
        dao_status s = reset_state<T>(c);
        if (s != DAO_OK) return s;
        r.eps = c->opt.eps;
        r.rc1 = NAN;
        r.tighten = 0;
    }
    HIPCHK(c, hipMemcpyAsync(c->ms_h, c->ms, sizeof(MasterState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    r.steps0 = c->ms_h->total_steps;
    r.ls0 = c->ms_h->total_ls;
    r.lv.assign(2 * c->maxRB, 0);
    return DAO_OK;
}

// Pricing, entry test and column of the next round.  Either finishes the
// solve (r.finished) or leaves a master solve to run to r.tol.
template <class T>
dao_status plan_round_begin(PlanRun& r) {
    dao_ctx* c = r.c;
    r.added = false;
    if (c->K >= r.n_ap) {
        r.finished = true;
        return DAO_OK;
    }
    const auto tp = clk::now();
    if (c->opt.d_residual == 2 && !c->final_phase && c->K >= r.n_ap - c->opt.residual_rounds) {
        const dao_status f = enter_final_phase<T>(c);
        if (f != DAO_OK) return f;
    }
    dao_status s = price_selective<T>(c, &r.beam, r.lv.data(), &r.rc, &r.gap);
    if (s != DAO_OK) return s;
    r.t_price += since(tp);
    r.tm = clk::now();
    if (std::isnan(r.rc1)) {
        r.rc1 = r.rc;
        if (!(r.rc1 < 0.0)) {
            r.stop = DAO_EOPTIMAL;
            r.finished = true;
            return DAO_OK;
        }
    }
    const double scale = std::fabs(r.rc1);
    if (r.rc >= -c->opt.tau_rel * scale) {
        r.stop = DAO_EOPTIMAL;
        r.finished = true;
        return DAO_OK;
    }
    if (in_pool(c, r.beam, r.lv.data())) {
        if (r.tighten >= c->opt.max_tighten) {
            r.stop = DAO_ESTALLED;
            r.finished = true;
            return DAO_OK;
        }
        ++r.tighten;
        r.eps /= 10.0;
        r.tol = r.eps * scale;   // re-solve the same pool more tightly
        return DAO_OK;
    }
    if (c->K >= c->opt.max_apertures) return c->fail(DAO_ESTATE, "pool capacity reached");
    k_add_from_price<<<1, 256, 0, c->stream>>>(c->pr, c->K, c->maxRB, c->ap_beam, c->ap_lv, c->y);
    LAUNCHCHK(c);
    s = build_dk_column<T>(c, c->K);
    if (s != DAO_OK) return s;
    mirror_add(c, r.beam, r.lv.data());
    c->K += 1;
    r.added = true;
    r.tol = r.eps * scale;
    if (c->opt.apertures_per_round > 1) {
        int more = 0;
        s = add_ranked_apertures<T>(c, c->opt.apertures_per_round, r.n_ap, c->opt.tau_rel * scale, &more);
        if (s != DAO_OK) return s;
    }
    return DAO_OK;
}

// After the round's master solve (c->ms_h holds its final state).
void plan_round_end(PlanRun& r) {
    dao_ctx* c = r.c;
    r.t_master += since(r.tm);
    if (!r.added) return;
    if (dao_plan* out = r.out) {
        if (out->round_beam) out->round_beam[r.rounds] = r.beam;
        if (out->round_rc) out->round_rc[r.rounds] = r.rc;
        if (out->round_gap) out->round_gap[r.rounds] = r.gap;
        if (out->round_steps) out->round_steps[r.rounds] = c->ms_h->steps;
        if (out->round_kkt) out->round_kkt[r.rounds] = c->ms_h->kkt;
        if (out->round_F) out->round_F[r.rounds] = c->ms_h->F;
        if (out->round_stop) out->round_stop[r.rounds] = c->ms_h->stop_reason;
    }
    if (c->ms_h->stop_reason == 2) ++r.capped;
    ++r.rounds;
}

dao_status plan_finish(PlanRun& r) {
    dao_ctx* c = r.c;
    HIPCHK(c, hipMemcpyAsync(c->ms_h, c->ms, sizeof(MasterState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (dao_plan* out = r.out) {
        out->rounds = r.rounds;
        out->stop = r.stop;
        out->F = c->ms_h->F;
        out->rc1 = r.rc1;
        out->total_steps = c->ms_h->total_steps - r.steps0;
        out->total_ls_evals = c->ms_h->total_ls - r.ls0;
        out->price_s = r.t_price;
        out->master_s = r.t_master;
        out->capped_rounds = r.capped;
    }
    c->loop_rc1 = r.rc1;
    c->loop_eps = r.eps;
    c->loop_tighten = r.tighten;
    return DAO_OK;
}

template <class T>
dao_status solve_typed(dao_ctx* c, int32_t n_ap, dao_plan* out, bool resume = false) {
    PlanRun r;
    r.c = c;
    r.n_ap = n_ap;
    r.out = out;
    dao_status s = plan_start<T>(r, resume);
    if (s != DAO_OK) return s;
    for (;;) {
        s = plan_round_begin<T>(r);
        if (s != DAO_OK) return s;
        if (r.finished) break;
        s = run_master<T>(c, r.tol, c->opt.max_steps);
        if (s != DAO_OK) return s;
        plan_round_end(r);
    }
    return plan_finish(r);
}

// The round's master solves of several contexts in one cooperative launch of
// k_master_batch (when all use the persistent master on one stream; else one
// after another).  Workgroups are shared out in proportion to the solves'
// voxel rows, at least one each.
template <class T, class DT>
dao_status run_master_batch_dt(std::vector<PlanRun*>& live) {
    for (PlanRun* r : live)
        if (r->c->Vpad % Batch<DT>::ROWS != 0)
            return r->c->fail(DAO_ESTATE, "padded rows not a multiple of the D_K batch");
    dao_ctx* c0 = live[0]->c;
    bool together = live.size() > 1 && int(live.size()) <= std::min(MAX_BATCH, c0->coop_grid);
    for (PlanRun* r : live)
        together = together && r->c->coop_master() && r->c->batch_ok && r->c->stream == c0->stream &&
                   r->c->coop_grid == c0->coop_grid && r->c->prof_kernel < 0;
    if (!together) {
        for (PlanRun* r : live) {
            dao_status s = run_master<T>(r->c, r->tol, r->c->opt.max_steps);
            if (s != DAO_OK) return s;
        }
        return DAO_OK;
    }
    const int n = int(live.size()), G = c0->coop_grid;
    if (!c0->batch_args) {
        dao_status s = dev_alloc(c0, &c0->batch_args, size_t(MAX_BATCH) * sizeof(CoopArgs<double>));
        if (s != DAO_OK) return s;
        s = dev_alloc(c0, &c0->batch_gstart, size_t(MAX_BATCH + 1) * sizeof(int32_t));
        if (s != DAO_OK) return s;
        HIPCHK(c0, hipHostMalloc(&c0->batch_host, size_t(MAX_BATCH) * sizeof(CoopArgs<double>) +
                                                    size_t(MAX_BATCH + 1) * sizeof(int32_t), hipHostMallocDefault));
    }
    // workgroups in proportion to the rows
    double tot = 0.0;
    for (PlanRun* r : live) tot += double(r->c->Vpad);
    std::vector<int> g(n);
    int used = 0;
    for (int i = 0; i < n; ++i) {
        g[i] = std::max(1, int(double(G) * double(live[i]->c->Vpad) / tot));
        used += g[i];
    }
    while (used > G)   // take back from the largest shares
        for (int i = 0; i < n && used > G; ++i)
            if (g[i] > 1 && g[i] == *std::max_element(g.begin(), g.end())) {
                --g[i];
                --used;
            }
    for (int i = 0; used < G; i = (i + 1) % n) {   // hand out what is left
        ++g[i];
        ++used;
    }
    auto* hargs = reinterpret_cast<CoopArgs<T>*>(c0->batch_host);
    auto* hstart = reinterpret_cast<int32_t*>(static_cast<char*>(c0->batch_host) +
                                              size_t(MAX_BATCH) * sizeof(CoopArgs<double>));
    size_t lds = 0, lds_h = 0;
    bool fits = c0->opt.persistent == 2 && c0->coop_lds_max > 0;
    bool fits_h = fits;
    hstart[0] = 0;
    for (int i = 0; i < n; ++i) {
        dao_ctx* c = live[i]->c;
        k_master_init_ap<<<1, 1, 0, c->stream>>>(c->ms, c->K, live[i]->tol, c->opt.max_steps);
        LAUNCHCHK(c);
        HIPCHK(c, hipMemsetAsync(c->coop, 0, sizeof(CoopSync), c->stream));
        hargs[i] = CoopArgs<T>{c->dk, c->dk_scale, c->Vpad, c->Vnz, c->d, static_cast<T*>(c->q), c->cls_int,
                               c->classes, c->ncls, c->y, c->p, c->gradk, c->cgm, c->tau_int, c->ms,
                               c->coop_recs, c->coop_bpart, c->coop, c->pc, 0};
        hstart[i + 1] = hstart[i] + g[i];
        const int nc = (c->K + DKG<DT>::EPL - 1) / DKG<DT>::EPL;
        const int64_t rows_i = coop_batches_per_group<DT>(c->Vpad, g[i]) * Batch<DT>::ROWS;
        const size_t li = coop_lds_bytes<T>(rows_i, nc), lh = coop_hybrid_lds<T, DT>(rows_i);
        lds = std::max(lds, li);
        lds_h = std::max(lds_h, lh);
        fits = fits && c->opt.persistent == 2 && li <= size_t(c0->coop_lds_max);
        fits_h = fits_h && c->opt.persistent == 2 && lh <= size_t(c0->coop_lds_max);
    }
    HIPCHK(c0, hipMemcpyAsync(c0->batch_args, hargs, size_t(n) * sizeof(CoopArgs<T>), hipMemcpyHostToDevice,
                              c0->stream));
    HIPCHK(c0, hipMemcpyAsync(c0->batch_gstart, hstart, size_t(n + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                              c0->stream));
    const CoopArgs<T>* dargs = static_cast<const CoopArgs<T>*>(c0->batch_args);
    const int32_t* dstart = c0->batch_gstart;
    int nn = n;
    void* kargs[] = {&dargs, &dstart, &nn};
    // the form every solve of the launch can take (as for one solve)
    if (fits)
        HIPCHK(c0, hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_master_batch<T, DT, COOP_CHIP>),
                                              dim3(G), dim3(COOP_THREADS), kargs, lds, c0->stream));
    else if (fits_h)
        HIPCHK(c0, hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_master_batch<T, DT, COOP_HYBRID>),
                                              dim3(G), dim3(COOP_THREADS), kargs, lds_h, c0->stream));
    else
        HIPCHK(c0, hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_master_batch<T, DT, COOP_STREAM>),
                                              dim3(G), dim3(COOP_THREADS), kargs, coop_stream_lds<DT>(),
                                              c0->stream));
    for (PlanRun* r : live) r->c->last_form = fits ? 4 : fits_h ? 6 : 3;
    for (PlanRun* r : live)
        HIPCHK(r->c, hipMemcpyAsync(r->c->ms_h, r->c->ms, sizeof(MasterState), hipMemcpyDeviceToHost, r->c->stream));
    HIPCHK(c0, hipStreamSynchronize(c0->stream));
    for (PlanRun* r : live) {
        if (r->c->ms_h->stop_reason == 4 || !r->c->ms_h->done)
            return r->c->fail(DAO_EDEVICE, "batched persistent master: grid reduction timed out");
        r->c->last_steps = r->c->ms_h->steps;
        r->c->last_stop = r->c->ms_h->stop_reason;
    }
    return DAO_OK;
}

// Solves whose D_K storage differs run in separate batched launches.
template <class T>
dao_status run_master_batch(std::vector<PlanRun*>& live) {
    if constexpr (std::is_same<T, float>::value) {
        std::vector<PlanRun*> h, n;
        for (PlanRun* r : live) (r->c->dk16 ? h : n).push_back(r);
        if (!h.empty()) {
            const dao_status s = run_master_batch_dt<T, __half>(h);
            if (s != DAO_OK) return s;
        }
        return n.empty() ? DAO_OK : run_master_batch_dt<T, T>(n);
    }
    return run_master_batch_dt<T, T>(live);
}

// Several solves advanced round by round together: each round prices every
// live solve, adds its column, then runs all their master solves in one
// launch.  A solve leaves the batch when it finishes.
template <class T>
dao_status solve_batch_typed(dao_ctx* const* ctxs, int n, const int32_t* n_ap, dao_plan* outs) {
    std::vector<PlanRun> runs(n);
    for (int i = 0; i < n; ++i) {
        runs[i].c = ctxs[i];
        runs[i].n_ap = n_ap[i];
        runs[i].out = outs ? &outs[i] : nullptr;
        dao_status s = plan_start<T>(runs[i]);
        if (s != DAO_OK) return s;
    }
    for (;;) {
        std::vector<PlanRun*> live;
        for (PlanRun& r : runs) {
            if (r.finished) continue;
            dao_status s = plan_round_begin<T>(r);
            if (s != DAO_OK) return s;
            if (!r.finished) live.push_back(&r);
        }
        if (live.empty()) break;
        dao_status s = run_master_batch<T>(live);
        if (s != DAO_OK) return s;
        for (PlanRun* r : live) plan_round_end(*r);
    }
    for (PlanRun& r : runs) {
        dao_status s = plan_finish(r);
        if (s != DAO_OK) return s;
    }
    return DAO_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void dao_default_options(dao_options* o) {
    if (!o) return;
    o->dtype = DAO_F32;
    o->max_apertures = 64;
    o->eps = 1e-6;
    o->max_steps = 500;
    o->tau_rel = 1e-10;
    o->max_tighten = 3;
    o->refresh_every = 50;
    o->ls_slots = 2;
    o->mem_cap_bytes = 0;
    o->master = DAO_MASTER_APERTURE;
    o->d_format = DAO_DFMT_NATIVE;
    o->d_residual = 0;
    o->persistent = 2;
    o->product_tune = 1;
    o->dose_variant = 0;
    o->gradient_depth = 4;
    o->direction = DAO_DIR_CONJUGATE;
    o->apertures_per_round = 1;
    o->dk_format = DAO_DFMT_NATIVE;
    o->residual_rounds = 5;
    o->graphs = 0;
}

const char* dao_create_error(void) { return g_create_error.c_str(); }

const char* dao_last_error(const dao_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

namespace {

// The host half of dao_create: validate the inputs and lay them out; *need is
// the predicted device footprint.  Sets g_create_error on failure.
dao_status prepare_layout(const dao_matrix* D, const dao_beams* beams, const dao_structures* structs,
                          const dao_prescription* presc, dao_options* opt, std::unique_ptr<HostLayout>* L,
                          int64_t* need) {
    std::string err;
    const dao_status s = validate_inputs(D, beams, structs, presc, opt, &err);
    if (s != DAO_OK) {
        g_create_error = err;
        return s;
    }
    *L = std::make_unique<HostLayout>();
    build_layout(D, beams, structs, presc, L->get());
    *need = predicted_bytes(**L, opt->dtype == DAO_F64 ? 8 : 4, opt->max_apertures, *opt);
    if (opt->mem_cap_bytes > 0 && *need > opt->mem_cap_bytes) {
        g_create_error = "device footprint " + std::to_string(*need) + " B exceeds mem_cap_bytes";
        return DAO_ENOMEM;
    }
    return DAO_OK;
}

// The device half: allocate, upload, tune.  Sets g_create_error on failure.
dao_status create_on_device(std::unique_ptr<HostLayout> L, const dao_beams* beams, const dao_options& opt,
                            void* stream, dao_ctx** out) {
    const size_t ts = opt.dtype == DAO_F64 ? 8 : 4;
    auto c = std::make_unique<dao_ctx>();
    c->opt = opt;
    c->dtype = opt.dtype;
    c->tsize = ts;
    c->stream = static_cast<hipStream_t>(stream);
    c->V = L->V;
    c->N = L->N;
    c->nnz = L->nnz;
    c->Vnz = L->Vnz;
    c->Vpad = std::max<int64_t>(L->Vpad, SLICE);
    c->nslices = L->nslices;
    c->B = L->B;
    c->R = L->R;
    c->maxRB = L->max_rows_per_beam;
    c->ncls = int32_t(L->classes.size());
    c->sell_entries = L->slice_ptr.back();
    c->F_const = L->F_const;
    c->rows_per_beam.assign(beams->rows_per_beam, beams->rows_per_beam + beams->n_beams);
    c->row_len = L->row_len;
    c->beam_row0 = L->beam_row0;
    if (L->Vpad < c->Vpad) {   // no non-empty row at all: keep one padding slice
        L->perm.resize(c->Vpad, -1);
        L->cls_int.resize(c->Vpad, uint8_t(L->n_struct));
        if (!L->tau_int.empty()) L->tau_int.resize(c->Vpad, 0.0);
    }
    const dao_status s = (c->dtype == DAO_F64) ? create_typed<double>(c.get(), *L) : create_typed<float>(c.get(), *L);
    if (s != DAO_OK) {
        g_create_error = c->err;
        return s;
    }
    *out = c.release();
    return DAO_OK;
}

}  // namespace

extern "C" {

dao_status dao_create(const dao_matrix* D, const dao_beams* beams, const dao_structures* structs,
                      const dao_prescription* presc, const dao_options* opt_in, void* stream,
                      dao_ctx** out) {
    g_create_error.clear();
    if (!out) {
        g_create_error = "null output pointer";
        return DAO_EINVAL;
    }
    *out = nullptr;
    dao_options opt;
    if (opt_in)
        opt = *opt_in;
    else
        dao_default_options(&opt);
    std::unique_ptr<HostLayout> L;
    int64_t need = 0;
    const dao_status s = prepare_layout(D, beams, structs, presc, &opt, &L, &need);
    if (s != DAO_OK) return s;
    return create_on_device(std::move(L), beams, opt, stream, out);
}

void dao_destroy(dao_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    delete c;
}

dao_status dao_info(const dao_ctx* c, dao_info_t* o) {
    if (!c || !o) return DAO_EINVAL;
    o->n_vox = c->V;
    o->n_vox_nonempty = c->Vnz;
    o->n_blt = c->N;
    o->nnz = c->nnz;
    o->n_rows = c->R;
    o->n_beams = c->B;
    o->max_rows_per_beam = c->maxRB;
    o->dtype = c->dtype;
    o->n_slices = int32_t(c->nslices);
    o->sell_entries = c->sell_entries;
    o->device_bytes = c->device_bytes;
    const int64_t ts = int64_t(c->tsize);
    o->d_format = c->opt.d_format;
    o->d_residual = c->opt.d_residual;
    o->dose_variant = c->dose_var;
    o->gradient_depth = c->gradT_pf;
    o->last_master_form = c->last_form;
    o->onchip_lds_bytes = c->coop_lds_max;
    o->dk_format = c->dk16 ? DAO_DFMT_F16 : DAO_DFMT_NATIVE;
    o->residual_reprices = c->reprices;
    // stored bytes per value: the ctx type, or 16 bits (+ 16 for the residual)
    const bool narrow = c->opt.d_format != DAO_DFMT_NATIVE;
    const int64_t vs = narrow ? 2 + (c->opt.d_residual ? 2 : 0) : ts;
    const int64_t sc = narrow ? c->N * 4 : 0;   // per-beamlet scales
    // forward: every entry (value + 16-bit column) + slice headers + x once +
    // scales + d once (caller order)
    o->bytes_dose = c->nnz * (vs + 2) + (c->nslices + 1) * 4 + c->nslices * 4 + c->N * ts + sc + c->Vnz * (ts + 4);
    // transpose: every entry (value + 32-bit row) + column pointers + u once +
    // scales + g once
    o->bytes_gradient = c->nnz * (vs + 4) + (c->N + 1) * 4 + c->Vnz * ts + sc + c->N * ts;
    return DAO_OK;
}

dao_status dao_dose(dao_ctx* c, const void* x, void* d) {
    if (!c) return DAO_EINVAL;
    if (!x || !d) return c->fail(DAO_EINVAL, "null vector");
    return c->dtype == DAO_F64 ? dose_typed<double>(c, x, d) : dose_typed<float>(c, x, d);
}

dao_status dao_gradient(dao_ctx* c, const void* d, void* g, double* F) {
    if (!c) return DAO_EINVAL;
    if (!d || !g) return c->fail(DAO_EINVAL, "null vector");
    return c->dtype == DAO_F64 ? gradient_typed<double>(c, d, g, F) : gradient_typed<float>(c, d, g, F);
}

dao_status dao_price(dao_ctx* c, const double* g, int32_t* beam, int16_t* leaves, double* rc,
                     double* gap) {
    if (!c) return DAO_EINVAL;
    if (!g) return c->fail(DAO_EINVAL, "null prices");
    return price_on(c, g, beam, leaves, rc, gap);
}

dao_status dao_price_noalloc(dao_ctx* c, const double* g, int32_t* beam, int16_t* leaves, double* rc,
                             double* gap) {
    if (!c) return DAO_EINVAL;
    if (!g) return c->fail(DAO_EINVAL, "null prices");
    if (c->R > NOALLOC_MAX_ROWS)
        return c->fail(DAO_EINVAL, std::to_string(c->R) + " MLC rows exceed the " +
                                       std::to_string(NOALLOC_MAX_ROWS) + " rows of the static pricing scratch");
    if (!c->scratch_dev) return c->fail(DAO_ESTATE, "static pricing scratch unavailable");
    RowRec* rows = reinterpret_cast<RowRec*>(c->scratch_dev + NOALLOC_ROWS_OFF);
    PriceResult* pr = reinterpret_cast<PriceResult*>(c->scratch_dev + NOALLOC_PR_OFF);
    Arrival* arr = reinterpret_cast<Arrival*>(c->scratch_dev + NOALLOC_ARR_OFF);
    // the arrival counters must start at zero whatever the last call left
    // (a fill kernel: no memset node if the caller captures the stream)
    constexpr int64_t narr = int64_t(sizeof(Arrival) / sizeof(uint32_t));
    k_fill<uint32_t><<<(narr + BLOCK - 1) / BLOCK, BLOCK, 0, c->stream>>>(reinterpret_cast<uint32_t*>(arr), narr,
                                                                         0u);
    LAUNCHCHK(c);
    return price_with(c, g, rows, pr, arr, beam, leaves, rc, gap);
}

dao_status dao_reset(dao_ctx* c) {
    if (!c) return DAO_EINVAL;
    dao_status s = c->dtype == DAO_F64 ? reset_state<double>(c) : reset_state<float>(c);
    if (s != DAO_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return DAO_OK;
}

dao_status dao_add_aperture(dao_ctx* c, int32_t beam, const int16_t* leaves) {
    if (!c) return DAO_EINVAL;
    dao_status s = check_aperture(c, beam, leaves);
    if (s != DAO_OK) return s;
    return add_aperture_host(c, beam, leaves);
}

dao_status dao_master_step(dao_ctx* c, double* F, double* kkt, double* step) {
    if (!c) return DAO_EINVAL;
    dao_status s = c->dtype == DAO_F64 ? run_master<double>(c, 0.0, 1) : run_master<float>(c, 0.0, 1);
    if (s != DAO_OK) return s;
    if (F) *F = c->ms_h->F;
    if (kkt) *kkt = c->ms_h->kkt;
    if (step) *step = c->ms_h->steps > 0 ? c->ms_h->last_step : 0.0;
    return DAO_OK;
}

dao_status dao_master_solve(dao_ctx* c, double tol, int32_t max_steps, int32_t* steps, double* kkt,
                            double* F) {
    if (!c) return DAO_EINVAL;
    if (!(tol >= 0) || max_steps < 0) return c->fail(DAO_EINVAL, "bad tolerance or step cap");
    return c->dtype == DAO_F64 ? master_solve_typed<double>(c, tol, max_steps, steps, kkt, F)
                               : master_solve_typed<float>(c, tol, max_steps, steps, kkt, F);
}

dao_status dao_price_current(dao_ctx* c, int32_t* beam, int16_t* leaves, double* rc, double* gap) {
    if (!c) return DAO_EINVAL;
    return c->dtype == DAO_F64 ? price_current<double>(c, beam, leaves, rc, gap)
                               : price_current<float>(c, beam, leaves, rc, gap);
}

dao_status dao_get_pool(dao_ctx* c, int32_t cap, int32_t* n, int32_t* beams, int16_t* leaves, double* y) {
    if (!c) return DAO_EINVAL;
    if (n) *n = c->K;
    const int m = std::min<int>(std::max(cap, 0), c->K);
    if (beams) std::copy(c->pool_beam.begin(), c->pool_beam.begin() + m, beams);
    if (leaves) std::copy(c->pool_lv.begin(), c->pool_lv.begin() + size_t(m) * 2 * c->maxRB, leaves);
    if (y && m > 0) {
        HIPCHK(c, hipMemcpyAsync(y, c->y, size_t(m) * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return DAO_OK;
}

dao_status dao_get_dose(dao_ctx* c, double* d_dev, double* F) {
    if (!c) return DAO_EINVAL;
    if (d_dev) {
        k_fill<double><<<c->elem_blocks(c->V), BLOCK, 0, c->stream>>>(d_dev, c->V, 0.0);
        // the master keeps d - tau: add the shifts back
        k_scatter_shift<<<c->elem_blocks(c->Vpad), BLOCK, 0, c->stream>>>(c->d, c->tau_int, c->perm, c->Vpad,
                                                                          d_dev);
        LAUNCHCHK(c);
    }
    HIPCHK(c, hipMemcpyAsync(c->ms_h, c->ms, sizeof(MasterState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (F) *F = c->ms_h->F;
    return DAO_OK;
}

dao_status dao_time_product(dao_ctx* c, int32_t kernel, int32_t iters, double* us_per_launch) {
    if (!c) return DAO_EINVAL;
    if ((kernel != 0 && kernel != 1) || iters < 1 || !us_per_launch)
        return c->fail(DAO_EINVAL, "kernel must be 0 or 1, iters >= 1");
    return c->dtype == DAO_F64 ? time_product_typed<double>(c, kernel, iters, us_per_launch)
                               : time_product_typed<float>(c, kernel, iters, us_per_launch);
}

dao_status dao_encode_values(int32_t d_format, int64_t n, const double* r, uint16_t* hi, uint16_t* lo) {
    if (d_format != DAO_DFMT_F16 && d_format != DAO_DFMT_BF16) return DAO_EINVAL;
    if (n < 0 || (n > 0 && (!r || !hi))) return DAO_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (!(r[i] >= 0.0) || !std::isfinite(r[i])) return DAO_EINVAL;
    for (int64_t i = 0; i < n; ++i) encode_value(d_format, r[i], &hi[i], lo ? &lo[i] : nullptr);
    return DAO_OK;
}

dao_status dao_time_product_cold(dao_ctx* c, int32_t kernel, int32_t iters, void* scrub, int64_t scrub_bytes,
                                 double* us_per_launch) {
    if (!c) return DAO_EINVAL;
    if ((kernel != 0 && kernel != 1) || iters < 1 || !us_per_launch)
        return c->fail(DAO_EINVAL, "kernel must be 0 or 1, iters >= 1");
    if (!scrub || scrub_bytes < (int64_t(1) << 20) || scrub_bytes % 16 != 0)
        return c->fail(DAO_EINVAL, "scrub must be a device buffer of >= 1 MiB, a multiple of 16 bytes");
    return c->dtype == DAO_F64 ? time_product_cold_typed<double>(c, kernel, iters, scrub, scrub_bytes, us_per_launch)
                               : time_product_cold_typed<float>(c, kernel, iters, scrub, scrub_bytes, us_per_launch);
}

dao_status dao_time_read_cold(dao_ctx* c, void* buf, int64_t bytes, int32_t iters, void* scrub,
                              int64_t scrub_bytes, double* us_per_launch) {
    if (!c) return DAO_EINVAL;
    if (!buf || bytes < 16 || bytes % 16 != 0 || iters < 1 || !us_per_launch)
        return c->fail(DAO_EINVAL, "buf must be a device buffer of >= 16 bytes, a multiple of 16; iters >= 1");
    if (!scrub || scrub_bytes < (int64_t(1) << 20) || scrub_bytes % 16 != 0)
        return c->fail(DAO_EINVAL, "scrub must be a device buffer of >= 1 MiB, a multiple of 16 bytes");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(c, hipEventCreate(&e0));
    const hipError_t ec = hipEventCreate(&e1);
    if (ec != hipSuccess) {
        (void)hipEventDestroy(e0);
        return c->fail(DAO_EDEVICE, "hipEventCreate failed");
    }
    double tot = 0.0;
    hipError_t he = hipSuccess;
    for (int i = 0; i < iters && he == hipSuccess; ++i) {
        k_scrub<<<2048, BLOCK, 0, c->stream>>>(static_cast<uint4*>(scrub), scrub_bytes / 16, 0x9E3779B9u + uint32_t(i));
        he = hipGetLastError();
        if (he == hipSuccess) he = hipEventRecord(e0, c->stream);
        if (he == hipSuccess) {
            k_scrub<<<2048, BLOCK, 0, c->stream>>>(static_cast<uint4*>(buf), bytes / 16, 0x85EBCA6Bu + uint32_t(i));
            he = hipGetLastError();
        }
        if (he == hipSuccess) he = hipEventRecord(e1, c->stream);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        tot += double(ms) * 1e3;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (he != hipSuccess) return c->fail(DAO_EDEVICE, std::string("read timing: ") + hipGetErrorString(he));
    *us_per_launch = tot / iters;
    return DAO_OK;
}

dao_status dao_profile_phases(dao_ctx* c, double* us) {
    if (!c || !us) return DAO_EINVAL;
    for (int i = 0; i < PROF_PHASES; ++i) us[i] = c->prof_phase_us[i];
    return DAO_OK;
}

dao_status dao_profile_start(dao_ctx* c, int32_t kernel) {
    if (!c) return DAO_EINVAL;
    if (kernel < 0 || kernel > 4) return c->fail(DAO_EINVAL, "kernel must be in [0, 4]");
    if (kernel == 4 && !c->coop_master()) return c->fail(DAO_ESTATE, "the persistent master is not in use");
    if (kernel < 4 && c->coop_master()) return c->fail(DAO_ESTATE, "the per-phase kernels are not in use");
    if (!c->ap_master()) return c->fail(DAO_ESTATE, "profiling covers the aperture-matrix master");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemsetAsync(c->pc, 0, sizeof(ProfCounters), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->prof_kernel = kernel;
    c->prof_used = 0;
    return DAO_OK;
}

dao_status dao_profile_stop(dao_ctx* c, int64_t* launches, int64_t* working_launches, double* total_us,
                            double* total_bytes) {
    if (!c) return DAO_EINVAL;
    const int k = c->prof_kernel;
    if (k < 0) return c->fail(DAO_ESTATE, "profiling was not started");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double us = 0.0;
    for (size_t i = 0; i + 1 < c->prof_used; i += 2) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->prof_events[i], c->prof_events[i + 1]));
        us += 1e3 * double(ms);
    }
    HIPCHK(c, hipMemcpyAsync(c->pc_h, c->pc, sizeof(ProfCounters), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (k == 4) {
        int rate_khz = 0;
        HIPCHK(c, hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, c->device));
        for (int i = 0; i < PROF_PHASES; ++i)
            c->prof_phase_us[i] = rate_khz > 0 ? 1e3 * double(c->pc_h->ticks[i]) / rate_khz : 0.0;
    }
    if (launches) *launches = int64_t(c->prof_used / 2);
    if (working_launches) *working_launches = k == 4 ? int64_t(c->prof_used / 2) : int64_t(c->pc_h->real[k]);
    if (total_us) *total_us = us;
    if (total_bytes)
        *total_bytes = k == 4 ? c->pc_h->bytes[0] + c->pc_h->bytes[1] + c->pc_h->bytes[2] : c->pc_h->bytes[k];
    c->prof_kernel = -1;
    c->prof_used = 0;
    return DAO_OK;
}

dao_status dao_solve_batch(dao_ctx* const* ctxs, int32_t n, const int32_t* n_apertures, dao_plan* plans) {
    if (!ctxs || !n_apertures || n < 1 || n > MAX_BATCH) return DAO_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return DAO_EINVAL;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return ctxs[i]->fail(DAO_EINVAL, "a context appears twice in the batch");
        if (ctxs[i]->dtype != ctxs[0]->dtype) return ctxs[i]->fail(DAO_EINVAL, "contexts of one batch share the dtype");
        if (n_apertures[i] < 0 || n_apertures[i] > ctxs[i]->opt.max_apertures)
            return ctxs[i]->fail(DAO_EINVAL, "n_apertures must be in [0, max_apertures]");
    }
    return ctxs[0]->dtype == DAO_F64 ? solve_batch_typed<double>(ctxs, n, n_apertures, plans)
                                     : solve_batch_typed<float>(ctxs, n, n_apertures, plans);
}

dao_status dao_get_state(dao_ctx* c, int32_t cap, int32_t* beams, int16_t* leaves, double* y,
                         dao_state_info* info) {
    if (!c) return DAO_EINVAL;
    if (!info) return c->fail(DAO_EINVAL, "null state info");
    const int m = std::min<int>(std::max(cap, 0), c->K);
    if (m > 0 && (!beams || !leaves || !y)) return c->fail(DAO_EINVAL, "null state arrays");
    if (m < c->K) return c->fail(DAO_EINVAL, "cap is smaller than the pool");
    dao_status s = dao_get_pool(c, cap, nullptr, beams, leaves, y);
    if (s != DAO_OK) return s;
    HIPCHK(c, hipMemcpyAsync(c->ms_h, c->ms, sizeof(MasterState), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    info->n = c->K;
    info->tighten = c->loop_tighten;
    info->rc1 = c->loop_rc1;
    info->eps = c->loop_eps > 0.0 ? c->loop_eps : c->opt.eps;
    info->last_step = c->ms_h->last_step;
    info->prev_step = c->ms_h->prev_step;
    return DAO_OK;
}

dao_status dao_set_state(dao_ctx* c, const dao_state_info* info, const int32_t* beams, const int16_t* leaves,
                         const double* y) {
    if (!c) return DAO_EINVAL;
    if (!info) return c->fail(DAO_EINVAL, "null state info");
    const int n = info->n;
    if (n < 0 || n > c->opt.max_apertures) return c->fail(DAO_EINVAL, "pool size out of range");
    if (n > 0 && (!beams || !leaves || !y)) return c->fail(DAO_EINVAL, "null state arrays");
    if (!(info->eps > 0.0) || !std::isfinite(info->eps)) return c->fail(DAO_EINVAL, "eps must be finite and > 0");
    if (info->tighten < 0) return c->fail(DAO_EINVAL, "negative tighten count");
    if (!(info->last_step >= 0.0) || !(info->prev_step >= 0.0) || !std::isfinite(info->last_step) ||
        !std::isfinite(info->prev_step))
        return c->fail(DAO_EINVAL, "step history must be finite and >= 0");
    if (!std::isnan(info->rc1) && !std::isfinite(info->rc1)) return c->fail(DAO_EINVAL, "rc1 must be finite or NaN");
    for (int k = 0; k < n; ++k) {
        dao_status s = check_aperture(c, beams[k], leaves + size_t(k) * 2 * c->maxRB);
        if (s != DAO_OK) return s;
        if (!(y[k] >= 0.0) || !std::isfinite(y[k])) return c->fail(DAO_EINVAL, "intensities must be finite and >= 0");
    }
    return c->dtype == DAO_F64 ? set_state_typed<double>(c, info, beams, leaves, y)
                               : set_state_typed<float>(c, info, beams, leaves, y);
}

dao_status dao_solve_resume(dao_ctx* c, int32_t n_apertures, dao_plan* out) {
    if (!c) return DAO_EINVAL;
    if (n_apertures < 0 || n_apertures > c->opt.max_apertures)
        return c->fail(DAO_EINVAL, "n_apertures must be in [0, max_apertures]");
    dao_status s = c->dtype == DAO_F64 ? solve_typed<double>(c, n_apertures, out, true)
                                       : solve_typed<float>(c, n_apertures, out, true);
    if (s != DAO_OK) return s;
    return out ? dao_status(out->stop) : DAO_OK;
}

dao_status dao_solve(dao_ctx* c, int32_t n_apertures, dao_plan* out) {
    if (!c) return DAO_EINVAL;
    if (n_apertures < 0 || n_apertures > c->opt.max_apertures)
        return c->fail(DAO_EINVAL, "n_apertures must be in [0, max_apertures]");
    dao_status s = c->dtype == DAO_F64 ? solve_typed<double>(c, n_apertures, out)
                                       : solve_typed<float>(c, n_apertures, out);
    if (s != DAO_OK) return s;
    return out ? dao_status(out->stop) : DAO_OK;
}

}  // extern "C"

// ===========================================================================
// Serving loop: continuous batching of solves under a device-memory cap
// ===========================================================================
// A worker thread admits queued requests (first come, first served): it
// builds each context (host layout, uploads on its own stream) while the
// device works on the live solves, as long as the live plus admitted
// contexts stay within max_live and the memory cap.  dao_server_step takes
// the admitted contexts in and advances every live solve by one round.
struct dao_server {
    hipStream_t stream = nullptr;   // solves
    std::vector<hipStream_t> uploads;   // context creation, one per admission thread
    int max_live = 8;
    int64_t cap = 0;                // 0: no cap
    bool batch_masters = true;
    struct Req {
        const dao_matrix* D;
        const dao_beams* B;
        const dao_structures* S;
        const dao_prescription* P;
        dao_options opt;
        int32_t n_ap;
        int64_t ticket;
    };
    struct Admitted {
        Req q;
        dao_ctx* c;
        dao_status st;
        std::string err;
    };
    struct Result {
        dao_status status = DAO_OK;
        dao_plan plan{};
        std::vector<int32_t> beam, steps;
        std::vector<double> rc, gap, kkt, F;
        std::string error;
    };
    struct Live {
        dao_ctx* c = nullptr;
        PlanRun run;
        int64_t ticket = 0;
        int64_t bytes = 0;
    };
    // shared with the worker (under mu)
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::deque<Req> queue;
    std::deque<Admitted> admitted;
    int64_t used = 0;   // device bytes of admitted and live contexts, and reserved by creations
    int n_live = 0;
    std::set<int64_t> building;   // tickets taken off the queue whose contexts are being built
    // main thread only
    std::vector<std::unique_ptr<Live>> live;
    std::map<int64_t, Result> done;
    std::map<int64_t, Result> running;   // results being filled by live solves
    int64_t next_ticket = 0;
    std::vector<std::thread> workers;
};

namespace {

// An admission thread: takes the oldest queued request while fewer than
// max_live solves are live, admitted or being built, lays out its inputs
// (host only), reserves its predicted device footprint under the cap
// (waiting for retirements while it does not fit), then allocates and
// uploads on its own stream.  Several threads build contexts at once; each
// request is admitted when its context is ready.
void server_worker(dao_server* sv, int w) {
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        sv->cv.wait(lk, [&] {
            return sv->stop ||
                   (!sv->queue.empty() &&
                    sv->n_live + int(sv->admitted.size()) + int(sv->building.size()) < sv->max_live);
        });
        if (sv->stop) return;
        dao_server::Req q = sv->queue.front();
        sv->queue.pop_front();
        sv->building.insert(q.ticket);
        lk.unlock();
        dao_options o = q.opt;
        std::unique_ptr<HostLayout> L;
        int64_t need = 0;
        dao_status st = prepare_layout(q.D, q.B, q.S, q.P, &o, &L, &need);
        std::string err = st == DAO_OK ? std::string() : std::string(dao_create_error());
        lk.lock();
        bool reserved = false;
        if (st == DAO_OK && sv->cap > 0 && need > sv->cap) {
            st = DAO_ENOMEM;
            err = "device footprint " + std::to_string(need) + " B exceeds the server's hbm_cap_bytes";
        }
        if (st == DAO_OK) {
            if (sv->cap > 0) sv->cv.wait(lk, [&] { return sv->stop || sv->used + need <= sv->cap; });
            if (sv->stop) {
                sv->building.erase(q.ticket);
                return;
            }
            sv->used += need;
            reserved = true;
        }
        lk.unlock();
        dao_ctx* c = nullptr;
        if (st == DAO_OK) {
            st = create_on_device(std::move(L), q.B, o, sv->uploads[size_t(w)], &c);
            if (st != DAO_OK) err = dao_create_error();
            if (st == DAO_OK && hipStreamSynchronize(sv->uploads[size_t(w)]) != hipSuccess) {
                dao_destroy(c);
                c = nullptr;
                st = DAO_EDEVICE;
                err = "upload failed";
            }
        }
        lk.lock();
        if (reserved) sv->used -= need;
        if (st == DAO_OK) {
            c->stream = sv->stream;   // the solve runs on the serving stream
            sv->used += c->device_bytes;
        }
        sv->building.erase(q.ticket);
        sv->admitted.push_back(dao_server::Admitted{q, c, st, err});
        sv->cv.notify_all();
    }
}

void server_retire(dao_server* sv, size_t i, dao_status st, const char* why) {
    dao_server::Live& L = *sv->live[i];
    auto it = sv->running.find(L.ticket);
    dao_server::Result r = std::move(it->second);
    sv->running.erase(it);
    r.status = st == DAO_OK ? dao_status(L.run.stop) : st;
    if (why) r.error = why;
    r.plan.round_beam = r.beam.data();
    r.plan.round_steps = r.steps.data();
    r.plan.round_rc = r.rc.data();
    r.plan.round_gap = r.gap.data();
    r.plan.round_kkt = r.kkt.data();
    r.plan.round_F = r.F.data();
    sv->done[L.ticket] = std::move(r);
    dao_destroy(L.c);
    const int64_t bytes = L.bytes;
    sv->live.erase(sv->live.begin() + long(i));
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->used -= bytes;
        sv->n_live = int(sv->live.size());
    }
    sv->cv.notify_all();
}

// Take the contexts the worker has admitted into the live set.
void server_take_admitted(dao_server* sv) {
    std::deque<dao_server::Admitted> got;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        got.swap(sv->admitted);
        sv->n_live = int(sv->live.size() + got.size());
    }
    for (auto& a : got) {
        dao_server::Result r;
        if (a.st != DAO_OK) {
            r.status = a.st;
            r.error = a.err;
            sv->done[a.q.ticket] = std::move(r);
            std::lock_guard<std::mutex> g(sv->mu);
            sv->n_live -= 1;
            continue;
        }
        dao_ctx* c = a.c;
        const int n = std::max(1, int(a.q.n_ap));
        r.beam.assign(n, 0);
        r.steps.assign(n, 0);
        r.rc.assign(n, 0.0);
        r.gap.assign(n, 0.0);
        r.kkt.assign(n, 0.0);
        r.F.assign(n, 0.0);
        sv->running[a.q.ticket] = std::move(r);
        dao_server::Result& rr = sv->running[a.q.ticket];
        rr.plan.round_beam = rr.beam.data();
        rr.plan.round_steps = rr.steps.data();
        rr.plan.round_rc = rr.rc.data();
        rr.plan.round_gap = rr.gap.data();
        rr.plan.round_kkt = rr.kkt.data();
        rr.plan.round_F = rr.F.data();
        auto L = std::make_unique<dao_server::Live>();
        L->c = c;
        L->ticket = a.q.ticket;
        L->bytes = c->device_bytes;
        L->run.c = c;
        L->run.n_ap = std::min(a.q.n_ap, c->opt.max_apertures);
        L->run.out = &rr.plan;
        const dao_status s2 = c->dtype == DAO_F64 ? plan_start<double>(L->run) : plan_start<float>(L->run);
        sv->live.push_back(std::move(L));
        if (s2 != DAO_OK) server_retire(sv, sv->live.size() - 1, s2, c->err.c_str());
    }
    sv->cv.notify_all();
}

}  // namespace

extern "C" {

dao_status dao_server_create(const dao_server_options* o, void* stream, dao_server** out) {
    if (!out || !o || o->max_live < 1 || o->max_live > MAX_BATCH || o->hbm_cap_bytes < 0 ||
        (o->batch_masters != 0 && o->batch_masters != 1) || o->workers < 0 || o->workers > 16)
        return DAO_EINVAL;
    auto* sv = new dao_server();
    sv->stream = static_cast<hipStream_t>(stream);
    sv->max_live = o->max_live;
    sv->cap = o->hbm_cap_bytes;
    sv->batch_masters = o->batch_masters != 0;
    const int nw = o->workers > 0 ? o->workers : 4;
    for (int w = 0; w < nw; ++w) {
        hipStream_t u = nullptr;
        if (hipStreamCreateWithFlags(&u, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : sv->uploads) (void)hipStreamDestroy(x);
            delete sv;
            return DAO_EDEVICE;
        }
        sv->uploads.push_back(u);
    }
    for (int w = 0; w < nw; ++w) sv->workers.emplace_back(server_worker, sv, w);
    *out = sv;
    return DAO_OK;
}

void dao_server_destroy(dao_server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->stop = true;
    }
    sv->cv.notify_all();
    for (auto& t : sv->workers)
        if (t.joinable()) t.join();
    for (auto& a : sv->admitted)
        if (a.c) dao_destroy(a.c);
    sv->admitted.clear();
    while (!sv->live.empty()) server_retire(sv, sv->live.size() - 1, DAO_ESTATE, "server destroyed");
    for (auto u : sv->uploads) (void)hipStreamDestroy(u);
    delete sv;
}

dao_status dao_server_submit(dao_server* sv, const dao_matrix* D, const dao_beams* beams, const dao_structures* structs,
                             const dao_prescription* presc, const dao_options* opt, int32_t n_apertures,
                             int64_t* ticket) {
    if (!sv || !D || !beams || !structs || !ticket || n_apertures < 0) return DAO_EINVAL;
    dao_server::Req q{D, beams, structs, presc, {}, n_apertures, 0};
    if (opt)
        q.opt = *opt;
    else
        dao_default_options(&q.opt);
    {
        std::lock_guard<std::mutex> g(sv->mu);
        q.ticket = sv->next_ticket++;
        sv->queue.push_back(q);
    }
    sv->cv.notify_all();
    *ticket = q.ticket;
    return DAO_OK;
}

dao_status dao_server_step(dao_server* sv, int32_t* n_live, int32_t* n_done) {
    if (!sv) return DAO_EINVAL;
    server_take_admitted(sv);
    int finished = 0;
    std::vector<PlanRun*> need32, need64;
    for (size_t i = 0; i < sv->live.size();) {
        dao_server::Live& L = *sv->live[i];
        const dao_status s = L.c->dtype == DAO_F64 ? plan_round_begin<double>(L.run) : plan_round_begin<float>(L.run);
        if (s != DAO_OK) {
            server_retire(sv, i, s, L.c->err.c_str());
            ++finished;
            continue;
        }
        if (L.run.finished) {
            const dao_status f = plan_finish(L.run);
            server_retire(sv, i, f, nullptr);
            ++finished;
            continue;
        }
        (L.c->dtype == DAO_F64 ? need64 : need32).push_back(&L.run);
        ++i;
    }
    dao_status s = DAO_OK;
    if (sv->batch_masters) {
        // small solves (fewer rows than a few batches per workgroup of the
        // whole grid) share one launch; a large solve keeps the whole grid
        auto run_group = [&](std::vector<PlanRun*>& need, auto tag) -> dao_status {
            using T = decltype(tag);
            std::vector<PlanRun*> small;
            for (PlanRun* r : need) {
                const int64_t rows_per_wg = r->c->Vpad / std::max(1, r->c->coop_grid);
                if (rows_per_wg < 4 * Batch<T>::ROWS)
                    small.push_back(r);
                else {
                    const dao_status e = run_master<T>(r->c, r->tol, r->c->opt.max_steps);
                    if (e != DAO_OK) return e;
                }
            }
            return small.empty() ? DAO_OK : run_master_batch<T>(small);
        };
        if (!need32.empty()) s = run_group(need32, float{});
        if (s == DAO_OK && !need64.empty()) s = run_group(need64, double{});
    } else {
        // each master with the whole grid, one after another
        for (PlanRun* r : need32)
            if (s == DAO_OK) s = run_master<float>(r->c, r->tol, r->c->opt.max_steps);
        for (PlanRun* r : need64)
            if (s == DAO_OK) s = run_master<double>(r->c, r->tol, r->c->opt.max_steps);
    }
    if (s != DAO_OK) {
        // a device error: every live solve ends with it
        while (!sv->live.empty()) server_retire(sv, sv->live.size() - 1, s, "master solve failed");
        if (n_live) *n_live = 0;
        if (n_done) *n_done = finished;
        return s;
    }
    for (auto& L : sv->live) plan_round_end(L->run);
    if (n_live) *n_live = int32_t(sv->live.size());
    if (n_done) *n_done = finished;
    return DAO_OK;
}

dao_status dao_server_poll(dao_server* sv, int64_t ticket, int32_t* state, dao_plan* out) {
    if (!sv || !state) return DAO_EINVAL;
    auto it = sv->done.find(ticket);
    if (it == sv->done.end()) {
        if (sv->running.count(ticket)) {
            *state = 1;
            return DAO_OK;
        }
        std::lock_guard<std::mutex> g(sv->mu);
        for (const auto& a : sv->admitted)
            if (a.q.ticket == ticket) {
                *state = 0;
                return DAO_OK;
            }
        for (const auto& q : sv->queue)
            if (q.ticket == ticket) {
                *state = 0;
                return DAO_OK;
            }
        if (sv->building.count(ticket)) {
            *state = 0;
            return DAO_OK;
        }
        return DAO_EINVAL;   // unknown or already collected
    }
    *state = 2;
    const dao_server::Result& r = it->second;
    if (out) {
        const int n = r.plan.rounds;
        out->rounds = r.plan.rounds;
        out->stop = r.plan.stop;
        out->F = r.plan.F;
        out->rc1 = r.plan.rc1;
        out->total_steps = r.plan.total_steps;
        out->total_ls_evals = r.plan.total_ls_evals;
        out->price_s = r.plan.price_s;
        out->master_s = r.plan.master_s;
        if (out->round_beam) std::copy(r.beam.begin(), r.beam.begin() + n, out->round_beam);
        if (out->round_steps) std::copy(r.steps.begin(), r.steps.begin() + n, out->round_steps);
        if (out->round_rc) std::copy(r.rc.begin(), r.rc.begin() + n, out->round_rc);
        if (out->round_gap) std::copy(r.gap.begin(), r.gap.begin() + n, out->round_gap);
        if (out->round_kkt) std::copy(r.kkt.begin(), r.kkt.begin() + n, out->round_kkt);
        if (out->round_F) std::copy(r.F.begin(), r.F.begin() + n, out->round_F);
    }
    const dao_status st = r.status;
    sv->done.erase(it);
    return st;
}

dao_status dao_server_info(const dao_server* sv_c, int32_t* queued, int32_t* live, int64_t* used_bytes) {
    if (!sv_c) return DAO_EINVAL;
    auto* sv = const_cast<dao_server*>(sv_c);
    std::lock_guard<std::mutex> g(sv->mu);
    if (queued) *queued = int32_t(sv->queue.size() + sv->admitted.size() + sv->building.size());
    if (live) *live = int32_t(sv->live.size());
    if (used_bytes) *used_bytes = sv->used;
    return DAO_OK;
}

}  // extern "C"
