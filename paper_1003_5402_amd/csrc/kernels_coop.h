// Persistent cooperative master over the aperture dose matrix (gfx950).
//
// One cooperative launch runs a whole master solve (Section 2.3's gradient
// projection, same step rule and line search as the per-phase kernels of
// kernels_ap.h).  The grid is co-resident (cooperative launch), each
// workgroup owns a fixed set of voxel-row batches for the whole solve (a
// contiguous range with D_K on chip, batches dealt with a skew otherwise),
// so the per-voxel vectors d and q are only ever touched by their owner and
// need no cross-workgroup coherence.  The only data that crosses
// workgroups are the small reduction records (objective, grad_y, line-search
// sums), moved with agent-scope atomic loads and stores (coherent across
// XCDs without writing back or invalidating caches).  Every workgroup then
// takes the same decisions from the same broadcast totals, so the direction,
// the line-search trial points and the intensities y are computed
// redundantly (and identically) in every workgroup instead of being
// broadcast.
//
// Grid-wide reduction: each workgroup publishes its record in one of two
// alternating buffers, waits for the data stores to complete, then raises its
// own flag to the reduction's sequence number.  Every workgroup polls all
// flags (one per thread) and then sums all records itself in a fixed order,
// identical everywhere, so no workgroup has to wait for a combining
// workgroup.  Two buffers suffice: a
// workgroup can only write a buffer again after every workgroup has raised
// its flag for the reduction in between, which each does only after it has
// finished reading.  Waits are bounded: a workgroup that waits too long
// raises an abort flag that every waiter checks, so the grid always drains.
#pragma once

#include "kernels_ap.h"

namespace dao {

constexpr int COOP_THREADS = 512;          // threads per workgroup: 8 wavefronts, 2 per SIMD
constexpr int RECW = KS + 8;               // doubles per reduction record
constexpr int MAX_COOP_GRID = 1024;        // workgroups of one persistent launch
constexpr long SPIN_LIMIT = 4000000L;      // ~1 s of waiting before the grid aborts

struct CoopSync {
    uint32_t abort_flag[SLOT_STRIDE];
    uint32_t flag[MAX_COOP_GRID * SLOT_STRIDE];   // one 128-byte line per workgroup
};

__device__ __forceinline__ double aload(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void astore(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t aload_u(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Combine of one record field: sums, except the line-search record's
// nearest-breakpoint fields (3: minimum, 4: maximum).
template <bool LS>
__device__ __forceinline__ double rec_comb(int i, double a, double b) {
    if (LS && i == 3) return fmin(a, b);
    if (LS && i == 4) return fmax(a, b);
    return a + b;
}
template <bool LS>
__device__ __forceinline__ double rec_init(int i) {
    if (LS && i == 3) return INFINITY;
    if (LS && i == 4) return -INFINITY;
    return 0.0;
}

__device__ __forceinline__ double field_reduce_dpp(bool ls, int f, double v) {
    if (ls && f == 3) return wave_reduce_dpp<1>(v);
    if (ls && f == 4) return wave_reduce_dpp<2>(v);
    return wave_reduce_dpp<0>(v);
}

// Fixed-order combine of the 8 wavefronts' partials part[w * stride + f]
// (f < nf) into out[f] (LDS): lane group f of 8 lanes holds the 8 partials
// of field f and combines them by three DPP moves inside the group (quad
// swaps, then half-row mirror).  With ls, fields 3 and 4 are a minimum and
// a maximum, the others sums.  Needs 8 wavefronts; all threads call it.
__device__ __forceinline__ void combine_waves8(const double* part, int stride, int nf, bool ls, double* out) {
    const int t = threadIdx.x, wave = t / WAVE;
    if (wave < (nf * 8 + WAVE - 1) / WAVE) {   // whole wavefronts take part in the moves
        const int f = t / 8, w = t % 8;
        const int op = (ls && f == 3) ? 1 : (ls && f == 4) ? 2 : 0;
        const double id = op == 0 ? 0.0 : op == 1 ? INFINITY : -INFINITY;
        double x = f < nf ? part[w * stride + f] : id;
        double m = dpp_move<0xB1, 0xF>(x, id);    // quad_perm [1,0,3,2]
        x = op == 0 ? x + m : op == 1 ? fmin(x, m) : fmax(x, m);
        m = dpp_move<0x4E, 0xF>(x, id);           // quad_perm [2,3,0,1]
        x = op == 0 ? x + m : op == 1 ? fmin(x, m) : fmax(x, m);
        m = dpp_move<0x141, 0xF>(x, id);          // row_half_mirror
        x = op == 0 ? x + m : op == 1 ? fmin(x, m) : fmax(x, m);
        if (w == 0 && f < nf) out[f] = x;
    }
    __syncthreads();
}

// Line-search record of a workgroup (fields as Rec: s0, s1, s2, mn, mx, s5)
// into out[0..6) (LDS), waves combined in a fixed order.  Needs 8
// wavefronts; all threads call it.
__device__ __forceinline__ void block_rec_dpp(const Rec& r, double* out) {
    __shared__ double s_w[1024 / WAVE][6];
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const double v0 = wave_reduce_dpp<0>(r.s0), v1 = wave_reduce_dpp<0>(r.s1), v2 = wave_reduce_dpp<0>(r.s2);
    const double v3 = wave_reduce_dpp<1>(r.mn), v4 = wave_reduce_dpp<2>(r.mx), v5 = wave_reduce_dpp<0>(r.s5);
    if (lane == 0) {
        s_w[wave][0] = v0;
        s_w[wave][1] = v1;
        s_w[wave][2] = v2;
        s_w[wave][3] = v3;
        s_w[wave][4] = v4;
        s_w[wave][5] = v5;
    }
    __syncthreads();
    combine_waves8(&s_w[0][0], 6, 6, true, out);
}

// Fixed-order combine of nb records of W doubles stored field-major (field i
// of workgroup b at buf[i * nb + b]) into out[0..W) (LDS).  Wavefront w takes
// fields w, w + nw, ...; lane l reduces records l, l + 64, ... of each field
// in that order, all its loads of a pass in flight together (coalesced
// across lanes); the lanes then combine by wave_reduce_dpp.  Every workgroup
// runs the same code on the same data, so all get the same bits.
// Needs W <= FMAX * wavefronts.
template <bool LS, int FMAX>
__device__ __forceinline__ void combine_fields(const double* buf, uint32_t nb, int W, double* out) {
    constexpr int L = 4;
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    const int nf = wave < W ? (W - wave + nw - 1) / nw : 0;
    double acc[FMAX];
#pragma unroll
    for (int i = 0; i < FMAX; ++i) acc[i] = rec_init<LS>(wave + nw * i);
    for (uint32_t q0 = 0; q0 < nb; q0 += L * WAVE) {
        double v[FMAX][L];
#pragma unroll
        for (int i = 0; i < FMAX; ++i)
#pragma unroll
            for (int u = 0; u < L; ++u) {
                const int f = wave + nw * i;
                const uint32_t rec = q0 + u * WAVE + lane;
                v[i][u] = (i < nf && rec < nb) ? aload(buf + size_t(f) * nb + rec) : rec_init<LS>(f);
            }
#pragma unroll
        for (int i = 0; i < FMAX; ++i)
#pragma unroll
            for (int u = 0; u < L; ++u) acc[i] = rec_comb<LS>(wave + nw * i, acc[i], v[i][u]);
    }
#pragma unroll
    for (int i = 0; i < FMAX; ++i) {
        if (i < nf) {
            const int f = wave + nw * i;
            const double tot = field_reduce_dpp(LS, f, acc[i]);
            if (lane == 0) out[f] = tot;
        }
    }
    __syncthreads();
}

// Grid-wide fixed-order reduction of W-double records over the nb workgroups
// of one solve (all their threads call it; b is this workgroup's index among
// them).  recs: two field-major buffers of nb records;
// mine: this workgroup's record (LDS); total: result (LDS, every workgroup);
// seq: this workgroup's count of reductions so far.  Returns false when the
// grid aborted.
template <bool LS>
__device__ bool grid_reduce(CoopSync* S, double* recs, const double* mine, int W, double* total,
                            uint32_t& seq, uint32_t b, uint32_t nb) {
    __shared__ int s_ok;
    seq += 1;
    double* buf = recs + size_t(seq & 1u) * nb * RECW;
    for (int i = threadIdx.x; i < W; i += blockDim.x) astore(&buf[size_t(i) * nb + b], mine[i]);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_store(&S->flag[b * SLOT_STRIDE], seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_ok = 1;
    }
    __syncthreads();
    for (uint32_t w = threadIdx.x; w < nb; w += blockDim.x) {
        long spins = 0;
        while (aload_u(&S->flag[w * SLOT_STRIDE]) < seq) {
            __builtin_amdgcn_s_sleep(1);
            if (aload_u(&S->abort_flag[0])) {
                s_ok = 0;
                break;
            }
            if (++spins > SPIN_LIMIT) {
                __hip_atomic_store(&S->abort_flag[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_ok = 0;
                break;
            }
        }
    }
    __syncthreads();
    if (!s_ok) return false;
    combine_fields<LS, LS ? (6 + COOP_THREADS / WAVE - 1) / (COOP_THREADS / WAVE)
                             : (KS + 1 + COOP_THREADS / WAVE - 1) / (COOP_THREADS / WAVE)>(buf, nb, W, total);
    return true;
}

// Line-search state kept in registers by every thread (the fields
// ls_decide uses).
struct LsRegs {
    double t, t_max, lo, hi;
    int hi_known, ls_iter;
    int64_t total_ls;
};

template <class T>
struct CoopArgs {
    const void* dk;     // D_K (KS slots per row, blocked by batch), storage type DT of the kernel
    double dk_scale;    // D_K = dk_scale * stored value (1 unless stored in FP16)
    int64_t Vpad, Vnz;
    double* d;
    T* q;
    const uint8_t* cls;
    const ObjClass* classes;
    int ncls;
    double* y;          // in: current intensities; out: final intensities (workgroup 0)
    double* p;          // out: last direction (workgroup 0)
    double* grad;       // out: last grad_y (workgroup 0)
    CgMem* cgm;         // in/out: conjugate-direction memory (with p: the last step's direction)
    const double* tau;  // per-voxel threshold shifts by internal row (null: none)
    MasterState* ms;    // in: state set by k_master_init_ap; out: final state (workgroup 0)
    double* recs;       // [2][workgroups of the solve][RECW]
    double* bpart;      // streaming form: grad_y partial of every batch (KS doubles each)
    CoopSync* sync;
    ProfCounters* pc;
    int timing;         // workgroup 0 accumulates per-phase wall-clock ticks in pc->ticks
};

// Rows of a workgroup: in the forms that stream D_K the batches of ROWS rows
// are dealt to the workgroups (coop_batch and coop_nbatches, dao_common.h).
// The most batches a workgroup owns (LDS sizing).  With D_K on chip a
// workgroup owns a contiguous range of that many batches (the last ones
// fewer): the update pass's skipped batches cost little there, D_K being read
// from LDS, so its rows need no dealing.
template <class T>
__host__ __device__ inline int64_t coop_batches_per_group(int64_t Vpad, int grid) {
    const int64_t nbat = Vpad / Batch<T>::ROWS;
    return (nbat + grid - 1) / grid;
}
// The update pass's LDS (hybrid form): dF/dz of every row (double), then
// each batch's grad_y partial (KS doubles), then each batch's mask of rows
// with dF/dz != 0 (64 bits).
template <class DT>
__host__ __device__ inline size_t coop_upd_lds(int64_t rows) {
    const int64_t nb = rows / Batch<DT>::ROWS;
    return size_t(rows) * 8 + size_t(nb) * KS * 8 + size_t(nb) * 8;
}

// Dynamic LDS of the streaming form: per wavefront, the per-slot partials of
// one batch's rows in the q pass (ROWS rows of LPR + 1 doubles; the pad
// spreads a lane's row reads over the banks).
template <class DT>
__host__ __device__ constexpr size_t coop_stream_lds() {
    return size_t(COOP_THREADS / WAVE) * Batch<DT>::ROWS * (DKG<DT>::LPR + 1) * sizeof(double);
}

// 16-byte vectors per on-chip D_K row: the nc the pool needs, rounded up to
// an odd count, so that lanes reading consecutive rows at the same slot
// (the line search's one row per thread) fall in distinct LDS banks.
__host__ __device__ inline int coop_row_vecs(int nc) { return nc | 1; }

// Dynamic LDS of the LDS-resident variant: the workgroup's D_K rows
// (coop_row_vecs(nc) 16-byte vectors each), then d, the two breakpoints
// (double), q (T), class (uint8).
template <class T>
__host__ __device__ inline size_t coop_lds_bytes(int64_t rows, int nc) {
    return size_t(rows) * coop_row_vecs(nc) * 16 + size_t(rows) * (3 * 8 + sizeof(T) + 1) + 64;
}
// Dynamic LDS of the hybrid form: the larger of the q pass's row partials
// and the update pass's area (coop_upd_lds), then the workgroup's d
// (double), q (T) and class (uint8).
template <class DT>
__host__ __device__ inline size_t coop_hybrid_front(int64_t rows) {
    const size_t a = coop_stream_lds<DT>(), b = coop_upd_lds<DT>(rows);
    return a > b ? a : b;
}
template <class T, class DT>
__host__ __device__ inline size_t coop_hybrid_lds(int64_t rows) {
    return coop_hybrid_front<DT>(rows) + size_t(rows) * (8 + sizeof(T) + 1) + 64;
}

// The three forms of the persistent master (FORM):
//   COOP_STREAM  every pass streams D_K, d, q and the classes from device memory;
//   COOP_HYBRID  D_K streamed; the workgroup keeps its rows of d, q and the
//                classes in LDS for the whole solve (d written back at the end);
//   COOP_CHIP    D_K too: the workgroup copies its rows of D_K into LDS once per
//                solve and keeps the breakpoints of each direction there.
constexpr int COOP_STREAM = 0, COOP_HYBRID = 1, COOP_CHIP = 2;
template <class T, class DT, int FORM>
__device__ __forceinline__ void master_body(const CoopArgs<T>& A, const uint32_t gb, const uint32_t gn) {
    constexpr bool LDSRES = FORM == COOP_CHIP;      // D_K on chip
    constexpr bool VEC_LDS = FORM != COOP_STREAM;   // d, q and the classes on chip
    using G = DKG<DT>;
    using V = typename Vec16<DT>::type;
    constexpr int IT = Batch<DT>::ITERS, ROWS = Batch<DT>::ROWS;
    const DT* dk = static_cast<const DT*>(A.dk);
    const double dks = A.dk_scale;
    constexpr int NW = COOP_THREADS / WAVE;
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ MasterState s_ms;
    __shared__ ObjClass cl[256];
    __shared__ double s_y[KS], s_p[KS], s_g[KS], s_r[KS];
    __shared__ int s_fr[KS];
    __shared__ double s_rec[RECW], s_tot[RECW];
    static_assert(NW == 8, "the wavefront combines assume 8 wavefronts");
    __shared__ double s_acc[NW][RECW];   // per wavefront: grad_y (the final objective in field 0)
    __shared__ double s_u[NW][ROWS];
    __shared__ int s_go;

    ms_load(s_ms, A.ms);
    for (int i = threadIdx.x; i < A.ncls; i += blockDim.x) cl[i] = A.classes[i];
    const int K = s_ms.K;
    // the conjugate memory of the pool's last step, if any
    const bool mem0 = s_ms.conj && s_ms.cg_valid;
    for (int k = threadIdx.x; k < KS; k += blockDim.x) {
        const bool in = k < K;
        s_y[k] = in ? A.y[k] : 0.0;
        s_p[k] = in && mem0 ? A.p[k] : 0.0;
        s_r[k] = in && mem0 ? A.cgm->r[k] : 0.0;
        s_fr[k] = in && mem0 ? A.cgm->free[k] : 0;
        s_g[k] = 0.0;
    }
    __syncthreads();
    uint32_t seq = 0;   // grid reductions so far (the flags start at 0 every launch)

    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int rg = lane / G::LPR, c = lane % G::LPR;
    const int nc = (K + G::EPL - 1) / G::EPL;
    // this workgroup's batches of ROWS rows: local batch lb (local rows
    // lb * ROWS ...) is batch bat0 + lb (D_K on chip) or coop_batch(lb, gb, gn)
    const int64_t nbat = A.Vpad / ROWS;
    const int64_t per = coop_batches_per_group<DT>(A.Vpad, gn);
    const int64_t bat0 = LDSRES ? min(nbat, int64_t(gb) * per) : 0;
    const int64_t nlb = LDSRES ? min(nbat, bat0 + per) - bat0 : coop_nbatches(nbat, gb, gn);
    const int64_t nrows = nlb * ROWS, rows_max = per * ROWS;   // rows_max: the LDS layout's row count
    auto batch_base = [&](int64_t lb) -> int64_t {
        return LDSRES ? (bat0 + lb) * ROWS : coop_batch(lb, gb, gn) * ROWS;
    };
    // on-chip copies: D_K rows (COOP_CHIP) or the q-pass partials
    // (COOP_HYBRID), then d, the breakpoints (COOP_CHIP), q and the classes
    V* dkl = reinterpret_cast<V*>(dyn);
    const int ncp = coop_row_vecs(nc);   // LDS row stride in vectors
    double* dl = reinterpret_cast<double*>(dyn + (LDSRES ? size_t(rows_max) * ncp * 16
                                                         : coop_hybrid_front<DT>(rows_max)));
    double* bul = dl + rows_max;   // breakpoints of the current direction
    double* bol = bul + rows_max;
    T* ql = reinterpret_cast<T*>(LDSRES ? bol + rows_max : dl + rows_max);
    uint8_t* cll = reinterpret_cast<uint8_t*>(ql + rows_max);
    // update pass of the hybrid form (at the front, where the q pass keeps
    // its row partials): dF/dz per row, then per batch its grad_y partial
    // and its mask of rows with dF/dz != 0
    double* ul = reinterpret_cast<double*>(dyn);
    double* bpl = ul + rows_max;
    uint64_t* msk = reinterpret_cast<uint64_t*>(bpl + (rows_max / ROWS) * KS);
    if (LDSRES) {
        // in storage order: per batch, vector c of its ROWS rows, contiguous
        for (int64_t idx = threadIdx.x; idx < nrows * nc; idx += blockDim.x) {
            const int64_t lb = idx / (int64_t(nc) * ROWS);
            const int64_t rem = idx - lb * (int64_t(nc) * ROWS);
            const int cc = int(rem / ROWS);
            const int64_t lr = rem - int64_t(cc) * ROWS;
            dkl[(lb * ROWS + lr) * ncp + cc] =
                reinterpret_cast<const V*>(dk)[dk_vec_index<DT>(batch_base(lb) + lr, cc)];
        }
    }
    if (VEC_LDS) {
        for (int64_t rr = threadIdx.x; rr < nrows; rr += blockDim.x) {
            const int64_t row = batch_base(rr / ROWS) + rr % ROWS;
            dl[rr] = A.d[row];
            ql[rr] = T(0);
            cll[rr] = A.cls[row];
        }
        __syncthreads();
    }
    // per-voxel vectors by (global row, local row)
    auto d_at = [&](int64_t row, int64_t lrow) -> double& { return VEC_LDS ? dl[lrow] : A.d[row]; };
    auto q_at = [&](int64_t row, int64_t lrow) -> T& { return VEC_LDS ? ql[lrow] : A.q[row]; };
    auto cls_at = [&](int64_t row, int64_t lrow) -> uint8_t { return VEC_LDS ? cll[lrow] : A.cls[row]; };
    bool alive = true;
    int mode = s_ms.refresh;   // first update keeps d (2) unless told otherwise
    // work counters of workgroup 0 (update, q and line-search passes), kept in
    // LDS and added to the device counters once at the end
    __shared__ double cnt_bytes[3];
    __shared__ uint64_t cnt_real[3];
    if (threadIdx.x < 3) {
        cnt_bytes[threadIdx.x] = 0.0;
        cnt_real[threadIdx.x] = 0;
    }
    // every thread takes the same line-search decisions and step counts from
    // the same totals, in registers; thread 0 mirrors them into s_ms
    LsRegs ls{0.0, 0.0, 0.0, 0.0, 0, 0, s_ms.total_ls};
    int steps = s_ms.steps;
    const int refresh_every = s_ms.refresh_every;
    // phase timing (workgroup 0, thread 0): 0 update pass, 1 its reduction,
    // 2 direction, 3 first line-search pass (q), 4 line-search reductions,
    // 5 final decision + step, 6 later line-search passes (with the decision
    // that asked for them)
    __shared__ uint64_t s_tk[PROF_PHASES], s_t0;
    const bool timer = A.timing && gb == 0 && threadIdx.x == 0;
    if (timer) {
        for (int i = 0; i < PROF_PHASES; ++i) s_tk[i] = 0;
        s_t0 = wall_clock64();
    }
    auto tick = [&](int ph) {
        if (timer) {
            const uint64_t now = wall_clock64();
            s_tk[ph] += now - s_t0;
            s_t0 = now;
        }
    };

    while (alive) {
        // ---------------- update pass: apply the step, dF/dz, grad_y partials
        // (the objective is summed once, at the final point of the solve)
        {
            if constexpr (LDSRES) {
                // D_K on chip: each wavefront sums grad_y over its batches
                // (lb = wave, wave + NW, ...) in registers
                const double t = ls.t;
                double yv[G::EPL], acc[G::EPL];
#pragma unroll
                for (int e = 0; e < G::EPL; ++e) {
                    const int k = c * G::EPL + e;
                    yv[e] = (mode == 1 && k < K) ? s_y[k] * dks : 0.0;
                    acc[e] = 0.0;
                }
                double* su = s_u[wave];
                // the batch's D_K rows, from LDS (COOP_CHIP) or device memory
                auto load_rows = [&](int64_t base, int64_t lbase, V (&v)[IT]) {
                    if (LDSRES) {
                        // running LDS offset, opaque to the compiler so it adds one
                        // stride per load instead of keeping IT addresses live
                        uint32_t off = uint32_t(((lbase + rg) * ncp + c) * 16);
                        const uint32_t stride = uint32_t(G::RPW * ncp * 16);
                        // one predicated region for all the loads (see load_batch)
                        if (c < nc) {
#pragma unroll
                            for (int it = 0; it < IT; ++it) {
                                asm volatile("" : "+v"(off));
                                v[it] = *reinterpret_cast<const V*>(dyn + off);
                                off += stride;
                            }
                        } else {
#pragma unroll
                            for (int it = 0; it < IT; ++it) v[it] = vzero<V>();
                        }
                    } else {
                        load_batch<DT>(dk, base, rg, c, nc, v);
                    }
                };
                for (int64_t lb = wave; lb < nlb; lb += NW) {
                    const int64_t base = batch_base(lb), lbase = lb * ROWS;
                    if (VEC_LDS && mode != 1) {
                        // the per-voxel stage first (d, q and the class are in
                        // LDS).  A row inside its dose window has dF/dz = 0 and
                        // adds exact zeros to grad_y (the partial sums start at +0
                        // and never become -0), so a batch with no other row
                        // leaves them bit for bit as they are and its D_K rows
                        // are not read.
                        double u = 0.0;
                        if (lane < ROWS) {
                            const int64_t lrow = lbase + lane;
                            double dn = dl[lrow];
                            if (mode == 0) dn = dn + t * double(ql[lrow]);
                            const ObjClass cc = cl[cll[lrow]];
                            if (mode != 2) dl[lrow] = dn;
                            u = grad_f(cc, dn);
                            su[lane] = u;
                        }
                        if (__any(u != 0.0)) {
                            V v[IT];
                            load_rows(base, lbase, v);
                            wave_sync();
#pragma unroll
                            for (int it = 0; it < IT; ++it) {
                                const double uu = su[it * G::RPW + rg];
#pragma unroll
                                for (int e = 0; e < G::EPL; ++e) acc[e] += uu * vget(v[it], e);
                            }
                        }
                        wave_sync();
                        continue;
                    }
                    // this lane's row of the per-voxel stage: its d, q and class
                    // are loaded together with the batch's D_K rows, so the two
                    // memory round trips overlap
                    double d_pre = 0.0, q_pre = 0.0;
                    uint8_t c_pre = 0;
                    if (lane < ROWS) {
                        const int64_t row = base + lane, lrow = lbase + lane;
                        if (mode != 1) d_pre = d_at(row, lrow);
                        if (mode == 0) q_pre = double(q_at(row, lrow));
                        c_pre = cls_at(row, lrow);
                    }
                    V v[IT];
                    load_rows(base, lbase, v);
                    if (mode == 1) {
#pragma unroll
                        for (int it = 0; it < IT; ++it) {
                            double part = 0.0;
#pragma unroll
                            for (int e = 0; e < G::EPL; ++e) part += vget(v[it], e) * yv[e];
                            part = group_sum<G::LPR>(part);
                            if (c == 0) su[it * G::RPW + rg] = part;
                        }
                    }
                    wave_sync();
                    if (lane < ROWS) {
                        const int64_t row = base + lane;
                        double dn;
                        if (mode == 1) {
                            dn = su[lane] - tau_at(A.tau, row);   // the master keeps d - tau
                        } else {
                            dn = d_pre;
                            if (mode == 0) dn = dn + t * q_pre;
                        }
                        const ObjClass cc = cl[c_pre];
                        if (mode != 2) d_at(row, lbase + lane) = dn;
                        su[lane] = grad_f(cc, dn);
                    }
                    wave_sync();
#pragma unroll
                    for (int it = 0; it < IT; ++it) {
                        const double u = su[it * G::RPW + rg];
#pragma unroll
                        for (int e = 0; e < G::EPL; ++e) acc[e] += u * vget(v[it], e);
                    }
                    wave_sync();
                }
#pragma unroll
                for (int off = G::LPR; off < WAVE; off <<= 1)
#pragma unroll
                    for (int e = 0; e < G::EPL; ++e) acc[e] += __shfl_xor(acc[e], off, WAVE);
                if (rg == 0)
#pragma unroll
                    for (int e = 0; e < G::EPL; ++e) s_acc[wave][c * G::EPL + e] = acc[e] * dks;
                __syncthreads();
                combine_waves8(&s_acc[0][0], RECW, K, false, s_rec);
            } else {
                //
                // grad_y is summed per batch (each lane over the batch's rows in
                // order, then across the lane groups), then over the workgroup's
                // batches in a fixed order, so the sum does not depend on which
                // wavefront handles a batch.  With the rows on chip (and outside
                // refresh steps) every row's new dose and dF/dz come first; a row
                // inside its dose window has dF/dz = +0 exactly and adds exact zeros,
                // so only batches with another row read their D_K rows (the sums
                // start at +0 and never become -0, so skipping a batch leaves the
                // bits as they are), and those batches are dealt to the wavefronts
                // round-robin.
                const double t = ls.t;
                double yv[G::EPL];
#pragma unroll
                for (int e = 0; e < G::EPL; ++e) {
                    const int k = c * G::EPL + e;
                    yv[e] = (mode == 1 && k < K) ? s_y[k] * dks : 0.0;
                }
                double* su = s_u[wave];
                // grad_y partial of one batch from its D_K rows and the rows'
                // dF/dz (u(r): row r of the batch), stored for the combine
                auto batch_partial = [&](int64_t lb, const V (&v)[IT], auto&& u) {
                    double a[G::EPL];
#pragma unroll
                    for (int e = 0; e < G::EPL; ++e) a[e] = 0.0;
#pragma unroll
                    for (int it = 0; it < IT; ++it) {
                        const double uu = u(it * G::RPW + rg);
#pragma unroll
                        for (int e = 0; e < G::EPL; ++e) a[e] += uu * vget(v[it], e);
                    }
#pragma unroll
                    for (int off = G::LPR; off < WAVE; off <<= 1)
#pragma unroll
                        for (int e = 0; e < G::EPL; ++e) a[e] += __shfl_xor(a[e], off, WAVE);
                    if (rg == 0) {
                        if (VEC_LDS) {
#pragma unroll
                            for (int e = 0; e < G::EPL; ++e) bpl[lb * KS + c * G::EPL + e] = a[e];
                        } else {
                            double* bp = A.bpart + (batch_base(lb) / ROWS) * KS + c * G::EPL;
#pragma unroll
                            for (int e = 0; e < G::EPL; ++e) astore(bp + e, a[e]);
                        }
                    }
                };
                if (VEC_LDS && mode != 1) {
                    // rows on chip: new dose and dF/dz of every row, one
                    // row per thread (wavefront w: rows w * 64 + lane, then
                    // every 512 further), and each batch's mask of rows with
                    // dF/dz != 0
                    static_assert(ROWS == WAVE || ROWS == WAVE / 2, "one or two batches per wavefront of rows");
                    for (int64_t r0 = int64_t(wave) * WAVE; r0 < nrows; r0 += int64_t(NW) * WAVE) {
                        const int64_t lrow = r0 + lane;
                        double u = 0.0;
                        if (lrow < nrows) {
                            double dn = dl[lrow];
                            if (mode == 0) dn = dn + t * double(ql[lrow]);
                            const ObjClass cc = cl[cll[lrow]];
                            if (mode != 2) dl[lrow] = dn;
                            u = grad_f(cc, dn);
                            ul[lrow] = u;
                        }
                        const uint64_t m = __ballot(u != 0.0);
                        if (lane == 0) {
                            if (ROWS == WAVE) {
                                msk[r0 / ROWS] = m;
                            } else {
                                msk[r0 / ROWS] = m & 0xFFFFFFFFull;
                                if (r0 + ROWS < nrows) msk[r0 / ROWS + 1] = m >> 32;
                            }
                        }
                    }
                    __syncthreads();
                    // the batches with a row to read, dealt to the wavefronts
                    // in batch order
                    int done = 0;
                    for (int64_t c0 = 0; c0 < nlb; c0 += WAVE) {
                        const bool on = c0 + lane < nlb && msk[c0 + lane] != 0;
                        const uint64_t m = __ballot(on);
                        const int rank = done + __popcll(m & ((uint64_t(1) << lane) - 1));
                        uint64_t mine = __ballot(on && rank % NW == wave);
                        done += __popcll(m);
                        while (mine) {
                            const int64_t lb = c0 + __builtin_ctzll(mine);
                            mine &= mine - 1;
                            V v[IT];
                            // only the groups of RPW rows that hold a row with dF/dz != 0
                            load_batch_rows<DT>(dk, batch_base(lb), rg, c, nc, msk[lb], v);
                            const double* ub = ul + lb * ROWS;
                            batch_partial(lb, v, [&](int r) { return ub[r]; });
                        }
                    }
                } else {
                    // refresh steps (d = D_K y needs every D_K row) and the
                    // streaming form: each batch in one go, d and the class
                    // loaded together with the D_K rows so that the two memory
                    // round trips overlap
                    for (int64_t lb = wave; lb < nlb; lb += NW) {
                        const int64_t base = batch_base(lb), lbase = lb * ROWS;
                        double d_pre = 0.0, q_pre = 0.0;
                        uint8_t c_pre = 0;
                        if (lane < ROWS) {
                            const int64_t row = base + lane, lrow = lbase + lane;
                            if (mode != 1) d_pre = d_at(row, lrow);
                            if (mode == 0) q_pre = double(q_at(row, lrow));
                            c_pre = cls_at(row, lrow);
                        }
                        V v[IT];
                        load_batch<DT>(dk, base, rg, c, nc, v);
                        if (mode == 1) {
#pragma unroll
                            for (int it = 0; it < IT; ++it) {
                                double part = 0.0;
#pragma unroll
                                for (int e = 0; e < G::EPL; ++e) part += vget(v[it], e) * yv[e];
                                part = group_sum<G::LPR>(part);
                                if (c == 0) su[it * G::RPW + rg] = part;
                            }
                        }
                        wave_sync();
                        if (lane < ROWS) {
                            const int64_t row = base + lane;
                            double dn;
                            if (mode == 1) {
                                dn = su[lane] - tau_at(A.tau, row);   // the master keeps d - tau
                            } else {
                                dn = d_pre;
                                if (mode == 0) dn = dn + t * q_pre;
                            }
                            const ObjClass cc = cl[c_pre];
                            if (mode != 2) d_at(row, lbase + lane) = dn;
                            su[lane] = grad_f(cc, dn);
                        }
                        wave_sync();
                        batch_partial(lb, v, [&](int r) { return su[r]; });
                        if (VEC_LDS && lane == 0) msk[lb] = ~uint64_t(0);
                        wave_sync();
                    }
                }
                    if (!VEC_LDS) __threadfence();   // the partials stored in device memory, before the barrier
                // grad_y: thread (k, j) sums the partials of batches j, j + 8,
                // ... (those with a row to read; the others are +0), then the
                // 8 sums of each slot are combined in a fixed order
                __syncthreads();
                {
                    const int k = threadIdx.x / NW, j = threadIdx.x % NW;
                    if (k < K) {
                        double sacc = 0.0;
                        for (int64_t lb = j; lb < nlb; lb += NW) {
                            if (VEC_LDS) {
                                const double x = bpl[lb * KS + k];
                                sacc += msk[lb] != 0 ? x : 0.0;
                            } else {
                                sacc += aload(A.bpart + (batch_base(lb) / ROWS) * KS + k);
                            }
                        }
                        s_acc[j][k] = sacc * dks;
                    }
                }
                __syncthreads();
                combine_waves8(&s_acc[0][0], RECW, K, false, s_rec);
            }
            if (gb == 0 && threadIdx.x == 0) {
                const double per_row = 16.0 * nc + 1.0 + (mode != 1 ? 8.0 : 0.0) +
                                       (mode == 0 ? double(sizeof(T)) : 0.0) + (mode != 2 ? 8.0 : 0.0);
                cnt_bytes[0] += per_row * double(A.Vnz);
                cnt_real[0] += 1;
            }
            tick(0);
            if (!grid_reduce<false>(A.sync, A.recs, s_rec, K, s_tot, seq, gb, gn)) {
                alive = false;
                break;
            }
            tick(1);
        }
        // ---------------- direction (identical in every workgroup)
        if (threadIdx.x < WAVE) {
            const int k = threadIdx.x;
            const bool in = k < K;
            const double yk = s_y[k];
            const double gk = in ? s_tot[k] : 0.0;
            double rk;
            bool fk;
            const double pk = cg_dir_wave(in, yk, gk, s_ms.conj && s_ms.cg_valid, s_p[k], s_r[k], s_fr[k] != 0,
                                          rk, fk);
            const double kkt = wave_reduce_dpp<2>(in ? fabs(fmin(yk, gk)) : 0.0);
            const double tmax = wave_reduce_dpp<1>(pk < 0.0 ? yk / (-pk) : INFINITY);
            const double gp = wave_reduce_dpp<0>(gk * pk);
            const bool any = __any(rk != 0.0);
            // the direction and its memory change only when a step is taken
            if (kkt > s_ms.tol && steps < s_ms.max_steps && any) {
                s_p[k] = pk;
                s_r[k] = rk;
                s_fr[k] = fk;
            }
            s_g[k] = gk;
            if (k == 0) {
                s_ms.kkt = kkt;
                int go = 1;
                if (!(kkt > s_ms.tol)) {
                    s_ms.stop_reason = 1;
                    go = 0;
                } else if (steps >= s_ms.max_steps) {
                    s_ms.stop_reason = 2;
                    go = 0;
                } else if (!any) {
                    s_ms.stop_reason = 3;
                    go = 0;
                }
                if (!go) {
                    s_ms.done = 1;
                } else {
                    s_ms.t_max = tmax;
                    s_ms.gphi0 = gp;
                    s_ms.t = ls_first_trial(s_ms.prev_step, tmax);
                    s_ms.lo = 0.0;
                    s_ms.hi = tmax;
                    s_ms.hi_known = 0;
                    s_ms.ls_iter = 0;
                }
                s_go = go;
            }
        }
        __syncthreads();
        tick(2);
        if (!s_go) break;
        ls.t_max = s_ms.t_max;
        ls.t = ls_first_trial(s_ms.prev_step, ls.t_max);
        ls.lo = 0.0;
        ls.hi = ls.t_max;
        ls.hi_known = 0;
        ls.ls_iter = 0;
        // ---------------- line search: first evaluation computes q = D_K p
        bool first = true;
        for (;;) {
            const double t = ls.t;
            Rec r = rec_identity();
            double pv[G::EPL];
#pragma unroll
            for (int e = 0; e < G::EPL; ++e) pv[e] = s_p[c * G::EPL + e] * dks;
            if (LDSRES) {
                // one row per thread, straight from LDS; q's per-slot partials
                // are combined in the order of the lane butterfly of the
                // streaming form below, so q is the same up to the sign of an
                // exact zero
                for (int64_t rr = threadIdx.x; rr < nrows; rr += blockDim.x) {
                    const ObjClass cc = cl[cll[rr]];
                    const double dv = dl[rr];
                    T qt;
                    if (first) {
                        const V* rp = dkl + rr * ncp;
                        // partial of slot vector j (slots past the pool add exact zeros)
                        auto part_of = [&](int j) {
                            double part = 0.0;
                            if (j < nc) {
                                const V v = rp[j];
#pragma unroll
                                for (int e = 0; e < G::EPL; ++e) part += vget(v, e) * (s_p[j * G::EPL + e] * dks);
                            }
                            return part;
                        };
                        // first butterfly level pairs j with j + LPR/2; only the
                        // LPR/2 pair sums stay live
                        constexpr int H = G::LPR / 2;
                        double pc[H];
#pragma unroll
                        for (int j = 0; j < H; ++j) pc[j] = part_of(j) + part_of(j + H);
#pragma unroll
                        for (int off = H / 2; off > 0; off >>= 1)
#pragma unroll
                            for (int j = 0; j < off; ++j) pc[j] = pc[j] + pc[j + off];
                        qt = T(pc[0]);   // the line search and the update use the stored value
                        ql[rr] = qt;
                        double bu, bo;
                        ls_breakpoints(cc, dv, double(qt), bu, bo);
                        bul[rr] = bu;
                        bol[rr] = bo;
                    } else {
                        qt = ql[rr];
                    }
                    ls_voxel_bp(cc, dv, double(qt), bul[rr], bol[rr], t, r);
                }
            } else {
                for (int64_t lb = wave; lb < nlb; lb += NW) {
                    const int64_t base = batch_base(lb), lbase = lb * ROWS;
                    // this lane's row: d and class loaded with the D_K rows
                    double d_pre = 0.0;
                    uint8_t c_pre = 0;
                    T q_pre = T(0);
                    if (lane < ROWS) {
                        d_pre = d_at(base + lane, lbase + lane);
                        c_pre = cls_at(base + lane, lbase + lane);
                        if (!first) q_pre = q_at(base + lane, lbase + lane);
                    }
                    double qsum = 0.0;
                    if (first) {
                        V v[IT];
                        load_batch<DT>(dk, base, rg, c, nc, v);
                        // each lane's per-slot partials go to LDS, then every
                        // row is summed by its own lane in the order of the lane
                        // butterfly (row_tree): the q of the on-chip form
                        constexpr int TPS = G::LPR + 1;
                        double* tp = reinterpret_cast<double*>(dyn) + size_t(wave) * ROWS * TPS;
#pragma unroll
                        for (int it = 0; it < IT; ++it) {
                            double part = 0.0;
#pragma unroll
                            for (int e = 0; e < G::EPL; ++e) part += vget(v[it], e) * pv[e];
                            tp[(it * G::RPW + rg) * TPS + c] = part;
                        }
                        wave_sync();
                        if (lane < ROWS) qsum = row_tree<G::LPR>(tp + lane * TPS);
                    }
                    if (lane < ROWS) {
                        const int64_t row = base + lane;
                        T qt;
                        if (first) {
                            qt = T(qsum);   // the line search and the update use the stored value
                            q_at(row, lbase + lane) = qt;
                        } else {
                            qt = q_pre;
                        }
                        ls_voxel(cl[c_pre], d_pre, double(qt), t, r);
                    }
                    wave_sync();
                }
            }
            block_rec_dpp(r, s_rec);
            if (gb == 0 && threadIdx.x == 0) {
                const int kk = first ? 1 : 2;
                cnt_bytes[kk] += (first ? (16.0 * nc + 8.0 + 1.0 + double(sizeof(T)))
                                          : (8.0 + double(sizeof(T)) + 1.0)) * double(A.Vnz);
                cnt_real[kk] += 1;
            }
            tick(first ? 3 : 6);
            if (!grid_reduce<true>(A.sync, A.recs, s_rec, 6, s_tot, seq, gb, gn)) {
                alive = false;
                break;
            }
            tick(4);
            const Rec tot{s_tot[0], s_tot[1], s_tot[2], s_tot[3], s_tot[4], s_tot[5]};
            const int fin = ls_decide(ls, tot);
            first = false;
            if (fin) break;
        }
        if (!alive) break;
        // ---------------- step: y update, counters, next update mode
        {
            const double t = ls.t, tmax = ls.t_max;
            if (threadIdx.x < K) {
                const int k = threadIdx.x;
                const double pk = s_p[k];
                double yn = s_y[k] + t * pk;
                if (t == tmax) {   // an aperture that blocks the step ends at exactly 0
                    const double ratio = pk < 0.0 ? s_y[k] / (-pk) : INFINITY;
                    if (ratio == t) yn = 0.0;
                }
                s_y[k] = fmax(yn, 0.0);
            }
            steps += 1;
            mode = (steps % refresh_every) == 0 ? 1 : 0;
            if (threadIdx.x == 0) {
                // a step that blocks ends the conjugate sequence
                s_ms.cg_valid = s_ms.conj && !(t == tmax);
                s_ms.cg_K = K;
                s_ms.steps = steps;
                s_ms.total_steps += 1;
                s_ms.prev_step = s_ms.last_step;
                s_ms.last_step = t;
                s_ms.refresh = mode;
                s_ms.t = t;
                s_ms.t_max = tmax;
                s_ms.lo = ls.lo;
                s_ms.hi = ls.hi;
                s_ms.hi_known = ls.hi_known;
                s_ms.ls_iter = ls.ls_iter;
                s_ms.total_ls = ls.total_ls;
            }
            // y must be visible before a refresh update pass reads it; every
            // other reader of y and of s_ms comes after the update pass's
            // own barriers
            if (mode == 1) __syncthreads();
            tick(5);
        }
    }
    // the objective at the final point: one row per thread (the same split
    // and order in every form), a fixed-order workgroup sum, one grid
    // reduction
    if (alive) {
        double Fp = 0.0;
        for (int64_t lrow = threadIdx.x; lrow < nrows; lrow += blockDim.x) {
            const int64_t row = batch_base(lrow / ROWS) + lrow % ROWS;
            Fp += obj_f(cl[cls_at(row, lrow)], d_at(row, lrow));
        }
        Fp = wave_reduce_dpp<0>(Fp);
        if (lane == 0) s_acc[wave][0] = Fp;
        __syncthreads();
        combine_waves8(&s_acc[0][0], RECW, 1, false, s_rec);
        if (grid_reduce<false>(A.sync, A.recs, s_rec, 1, s_tot, seq, gb, gn)) {
            if (threadIdx.x == 0) s_ms.F = s_ms.F_const + s_tot[0];
        } else {
            alive = false;
        }
    }
    if (VEC_LDS) {
        __syncthreads();
        for (int64_t rr = threadIdx.x; rr < nrows; rr += blockDim.x) A.d[batch_base(rr / ROWS) + rr % ROWS] = dl[rr];
    }
    if (timer)
        for (int i = 0; i < PROF_PHASES; ++i) A.pc->ticks[i] += s_tk[i];
    if (gb == 0 && threadIdx.x == 0)
        for (int i = 0; i < 3; ++i) {
            A.pc->bytes[i] += cnt_bytes[i];
            A.pc->real[i] += cnt_real[i];
        }
    // workgroup 0 publishes the final state
    if (gb == 0) {
        if (threadIdx.x < K) {
            A.y[threadIdx.x] = s_y[threadIdx.x];
            A.p[threadIdx.x] = s_p[threadIdx.x];
            A.grad[threadIdx.x] = s_g[threadIdx.x];
            A.cgm->r[threadIdx.x] = s_r[threadIdx.x];
            A.cgm->free[threadIdx.x] = s_fr[threadIdx.x];
        }
        if (threadIdx.x == 0 && !alive) s_ms.stop_reason = 4;
        ms_store(A.ms, s_ms);
    }
}

// One master solve per launch: every workgroup of the grid works on it.
template <class T, class DT, int FORM>
__global__ void __launch_bounds__(COOP_THREADS) k_master_coop(CoopArgs<T> A) {
    master_body<T, DT, FORM>(A, blockIdx.x, gridDim.x);
}

// Several master solves in one cooperative launch: solve i gets workgroups
// [gstart[i], gstart[i + 1]) and runs exactly as k_master_coop would on a grid
// of that size; solves never wait for each other, and the launch ends when
// the last one has converged.
template <class T, class DT, int FORM>
__global__ void __launch_bounds__(COOP_THREADS) k_master_batch(const CoopArgs<T>* __restrict__ args,
                                                               const int32_t* __restrict__ gstart, int nsolves) {
    __shared__ int s_i;
    if (threadIdx.x == 0) {
        int i = 0;
        while (i + 1 < nsolves && int(blockIdx.x) >= gstart[i + 1]) ++i;
        s_i = i;
    }
    __syncthreads();
    const int i = s_i;
    const uint32_t g0 = uint32_t(gstart[i]), g1 = uint32_t(gstart[i + 1]);
    if (blockIdx.x >= g1) return;   // workgroups past the last solve (none when the host fills the grid)
    const CoopArgs<T> A = args[i];
    master_body<T, DT, FORM>(A, blockIdx.x - g0, g1 - g0);
}

}  // namespace dao
