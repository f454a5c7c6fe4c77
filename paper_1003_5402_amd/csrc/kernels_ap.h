// Master over the aperture dose matrix (gfx950).
//
// Section 2.1, eq. 1 and eq. 2 give the voxel dose of the pool as
// z = D_K y with D_kj = sum_{i in A_k} D_ij.  Here D_K is kept on the device
// as a dense block of KS = 64 aperture slots per voxel row (internal row
// order), stored by batch: see dk_vec_index.  A round appends one column (one forward
// product of D with the aperture's 0/1 beamlet indicator); nothing is ever
// rebuilt or transposed.  Both master products then stream D_K row by row:
//   q = D_K p              (direction of the dose, k_qstep_ap)
//   grad_y = D_K^T dF/dz    (gradient over the pool, fused into k_upd_ap)
// LPR lanes each load one 16-byte vector of a row, so one wavefront
// instruction reads slot vector c of RPW consecutive rows (RPW runs of
// 16 B per c, contiguous across the batch's instructions).
//
// Step sequence: k_upd_ap -> k_dir_ap -> k_qstep_ap -> k_lseval x slots.
//   k_upd_ap   (PH_UPD) applies the last step to d (mode 0: d += t q,
//              mode 1: d = D_K y, mode 2: keep d), computes dF/dz, the
//              objective partials and the partials of grad_y per workgroup.
//   k_dir_ap   (PH_UPD) sums the partials in a fixed order, tests KKT and
//              builds the projected direction (-> PH_Q).
//   k_qstep_ap (PH_Q)   q = D_K p and the first line-search evaluation.
//   k_lseval   (PH_LS)  further evaluations (shared with the beamlet master).
#pragma once

#include "kernels.h"

namespace dao {

template <class T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int n = 4;
};
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int n = 2;
};
// FP16 storage of D_K (values over one global scale): 8 slots per vector
struct alignas(16) half8 {
    __half2 h[4];
};
template <>
struct Vec16<__half> {
    using type = half8;
    static constexpr int n = 8;
};

template <class T>
struct DKG {
    static constexpr int EPL = Vec16<T>::n;   // aperture slots per lane
    static constexpr int LPR = KS / EPL;      // lanes per row
    static constexpr int RPW = WAVE / LPR;    // rows per wavefront instruction
    static constexpr int VPR = KS / EPL;      // 16-byte slot vectors per row
};

// Rows are processed in batches of BATCH = ITERS * RPW consecutive rows per
// wavefront.  Each lane first issues all ITERS of its 16-byte D_K loads for
// the batch (lane group rg holds rows rg, rg + RPW, ...; lane c of the group
// holds aperture slots c*EPL .. c*EPL+EPL-1), then the batch is handled one
// row per lane for the per-voxel work (coalesced d, q and class access, all
// lanes active), with row results exchanged through LDS.
// The per-voxel stage of a batch gives each lane one row, so a batch holds at
// most WAVE rows: 16 loads per lane for FP32 and FP64 storage (64 and 32
// rows), 8 for FP16 storage (8 rows per instruction, 64 rows).
template <class T>
struct Batch {
    static constexpr int ITERS = 16 * DKG<T>::RPW > WAVE ? WAVE / DKG<T>::RPW : 16;
    static constexpr int ROWS = ITERS * DKG<T>::RPW;
    static_assert(ROWS <= WAVE, "one row per lane in the per-voxel stage");
};

// Layout of D_K in device memory: the rows in blocks of one batch; inside a
// block, slot vector c of every row of the block is stored contiguously.
// Vector (row, c) is element ((row / ROWS) * VPR + c) * ROWS + row % ROWS of
// the 16-byte vectors.  A pass that needs the first nc vectors of each row
// (the pool's K slots) then reads nc contiguous runs of ROWS * 16 bytes per
// batch and nothing else, whatever K is; with whole rows of KS slots the
// tail of the row's last cache line would be fetched too.
template <class DT>
__host__ __device__ __forceinline__ int64_t dk_vec_index(int64_t row, int c) {
    constexpr int ROWS = Batch<DT>::ROWS;
    const int64_t blk = row / ROWS;
    return (blk * DKG<DT>::VPR + c) * ROWS + (row - blk * ROWS);
}
// element index of aperture slot k of a row
template <class DT>
__host__ __device__ __forceinline__ int64_t dk_index(int64_t row, int k) {
    return dk_vec_index<DT>(row, k / DKG<DT>::EPL) * DKG<DT>::EPL + k % DKG<DT>::EPL;
}

__device__ __forceinline__ double vget(const float4& v, int e) {
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}
__device__ __forceinline__ double vget(const double2& v, int e) { return e == 0 ? v.x : v.y; }
__device__ __forceinline__ double vget(const half8& v, int e) {
    const __half2 p = v.h[e >> 1];
    return double((e & 1) ? __high2float(p) : __low2float(p));
}

template <class V>
__device__ __forceinline__ V vzero();
template <>
__device__ __forceinline__ float4 vzero<float4>() {
    return make_float4(0.f, 0.f, 0.f, 0.f);
}
template <>
__device__ __forceinline__ double2 vzero<double2>() {
    return make_double2(0.0, 0.0);
}
template <>
__device__ __forceinline__ half8 vzero<half8>() {
    half8 z;
#pragma unroll
    for (int i = 0; i < 4; ++i) z.h[i] = __float2half2_rn(0.0f);
    return z;
}

// This lane's D_K vectors of the batch that starts at row `base` (a
// multiple of the batch size, so the batch is one storage block): vector c
// of rows base + it * RPW + rg, zero where c >= nc.  All IT loads sit in one
// predicated region, so all are issued before the first is waited for (a
// branch per load lets the compiler wait on each load in turn).
template <class DT, int IT, class V>
__device__ __forceinline__ void load_batch(const DT* dk, int64_t base, int rg, int c, int nc, V (&v)[IT]) {
    static_assert(IT * DKG<DT>::RPW == Batch<DT>::ROWS, "one batch per block");
    if (c < nc) {
        const V* p = reinterpret_cast<const V*>(dk) + dk_vec_index<DT>(base + rg, c);
#pragma unroll
        for (int it = 0; it < IT; ++it) v[it] = p[it * DKG<DT>::RPW];
    } else {
#pragma unroll
        for (int it = 0; it < IT; ++it) v[it] = vzero<V>();
    }
}

// load_batch restricted to some rows: `rows` has bit r set for each row
// base + r that is needed; a load whose RPW rows are all unneeded reads
// nothing and gives zeros.  The loads are buffer loads through a descriptor
// of the batch's storage block, and an unneeded one gets an offset past the
// block's end (out of range: no memory access, zero data), so all of them
// still issue back to back with no branch.
template <class DT, int IT, class V>
__device__ __forceinline__ void load_batch_rows(const DT* dk, int64_t base, int rg, int c, int nc, uint64_t rows,
                                                V (&v)[IT]) {
    static_assert(IT * DKG<DT>::RPW == Batch<DT>::ROWS, "one batch per block");
    static_assert(sizeof(V) == 16, "16-byte vectors");
    constexpr int ROWS = Batch<DT>::ROWS, RPW = DKG<DT>::RPW;
    constexpr uint32_t BLOCK_BYTES = uint32_t(DKG<DT>::VPR) * ROWS * 16;
    const unsigned char* blk = reinterpret_cast<const unsigned char*>(dk) +
                               size_t(base / ROWS) * BLOCK_BYTES;   // base: a multiple of ROWS
    // word 3 of a GFX9 buffer descriptor: 32-bit data format, no swizzle
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char*>(blk), short(0), int(BLOCK_BYTES), 0x00020000);
    // out of range: at or past 2^31, also after adding a row offset (< 2^11)
    constexpr uint32_t OUT = 0x80000000u;
    const uint32_t lane_off = c < nc ? uint32_t((c * ROWS + rg) * 16) : OUT;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        // the same for every lane: a scalar select, no branch
        const bool grp = ((rows >> (it * RPW)) & ((uint64_t(1) << RPW) - 1)) != 0;
        const uint32_t off = grp ? lane_off + uint32_t(it * RPW * 16) : OUT;
        v[it] = __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(rsrc, int(off), 0, 0));
    }
}

// Order LDS traffic between lanes of one wavefront (used inside loops whose
// trip count differs between the wavefronts of a workgroup, where a
// workgroup barrier would be wrong).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// v of the lane OFF places further along its row of 16 lanes, cyclically:
// lane c gets lane (c + OFF) mod 16.  DPP row_ror:N moves data N lanes up
// the row (lane c receives lane c - N mod 16), so the move is row_ror by
// 16 - OFF (a VALU move; every lane of the wavefront must be active).
template <int OFF>
__device__ __forceinline__ double dpp_row_from(double v) {
    static_assert(OFF >= 1 && OFF <= 15, "offsets 1..15 inside a row");
    constexpr int CTRL = 0x120 + (16 - OFF);   // row_ror:(16 - OFF)
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
template <int OFF>
__device__ __forceinline__ double ror_tree(double v) {
    if constexpr (OFF == 0)
        return v;
    else
        return ror_tree<OFF / 2>(v + dpp_row_from<OFF>(v));
}

// Sum over the LPR lanes of one row (aligned lane groups); lane 0 of the
// group gets the sum, as the butterfly adds it: lane c with lane c + LPR/2
// first, then halves.  Groups inside one row of 16 lanes take their
// operands by DPP rotations of the row (for c below the offset, lane
// (c + off) mod 16 is lane c + off of the same group, so lane 0 adds
// exactly the butterfly's operands); wider groups go through lane permutes.
// Call with every lane of the wavefront active.
template <int LPR>
__device__ __forceinline__ double group_sum(double v) {
    if constexpr (LPR <= 16) {
        return ror_tree<LPR / 2>(v);
    } else {
#pragma unroll
        for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
        return v;
    }
}

// The same sum for one row whose LPR per-slot partials sit in memory (x[c]
// the partial of lane c): the butterfly's pairs, in the butterfly's order.
template <int LPR>
__device__ __forceinline__ double row_tree(const double* x) {
    constexpr int H = LPR / 2;
    double pc[H];
#pragma unroll
    for (int j = 0; j < H; ++j) pc[j] = x[j] + x[j + H];
#pragma unroll
    for (int off = H / 2; off > 0; off >>= 1)
#pragma unroll
        for (int j = 0; j < off; ++j) pc[j] = pc[j] + pc[j + off];
    return pc[0];
}

// ind[i] = 1 if beamlet i is open in pool aperture k, else 0.
template <class T>
__global__ void k_ap_indicator(PoolView P, int k, T* __restrict__ ind) {
    const int b = P.ap_beam[k];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P.N; i += gridDim.x * blockDim.x) {
        T v = T(0);
        if (P.blt_beam[i] == b) {
            const int lr = P.blt_row[i] - P.beam_row0[b];
            const int16_t* l = P.ap_lv + (size_t(k) * P.maxRB + lr) * 2;
            const int pos = P.blt_pos[i];
            if (pos >= l[0] && pos < l[1]) v = T(1);
        }
        ind[i] = v;
    }
}

// Column k of D_K: slot k of every row = (D ind)_row, FP64 sums rounded to
// the storage type DT (T, or FP16 of the sum times inv_scale).
__device__ __forceinline__ void dk_store(float* p, double v, double) { *p = float(v); }
__device__ __forceinline__ void dk_store(double* p, double v, double) { *p = v; }
__device__ __forceinline__ void dk_store(__half* p, double v, double inv) { *p = __float2half_rn(float(v * inv)); }

template <class T, class VT = T, bool LO = false, class DT = T>
__global__ void __launch_bounds__(SLAB_THREADS) k_dk_column(SellView<VT> S, int64_t Vpad,
                                                            const T* __restrict__ ind, int N, bool stage,
                                                            const float* __restrict__ scale, int k,
                                                            DT* __restrict__ dk, double inv_dk_scale) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double s_part[KSPLIT * SLAB];
    const double sum = slab_rows_x<VT, T, double, LO>(S, ind, N, reinterpret_cast<T*>(smem), stage, scale, s_part);
    const int64_t row = int64_t(blockIdx.x) * SLAB + threadIdx.x;
    if (threadIdx.x < SLAB && row < Vpad) dk_store(dk + dk_index<DT>(row, k), sum, inv_dk_scale);
}


// Update pass (PH_UPD).  Record of workgroup b in parts2[b * (KS + 1)]:
// [objective partial, grad_y partial for apertures 0..KS-1].
// DT: D_K storage (T, or FP16 of D_K / dk_scale); the products multiply back
// by dk_scale (exactly 1 for T storage).
template <class T, class DT = T>
__global__ void __launch_bounds__(BLOCK) k_upd_ap(const DT* __restrict__ dk, double dk_scale, int64_t Vpad,
                                                  double* __restrict__ d, const T* __restrict__ q,
                                                  const uint8_t* __restrict__ cls,
                                                  const ObjClass* __restrict__ classes, int ncls,
                                                  const double* __restrict__ y, double* __restrict__ parts2,
                                                  const MasterState* ms, ProfCounters* pc, int64_t Vnz,
                                                  const double* __restrict__ tau) {
    using G = DKG<DT>;
    using V = typename Vec16<DT>::type;
    constexpr int IT = Batch<DT>::ITERS, ROWS = Batch<DT>::ROWS;
    constexpr int NW = BLOCK / WAVE;
    __shared__ int s_skip, s_mode, s_K;
    __shared__ double s_t;
    __shared__ ObjClass cl[256];
    __shared__ double s_acc[NW][KS];
    __shared__ double s_F[NW];
    __shared__ double s_u[NW][ROWS];
    if (threadIdx.x == 0) {
        s_skip = (ms->done || ms->phase != PH_UPD);
        s_mode = ms->refresh;
        s_K = ms->K;
        s_t = ms->t;
    }
    __syncthreads();
    if (s_skip) return;
    for (int i = threadIdx.x; i < ncls; i += blockDim.x) cl[i] = classes[i];
    __syncthreads();
    const int mode = s_mode, K = s_K;
    const double t = s_t;
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int rg = lane / G::LPR, c = lane % G::LPR;
    const int nc = (K + G::EPL - 1) / G::EPL;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // D_K prefix + class + d read (unless recomputed) + q read (mode 0) + d write (modes 0, 1)
        const double per_row = 16.0 * nc + 1.0 + (mode != 1 ? 8.0 : 0.0) + (mode == 0 ? double(sizeof(T)) : 0.0) +
                               (mode != 2 ? 8.0 : 0.0);
        pc->bytes[0] += per_row * double(Vnz) + double(gridDim.x) * (KS + 1) * 8.0;
        pc->real[0] += 1;
    }
    double yv[G::EPL];
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
        const int k = c * G::EPL + e;
        yv[e] = (mode == 1 && k < K) ? y[k] * dk_scale : 0.0;
    }
    double acc[G::EPL];
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) acc[e] = 0.0;
    double Fp = 0.0;
    double* su = s_u[wave];
    const int64_t nw = int64_t(gridDim.x) * NW;
    for (int64_t base = (int64_t(blockIdx.x) * NW + wave) * ROWS; base < Vpad; base += nw * ROWS) {
        // 1. all D_K loads of the batch
        V v[IT];
        load_batch<DT>(dk, base, rg, c, nc, v);
        // 2. refresh: d = D_K y for the batch's rows
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
        // 3. one row per lane: new dose, dF/dz, objective
        if (lane < ROWS) {
            const int64_t row = base + lane;
            double dn;
            if (mode == 1) {
                dn = su[lane] - tau_at(tau, row);   // the master keeps d - tau
            } else {
                dn = d[row];
                if (mode == 0) dn = dn + t * double(q[row]);
            }
            const ObjClass cc = cl[cls[row]];
            if (mode != 2) d[row] = dn;
            Fp += obj_f(cc, dn);
            su[lane] = grad_f(cc, dn);
        }
        wave_sync();
        // 4. grad_y partials: u_row * D_K[row][k]
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const double u = su[it * G::RPW + rg];
#pragma unroll
            for (int e = 0; e < G::EPL; ++e) acc[e] += u * vget(v[it], e);
        }
        wave_sync();   // su is rewritten by the next batch
    }
    // lanes holding the same aperture slots: combine the wave's row groups
#pragma unroll
    for (int off = G::LPR; off < WAVE; off <<= 1)
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) acc[e] += __shfl_xor(acc[e], off, WAVE);
    if (rg == 0)
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) s_acc[wave][c * G::EPL + e] = acc[e] * dk_scale;
    Fp = wave_sum(Fp);
    if (lane == 0) s_F[wave] = Fp;
    __syncthreads();
    double* rec = parts2 + size_t(blockIdx.x) * (KS + 1);
    if (threadIdx.x < KS) {
        double sacc = 0.0;
        for (int w = 0; w < NW; ++w) sacc += s_acc[w][threadIdx.x];
        rec[1 + threadIdx.x] = sacc;
    } else if (threadIdx.x == KS) {
        double sacc = 0.0;
        for (int w = 0; w < NW; ++w) sacc += s_F[w];
        rec[0] = sacc;
    }
}

// Direction step (single block, 1024 threads, PH_UPD): F and grad_y from
// the update's partials (fixed order), KKT test, projected direction,
// longest feasible step.  One wavefront handles the (at most 64) apertures.
__global__ void __launch_bounds__(1024) k_dir_ap(const double* __restrict__ parts2, int nblk,
                                                 const double* __restrict__ y, double* __restrict__ p,
                                                 double* __restrict__ grad, MasterState* ms,
                                                 CgMem* __restrict__ cgm, ProfCounters* pc) {
    constexpr int SPLIT = 16;   // threads per record column
    __shared__ MasterState s_ms;
    __shared__ int s_skip;
    __shared__ double s_part[KS + 1][SPLIT];
    __shared__ double s_red[KS + 1];
    ms_load(s_ms, ms);
    if (threadIdx.x == 0) s_skip = s_ms.done || s_ms.phase != PH_UPD;
    __syncthreads();
    if (s_skip) return;
    const int K = s_ms.K;
    if (threadIdx.x == 0) {
        pc->bytes[3] += double(nblk) * (K + 1) * 8.0;
        pc->real[3] += 1;
    }
    // column j of the records (0: objective, 1 + k: aperture k), summed over
    // workgroups: SPLIT contiguous runs, then the runs in order
    for (int idx = threadIdx.x; idx < (K + 1) * SPLIT; idx += blockDim.x) {
        const int j = idx / SPLIT, part = idx % SPLIT;
        const int per = (nblk + SPLIT - 1) / SPLIT;
        const int b0 = part * per, b1 = min(nblk, b0 + per);
        double sacc = 0.0;
        for (int b = b0; b < b1; ++b) sacc += parts2[size_t(b) * (KS + 1) + j];
        s_part[j][part] = sacc;
    }
    __syncthreads();
    if (threadIdx.x <= K) {
        double sacc = 0.0;
        for (int qq = 0; qq < SPLIT; ++qq) sacc += s_part[threadIdx.x][qq];
        s_red[threadIdx.x] = sacc;
    }
    __syncthreads();
    if (threadIdx.x < WAVE) {
        const int k = threadIdx.x;
        const bool in = k < K;
        const double yk = in ? y[k] : 0.0;
        const double gk = in ? s_red[1 + k] : 0.0;
        const bool mem = s_ms.conj && s_ms.cg_valid;
        double rk;
        bool fk;
        const double pk = cg_dir_wave(in, yk, gk, mem, in && mem ? p[k] : 0.0, in && mem ? cgm->r[k] : 0.0,
                                      in && mem && cgm->free[k] != 0, rk, fk);
        const double kkt = wave_reduce_dpp<2>(in ? fabs(fmin(yk, gk)) : 0.0);
        const double tmax = wave_reduce_dpp<1>(pk < 0.0 ? yk / (-pk) : INFINITY);
        const double gp = wave_reduce_dpp<0>(gk * pk);   // as the persistent master sums it
        const bool any = __any(rk != 0.0);
        // the memory and p change only when a step is taken
        const bool take = kkt > s_ms.tol && s_ms.steps < s_ms.max_steps && any;
        if (in) {
            grad[k] = gk;
            if (take) {
                p[k] = pk;
                cgm->r[k] = rk;
                cgm->free[k] = fk;
            }
        }
        if (k == 0) {
            s_ms.F = s_ms.F_const + s_red[0];
            s_ms.kkt = kkt;
            int go = 1;
            if (!(kkt > s_ms.tol)) {
                s_ms.stop_reason = 1;
                go = 0;
            } else if (s_ms.steps >= s_ms.max_steps) {
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
                s_ms.phase = PH_Q;
            }
        }
    }
    ms_store(ms, s_ms);
}

// Final step of a line search in the aperture master (last block, on the
// LDS copy of the state): y update with exact zeros for blocking apertures,
// step count, update mode.
__device__ __forceinline__ void finish_step_ap(MasterState& m, double* y, const double* p, int fin) {
    if (!fin) return;
    const int K = m.K;
    const double t = m.t, tmax = m.t_max;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const double pk = p[k];
        const double ratio = pk < 0.0 ? y[k] / (-pk) : INFINITY;
        double yn = y[k] + t * pk;
        if (t == tmax && ratio == t) yn = 0.0;
        y[k] = fmax(yn, 0.0);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        m.steps += 1;
        m.total_steps += 1;
        m.prev_step = m.last_step;
        m.last_step = t;
        m.refresh = (m.steps % m.refresh_every) == 0 ? 1 : 0;
        // a step that blocks ends the conjugate sequence
        m.cg_valid = m.conj && !(t == tmax);
        m.cg_K = K;
        m.phase = PH_UPD;
    }
}

// q = D_K p and the first line-search evaluation (PH_Q).
template <class T, class DT = T>
__global__ void __launch_bounds__(BLOCK) k_qstep_ap(const DT* __restrict__ dk, double dk_scale, int64_t Vpad,
                                                    const double* __restrict__ d,
                                                    const uint8_t* __restrict__ cls,
                                                    const ObjClass* __restrict__ classes, int ncls,
                                                    T* __restrict__ q, Rec* parts, Arrival* arr,
                                                    MasterState* ms, double* y, const double* p,
                                                    ProfCounters* pc, int64_t Vnz) {
    using G = DKG<DT>;
    using V = typename Vec16<DT>::type;
    constexpr int IT = Batch<DT>::ITERS, ROWS = Batch<DT>::ROWS;
    constexpr int NW = BLOCK / WAVE;
    __shared__ int s_skip, s_K;
    __shared__ double s_t;
    __shared__ ObjClass cl[256];
    __shared__ double s_q[NW][ROWS];
    if (threadIdx.x == 0) {
        s_skip = (ms->done || ms->phase != PH_Q);
        s_K = ms->K;
        s_t = ms->t;
    }
    __syncthreads();
    if (s_skip) return;
    for (int i = threadIdx.x; i < ncls; i += blockDim.x) cl[i] = classes[i];
    __syncthreads();
    const int K = s_K;
    const double t = s_t;
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const int rg = lane / G::LPR, c = lane % G::LPR;
    const int nc = (K + G::EPL - 1) / G::EPL;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // D_K prefix + d + class read, q write
        pc->bytes[1] += (16.0 * nc + 8.0 + 1.0 + double(sizeof(T))) * double(Vnz);
        pc->real[1] += 1;
    }
    double pv[G::EPL];
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) {
        const int k = c * G::EPL + e;
        pv[e] = k < K ? p[k] * dk_scale : 0.0;
    }
    Rec r = rec_identity();
    double* sq = s_q[wave];
    const int64_t nw = int64_t(gridDim.x) * NW;
    for (int64_t base = (int64_t(blockIdx.x) * NW + wave) * ROWS; base < Vpad; base += nw * ROWS) {
        V v[IT];
        load_batch<DT>(dk, base, rg, c, nc, v);
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            double part = 0.0;
#pragma unroll
            for (int e = 0; e < G::EPL; ++e) part += vget(v[it], e) * pv[e];
            part = group_sum<G::LPR>(part);
            if (c == 0) sq[it * G::RPW + rg] = part;
        }
        wave_sync();
        if (lane < ROWS) {
            const int64_t row = base + lane;
            const T qt = T(sq[lane]);   // the line search and the update use the stored value
            q[row] = qt;
            ls_voxel(cl[cls[row]], d[row], double(qt), t, r);
        }
        wave_sync();   // sq is rewritten by the next batch
    }
    Rec tot;
    const Rec mine = block_reduce(r);
    if (!arrive_and_reduce(mine, parts, arr, &tot)) return;
    __shared__ MasterState s_ms;
    __shared__ int s_fin;
    ms_load(s_ms, ms);
    if (threadIdx.x == 0) {
        s_fin = ls_decide(s_ms, tot);
        if (!s_fin) s_ms.phase = PH_LS;
    }
    __syncthreads();
    finish_step_ap(s_ms, y, p, s_fin);
    ms_store(ms, s_ms);
}

// Line-search evaluations of the aperture master (PH_LS); same evaluation
// as k_lseval, finished by finish_step_ap.
template <class T>
__global__ void __launch_bounds__(BLOCK) k_lseval_ap(const double* __restrict__ d, const T* __restrict__ q,
                                                     const uint8_t* __restrict__ cls, int64_t Vpad,
                                                     const ObjClass* __restrict__ classes, int ncls,
                                                     Rec* parts, Arrival* arr, MasterState* ms, double* y,
                                                     const double* p, ProfCounters* pc, int64_t Vnz) {
    __shared__ int s_skip;
    __shared__ double s_t;
    __shared__ ObjClass cl[256];
    if (threadIdx.x == 0) {
        s_skip = (ms->done || ms->phase != PH_LS);
        s_t = ms->t;
    }
    __syncthreads();
    if (s_skip) return;
    for (int i = threadIdx.x; i < ncls; i += blockDim.x) cl[i] = classes[i];
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        pc->bytes[2] += (8.0 + double(sizeof(T)) + 1.0) * double(Vnz);
        pc->real[2] += 1;
    }
    const double t = s_t;
    Rec r = rec_identity();
    for (int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x; i < Vpad; i += int64_t(gridDim.x) * BLOCK)
        ls_voxel(cl[cls[i]], d[i], double(q[i]), t, r);
    Rec tot;
    const Rec mine = block_reduce(r);
    if (!arrive_and_reduce(mine, parts, arr, &tot)) return;
    __shared__ MasterState s_ms;
    __shared__ int s_fin;
    ms_load(s_ms, ms);
    if (threadIdx.x == 0) s_fin = ls_decide(s_ms, tot);
    __syncthreads();
    finish_step_ap(s_ms, y, p, s_fin);
    ms_store(ms, s_ms);
}

// Reset for a solve of the aperture master: the first update pass keeps d
// (mode 2) and only produces F and grad_y at the current point.
// Forget the step-length history (a new plan starts from an empty pool, and
// its line searches must not depend on what ran before).
__global__ void k_clear_steps(MasterState* ms) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ms->last_step = 0.0;
        ms->prev_step = 0.0;
        ms->cg_valid = 0;
    }
}

__global__ void k_master_init_ap(MasterState* ms, int K, double tol, int max_steps) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ms->phase = PH_UPD;
        ms->refresh = 2;
        ms->t = 0.0;
        ms->done = 0;
        ms->steps = 0;
        ms->max_steps = max_steps;
        ms->K = K;
        ms->tol = tol;
        ms->stop_reason = 0;
        ms->ls_iter = 0;
        if (ms->cg_K != K) ms->cg_valid = 0;   // the pool changed since the last step
    }
}

}  // namespace dao
