// Master over the aperture dose matrix (gfx950).
//
// Section 2.1, eq. 1 and eq. 2 give the voxel dose of the pool as
// z = D_K y with D_kj = sum_{i in A_k} D_ij.  Here D_K is kept on the device
// as a dense row-major block dk[row * KS + k] (KS = 64 aperture slots per
// voxel row, internal row order).  A round appends one column (one forward
// product of D with the aperture's 0/1 beamlet indicator); nothing is ever
// rebuilt or transposed.  Both master products then stream D_K row by row:
//   q = D_K p              (direction of the dose, k_qstep_ap)
//   grad_y = D_K^T dF/dz    (gradient over the pool, fused into k_upd_ap)
// A row of KS values is 256 B (FP32) or 512 B (FP64); LPR lanes each load
// one 16-byte vector of it, so one wavefront instruction reads RPW whole
// consecutive rows (1 KB, fully coalesced).
//
// Step sequence: k_upd_ap -> k_dir_ap -> k_qstep_ap -> k_lseval x slots.
//   k_upd_ap   (PH_UPD) applies the last step to d (mode 0: d += t q,
//              mode 1: d = D_K y, mode 2: keep d), computes dF/dz, the
//              objective partials and the partials of grad_y per workgroup.
//   k_dir_ap   (PH_UPD) sums the partials in a fixed order, tests KKT and
//              builds the projected direction (-> PH_Q).
//   k_qstep_ap (PH_Q)   q = D_K p and the line-search evaluation at t = 0.
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

template <class T>
struct DKG {
    static constexpr int EPL = Vec16<T>::n;   // aperture slots per lane
    static constexpr int LPR = KS / EPL;      // lanes per row
    static constexpr int RPW = WAVE / LPR;    // rows per wavefront instruction
};

__device__ __forceinline__ double vget(const float4& v, int e) {
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}
__device__ __forceinline__ double vget(const double2& v, int e) { return e == 0 ? v.x : v.y; }

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

// Sum over the LPR lanes of one row (aligned lane groups); all get the sum.
template <int LPR>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
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

// Column k of D_K: dk[row * KS + k] = (D ind)_row, FP64 sums rounded to T.
template <class T>
__global__ void __launch_bounds__(SLAB_THREADS) k_dk_column(SellView<T> S, int64_t Vpad,
                                                            const T* __restrict__ ind, int N, bool stage,
                                                            int k, T* __restrict__ dk) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double s_part[KSPLIT * SLAB];
    const T* xs = stage_vec<T, T>(ind, N, reinterpret_cast<T*>(smem), stage);
    const double sum = slab_rows<T, T, double>(S, xs, s_part);
    const int64_t row = int64_t(blockIdx.x) * SLAB + threadIdx.x;
    if (threadIdx.x < SLAB && row < Vpad) dk[row * KS + k] = T(sum);
}

// Update pass (PH_UPD).  Record of workgroup b in parts2[b * (KS + 1)]:
// [objective partial, grad_y partial for apertures 0..KS-1].
template <class T>
__global__ void __launch_bounds__(BLOCK) k_upd_ap(const T* __restrict__ dk, int64_t Vpad,
                                                  double* __restrict__ d, const T* __restrict__ q,
                                                  const uint8_t* __restrict__ cls,
                                                  const ObjClass* __restrict__ classes, int ncls,
                                                  const double* __restrict__ y, double* __restrict__ parts2,
                                                  const MasterState* ms, ProfCounters* pc, int64_t Vnz) {
    using G = DKG<T>;
    using V = typename Vec16<T>::type;
    __shared__ int s_skip, s_mode, s_K;
    __shared__ double s_t;
    __shared__ ObjClass cl[256];
    __shared__ double s_acc[BLOCK / WAVE][KS];
    __shared__ double s_F[BLOCK / WAVE];
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
        yv[e] = (mode == 1 && k < K) ? y[k] : 0.0;
    }
    double acc[G::EPL];
#pragma unroll
    for (int e = 0; e < G::EPL; ++e) acc[e] = 0.0;
    double Fp = 0.0;
    const int64_t nw = int64_t(gridDim.x) * (BLOCK / WAVE);
    const int64_t gw = int64_t(blockIdx.x) * (BLOCK / WAVE) + wave;
    for (int64_t row0 = gw * G::RPW; row0 < Vpad; row0 += nw * G::RPW) {
        const int64_t row = row0 + rg;
        V v = vzero<V>();
        if (c < nc) v = reinterpret_cast<const V*>(dk + row * KS)[c];
        double dn;
        if (mode == 1) {
            double part = 0.0;
#pragma unroll
            for (int e = 0; e < G::EPL; ++e) part += vget(v, e) * yv[e];
            dn = group_sum<G::LPR>(part);
        } else {
            dn = d[row];
            if (mode == 0) dn = dn + t * double(q[row]);
        }
        const ObjClass cc = cl[cls[row]];
        const double u = grad_f(cc, dn);
        if (c == 0) {
            if (mode != 2) d[row] = dn;
            Fp += obj_f(cc, dn);
        }
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) acc[e] += u * vget(v, e);
    }
    // lanes holding the same aperture slots: combine the wave's row groups
#pragma unroll
    for (int off = G::LPR; off < WAVE; off <<= 1)
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) acc[e] += __shfl_xor(acc[e], off, WAVE);
    if (rg == 0)
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) s_acc[wave][c * G::EPL + e] = acc[e];
    Fp = wave_sum(Fp);
    if (lane == 0) s_F[wave] = Fp;
    __syncthreads();
    double* rec = parts2 + size_t(blockIdx.x) * (KS + 1);
    if (threadIdx.x < KS) {
        double s = 0.0;
        for (int w = 0; w < BLOCK / WAVE; ++w) s += s_acc[w][threadIdx.x];
        rec[1 + threadIdx.x] = s;
    } else if (threadIdx.x == KS) {
        double s = 0.0;
        for (int w = 0; w < BLOCK / WAVE; ++w) s += s_F[w];
        rec[0] = s;
    }
}

// Direction step (single block, 1024 threads, PH_UPD): F and grad_y from
// the update's partials (fixed order), KKT test, projected direction,
// longest feasible step.
__global__ void __launch_bounds__(1024) k_dir_ap(const double* __restrict__ parts2, int nblk,
                                                 const double* __restrict__ y, double* __restrict__ p,
                                                 double* __restrict__ grad, MasterState* ms, ProfCounters* pc) {
    constexpr int SPLIT = 16;   // threads per record column
    __shared__ int s_skip, s_K;
    __shared__ double s_part[KS + 1][SPLIT];
    __shared__ double s_red[KS + 1];
    if (threadIdx.x == 0) {
        s_skip = ms->done || ms->phase != PH_UPD;
        s_K = ms->K;
    }
    __syncthreads();
    if (s_skip) return;
    const int K = s_K;
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
        double s = 0.0;
        for (int b = b0; b < b1; ++b) s += parts2[size_t(b) * (KS + 1) + j];
        s_part[j][part] = s;
    }
    __syncthreads();
    if (threadIdx.x <= K) {
        double s = 0.0;
        for (int q = 0; q < SPLIT; ++q) s += s_part[threadIdx.x][q];
        s_red[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    ms->F = ms->F_const + s_red[0];
    double kkt = 0.0;
    for (int k = 0; k < K; ++k) kkt = fmax(kkt, fabs(fmin(y[k], s_red[1 + k])));
    ms->kkt = kkt;
    int go = 1;
    if (!(kkt > ms->tol)) {
        ms->stop_reason = 1;
        go = 0;
    } else if (ms->steps >= ms->max_steps) {
        ms->stop_reason = 2;
        go = 0;
    }
    double tmax = INFINITY, gp = 0.0;
    int any = 0;
    if (go) {
        for (int k = 0; k < K; ++k) {
            const double gk = s_red[1 + k];
            double pk = -gk;
            if (y[k] == 0.0 && gk >= 0.0) pk = 0.0;
            p[k] = pk;
            grad[k] = gk;
            if (pk != 0.0) any = 1;
            if (pk < 0.0) tmax = fmin(tmax, y[k] / (-pk));
            gp += gk * pk;
        }
        if (!any) {
            ms->stop_reason = 3;
            go = 0;
        }
    }
    if (!go) {
        ms->done = 1;
        return;
    }
    ms->t_max = tmax;
    ms->gphi0 = gp;
    ms->t = 0.0;
    ms->lo = 0.0;
    ms->hi = tmax;
    ms->hi_known = 0;
    ms->ls_iter = 0;
    ms->phase = PH_Q;
}

// Final step of a line search in the aperture master (last block): y
// update with exact zeros for blocking apertures, step count, update mode.
__device__ __forceinline__ void finish_step_ap(MasterState* ms, double* y, const double* p, int fin) {
    if (!fin) return;
    const int K = ms->K;
    const double t = ms->t, tmax = ms->t_max;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const double pk = p[k];
        const double ratio = pk < 0.0 ? y[k] / (-pk) : INFINITY;
        double yn = y[k] + t * pk;
        if (t == tmax && ratio == t) yn = 0.0;
        y[k] = fmax(yn, 0.0);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ms->steps += 1;
        ms->total_steps += 1;
        ms->last_step = t;
        ms->refresh = (ms->steps % ms->refresh_every) == 0 ? 1 : 0;
        ms->phase = PH_UPD;
    }
}

// q = D_K p and the line-search evaluation at t = 0 (PH_Q).
template <class T>
__global__ void __launch_bounds__(BLOCK) k_qstep_ap(const T* __restrict__ dk, int64_t Vpad,
                                                    const double* __restrict__ d,
                                                    const uint8_t* __restrict__ cls,
                                                    const ObjClass* __restrict__ classes, int ncls,
                                                    T* __restrict__ q, Rec* parts, Arrival* arr,
                                                    MasterState* ms, double* y, const double* p,
                                                    ProfCounters* pc, int64_t Vnz) {
    using G = DKG<T>;
    using V = typename Vec16<T>::type;
    __shared__ int s_skip, s_K;
    __shared__ double s_t;
    __shared__ ObjClass cl[256];
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
        pv[e] = k < K ? p[k] : 0.0;
    }
    Rec r = rec_identity();
    const int64_t nw = int64_t(gridDim.x) * (BLOCK / WAVE);
    const int64_t gw = int64_t(blockIdx.x) * (BLOCK / WAVE) + wave;
    for (int64_t row0 = gw * G::RPW; row0 < Vpad; row0 += nw * G::RPW) {
        const int64_t row = row0 + rg;
        V v = vzero<V>();
        if (c < nc) v = reinterpret_cast<const V*>(dk + row * KS)[c];
        double part = 0.0;
#pragma unroll
        for (int e = 0; e < G::EPL; ++e) part += vget(v, e) * pv[e];
        const double qd = group_sum<G::LPR>(part);
        if (c == 0) {
            const T qt = T(qd);   // the line search and the update use the stored value
            q[row] = qt;
            ls_voxel(cl[cls[row]], d[row], double(qt), t, r);
        }
    }
    Rec tot;
    const Rec mine = block_reduce(r);
    if (!arrive_and_reduce(mine, parts, arr, &tot)) return;
    __shared__ int s_fin;
    if (threadIdx.x == 0) {
        s_fin = ls_decide(ms, tot);
        if (!s_fin) ms->phase = PH_LS;
    }
    __syncthreads();
    finish_step_ap(ms, y, p, s_fin);
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
    __shared__ int s_fin;
    if (threadIdx.x == 0) s_fin = ls_decide(ms, tot);
    __syncthreads();
    finish_step_ap(ms, y, p, s_fin);
}

// Reset for a solve of the aperture master: the first update pass keeps d
// (mode 2) and only produces F and grad_y at the current point.
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
    }
}

}  // namespace dao
