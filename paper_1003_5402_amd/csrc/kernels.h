// gfx950 kernels of the DAO hot path.
//
// Layouts (built on the host, see layout.cpp):
//   forward  : sliced ELL, 64 voxel rows per slice, entries of a slice stored
//              column-major (entry k of the slice's lane-l row at
//              slice_ptr[s] + 64 k + l) so a wavefront reads each k as one
//              contiguous 64-lane load; 16-bit beamlet indices.  A workgroup
//              ("slab") owns 4 slices = 256 rows; each slice's entries are
//              split into 4 contiguous k-ranges, one wavefront each, so 16
//              wavefronts stream one slab.
//   transpose: beamlet-major copy (one run of (internal row, value) per
//              beamlet), read by one workgroup per beamlet.
//   vectors  : "internal" voxel vectors (d, q, u, class) follow the slice
//              row order; rows past the last non-empty voxel are padding
//              with class "none" and zero coefficients.
//
// Reductions are deterministic: every sum is taken in a fixed order
// (per-lane sequential, then a fixed butterfly, then a fixed block order),
// never with floating-point atomics.  Grid-wide results are combined by the
// last workgroup to arrive (integer arrival counters only); no launch ever
// waits on another workgroup.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dao_common.h"

namespace dao {

constexpr int KSPLIT = 4;                          // wavefronts per slice
constexpr int SPB = 4;                             // slices per slab
constexpr int SLAB = SPB * SLICE;                  // rows per slab
constexpr int SLAB_THREADS = SPB * KSPLIT * WAVE;  // 1024
constexpr int NSLOT = 8;                           // arrival counters
constexpr int SLOT_STRIDE = 32;                    // 128 B between counters

// Arrival counters of the last-workgroup pattern.  Workgroups hash onto
// NSLOT counters (one cache line each) so that arrivals of different
// workgroups do not serialise on one address; the last arrival of every
// counter then arrives at a top-level counter.
struct Arrival {
    uint32_t c[(NSLOT + 1) * SLOT_STRIDE];
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double grad_f(const ObjClass& c, double z) {
    // dF/dz of eq. 9 + eq. 10 for one voxel (both structures' terms)
    return -2.0 * c.a * fmax(0.0, c.t_under - z) + 2.0 * c.b * fmax(0.0, z - c.t_over) -
           2.0 * c.a2 * fmax(0.0, c.t_under2 - z) + 2.0 * c.b2 * fmax(0.0, z - c.t_over2);
}

__device__ __forceinline__ double obj_f(const ObjClass& c, double z) {
    const double un = fmax(0.0, c.t_under - z);
    const double ov = fmax(0.0, z - c.t_over);
    const double un2 = fmax(0.0, c.t_under2 - z);
    const double ov2 = fmax(0.0, z - c.t_over2);
    return c.a * un * un + c.b * ov * ov + c.a2 * un2 * un2 + c.b2 * ov2 * ov2;
}

// Per-voxel threshold shift of internal row r (0 without shifts).
__device__ __forceinline__ double tau_at(const double* tau, int64_t r) { return tau ? tau[r] : 0.0; }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, WAVE));
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
    return v;
}

// Reduction record: (sum, sum, sum, min, max, sum).  The line search needs
// phi', the slopes of phi' right and left of t and the nearest breakpoints
// on both sides; the last slot carries an objective partial.
struct Rec {
    double s0, s1, s2, mn, mx, s5;
};

__device__ __forceinline__ Rec rec_identity() {
    return Rec{0.0, 0.0, 0.0, INFINITY, -INFINITY, 0.0};
}

__device__ __forceinline__ void rec_add(Rec& a, const Rec& b) {
    a.s0 += b.s0;
    a.s1 += b.s1;
    a.s2 += b.s2;
    a.mn = fmin(a.mn, b.mn);
    a.mx = fmax(a.mx, b.mx);
    a.s5 += b.s5;
}

// Reduce one Rec over the block (up to 1024 threads); valid in thread 0.
__device__ __forceinline__ Rec block_reduce(Rec r) {
    __shared__ Rec s_w[1024 / WAVE];
    r.s0 = wave_sum(r.s0);
    r.s1 = wave_sum(r.s1);
    r.s2 = wave_sum(r.s2);
    r.mn = wave_min(r.mn);
    r.mx = wave_max(r.mx);
    r.s5 = wave_sum(r.s5);
    const int nw = blockDim.x / WAVE;
    if ((threadIdx.x % WAVE) == 0) s_w[threadIdx.x / WAVE] = r;
    __syncthreads();
    Rec out = rec_identity();
    if (threadIdx.x == 0)
        for (int i = 0; i < nw; ++i) rec_add(out, s_w[i]);
    __syncthreads();
    return out;
}

// Called by thread 0 of every workgroup after it published its results:
// true in exactly one workgroup, the last to arrive, which may then read
// every other workgroup's results.  Counters are reset for the next launch.
__device__ __forceinline__ bool arrive_last(Arrival* A) {
    const uint32_t nb = gridDim.x;
    const uint32_t slot = blockIdx.x % NSLOT;
    const uint32_t expect = (nb - slot + NSLOT - 1) / NSLOT;   // workgroups on this counter
    __threadfence();
    const uint32_t prev = atomicAdd(&A->c[slot * SLOT_STRIDE], 1u);
    if (prev + 1 != expect) return false;
    atomicExch(&A->c[slot * SLOT_STRIDE], 0u);
    __threadfence();
    const uint32_t nslots = nb < NSLOT ? nb : NSLOT;
    const uint32_t p2 = atomicAdd(&A->c[NSLOT * SLOT_STRIDE], 1u);
    if (p2 + 1 != nslots) return false;
    atomicExch(&A->c[NSLOT * SLOT_STRIDE], 0u);
    __threadfence();
    return true;
}

// Thread 0 of every block stores its record; the last block to arrive
// reduces all records in block order.  Returns true in every thread of the
// last block, with the total in *total (valid in thread 0).
__device__ __forceinline__ bool arrive_and_reduce(Rec mine, Rec* parts, Arrival* A, Rec* total) {
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        parts[blockIdx.x] = mine;
        s_last = arrive_last(A);
    }
    __syncthreads();
    if (!s_last) return false;
    __threadfence();
    // fixed-order reduction: each thread a contiguous run, then the block
    Rec acc = rec_identity();
    const int n = gridDim.x;
    const int per = (n + blockDim.x - 1) / blockDim.x;
    const int b0 = threadIdx.x * per;
    const int b1 = min(n, b0 + per);
    for (int b = b0; b < b1; ++b) rec_add(acc, parts[b]);
    const Rec t = block_reduce(acc);
    if (threadIdx.x == 0) *total = t;
    __syncthreads();
    return true;
}

// The device-resident master state is read and written through an LDS copy:
// one parallel load and one parallel store per launch instead of a chain of
// dependent single-field accesses (each of which may cross XCDs).
constexpr int MS_WORDS = int(sizeof(MasterState) / 8);
static_assert(sizeof(MasterState) % 8 == 0, "state is copied in 8-byte words");

__device__ __forceinline__ void ms_load(MasterState& s, const MasterState* g) {
    if (threadIdx.x < MS_WORDS)
        reinterpret_cast<uint64_t*>(&s)[threadIdx.x] = reinterpret_cast<const uint64_t*>(g)[threadIdx.x];
    __syncthreads();
}

__device__ __forceinline__ void ms_store(MasterState* g, const MasterState& s) {
    __syncthreads();
    if (threadIdx.x < MS_WORDS)
        reinterpret_cast<uint64_t*>(g)[threadIdx.x] = reinterpret_cast<const uint64_t*>(&s)[threadIdx.x];
}

// Contribution of one voxel to the line-search evaluation at step t:
// phi'(t) = sum q_j dF/dz_j(d_j + t q_j); slopes of phi' just right / left of
// t (without the factor 2); nearest breakpoint above / below t.
// Breakpoints of voxel z(t) = d + t q against its thresholds (NaN when the
// term is absent or q = 0, so they never count).  They do not depend on t.
__device__ __forceinline__ void ls_breakpoints(const ObjClass& c, double d, double q, double& bu, double& bo) {
    bu = (c.a > 0.0 && q != 0.0) ? (c.t_under - d) / q : NAN;
    bo = (c.b > 0.0 && q != 0.0) ? (c.t_over - d) / q : NAN;
}

// Curvature flags and breakpoints of one (a, T-, b, T+) term at z = d + t q.
__device__ __forceinline__ void ls_term(double a, double tu, double b, double to, double z, double q,
                                        double q2, double bu, double bo, double t, Rec& r) {
    const bool ua = a > 0.0, ob = b > 0.0;
    const bool under_r = ua && ((z < tu) || (z == tu && q < 0.0));
    const bool over_r = ob && ((z > to) || (z == to && q > 0.0));
    const bool under_l = ua && ((z < tu) || (z == tu && q > 0.0));
    const bool over_l = ob && ((z > to) || (z == to && q < 0.0));
    r.s1 += q2 * ((under_r ? a : 0.0) + (over_r ? b : 0.0));
    r.s2 += q2 * ((under_l ? a : 0.0) + (over_l ? b : 0.0));
    // comparisons with NaN are false: absent breakpoints never count
    if (bu > t) r.mn = fmin(r.mn, bu);
    if (bu < t) r.mx = fmax(r.mx, bu);
    if (bo > t) r.mn = fmin(r.mn, bo);
    if (bo < t) r.mx = fmax(r.mx, bo);
}

// Line-search sums of one voxel at t, with the first structure's
// breakpoints given (a second structure's are computed here).
__device__ __forceinline__ void ls_voxel_bp(const ObjClass& c, double d, double q, double bu, double bo, double t,
                                            Rec& r) {
    const double z = d + t * q;
    r.s0 += q * grad_f(c, z);
    const double q2 = q * q;
    ls_term(c.a, c.t_under, c.b, c.t_over, z, q, q2, bu, bo, t, r);
    if (c.a2 > 0.0 || c.b2 > 0.0) {
        const double bu2 = (c.a2 > 0.0 && q != 0.0) ? (c.t_under2 - d) / q : NAN;
        const double bo2 = (c.b2 > 0.0 && q != 0.0) ? (c.t_over2 - d) / q : NAN;
        ls_term(c.a2, c.t_under2, c.b2, c.t_over2, z, q, q2, bu2, bo2, t, r);
    }
}

__device__ __forceinline__ void ls_voxel(const ObjClass& c, double d, double q, double t, Rec& r) {
    double bu, bo;
    ls_breakpoints(c, d, q, bu, bo);
    ls_voxel_bp(c, d, q, bu, bo, t, r);
}

// First trial point of a line search: the length of the step before the
// last, capped at t_max, when positive, else 0.  Gradient projection with
// exact line searches tends to alternate between two step lengths, so that
// point usually lies inside the linear piece of phi' that holds the
// minimiser, where the Newton point from it is exact and one evaluation
// ends the search.  The search needs no evaluation at 0: phi'(0) < 0 holds
// for every direction that is not zero.
__device__ __forceinline__ double ls_first_trial(double prev_step, double t_max) {
    const double tb = fmin(prev_step, t_max);
    return tb > 0.0 ? tb : 0.0;
}

// Wavefront reductions through DPP lane moves (no LDS round trip).  The
// order is fixed: xor 1, xor 2 inside quads, half-row mirror, row mirror,
// then the row broadcasts; lane 63 ends with the total, which is then read
// into every lane.  Call with all 64 lanes active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_move(double v, double ident) {
    const long long b = __double_as_longlong(v), id = __double_as_longlong(ident);
    const int lo = __builtin_amdgcn_update_dpp(int(id), int(b), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(int(id >> 32), int(b >> 32), CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double lane63(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(int(b), 63), hi = __builtin_amdgcn_readlane(int(b >> 32), 63);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
// op: 0 sum, 1 min, 2 max
template <int OP>
__device__ __forceinline__ double dpp_comb(double a, double b) {
    return OP == 0 ? a + b : OP == 1 ? fmin(a, b) : fmax(a, b);
}
template <int OP>
__device__ __forceinline__ double wave_reduce_dpp(double v) {
    const double id = OP == 0 ? 0.0 : OP == 1 ? INFINITY : -INFINITY;
    v = dpp_comb<OP>(v, dpp_move<0xB1, 0xF>(v, id));    // quad_perm [1,0,3,2]
    v = dpp_comb<OP>(v, dpp_move<0x4E, 0xF>(v, id));    // quad_perm [2,3,0,1]
    v = dpp_comb<OP>(v, dpp_move<0x141, 0xF>(v, id));   // row_half_mirror
    v = dpp_comb<OP>(v, dpp_move<0x140, 0xF>(v, id));   // row_mirror
    v = dpp_comb<OP>(v, dpp_move<0x142, 0xA>(v, id));   // row_bcast15 into rows 1, 3
    v = dpp_comb<OP>(v, dpp_move<0x143, 0xC>(v, id));   // row_bcast31 into rows 2, 3
    return lane63(v);
}

// Search direction of gradient projection for one wavefront, lane k holding
// pool aperture k (K <= 64; every lane of the wavefront calls it).  The
// projected negative gradient r is -grad_k except 0 where y_k = 0 and
// grad_k >= 0 (the free set is where it may be non-zero).  With mem (the
// last step of this pool did not block and the conjugate direction is on)
// and an unchanged free set, p = r + beta p_prev with the Polak-Ribiere
// beta truncated at 0, kept only if it is a descent direction; else p = r.
__device__ __forceinline__ double cg_dir_wave(bool in, double yk, double gk, bool mem, double pprev,
                                              double rprev, bool fprev, double& r, bool& fr) {
    fr = in && !(yk == 0.0 && gk >= 0.0);
    r = fr ? -gk : 0.0;
    double p = r;
    if (mem && __all(fr == (in && fprev))) {
        const double rp = in ? rprev : 0.0;
        const double num = wave_reduce_dpp<0>(r * (r - rp));
        const double den = wave_reduce_dpp<0>(rp * rp);
        const double beta = den > 0.0 ? fmax(0.0, num / den) : 0.0;
        const double cand = r + beta * (in ? pprev : 0.0);
        if (wave_reduce_dpp<0>(in ? gk * cand : 0.0) < 0.0) p = cand;
    }
    return p;
}

// ---------------------------------------------------------------------------
// forward products over slabs
// ---------------------------------------------------------------------------
// Stored value of D: the context type, or a 16-bit pattern scaled per
// beamlet (FP16 / BF16, optionally with an FP16 residual).
__device__ __forceinline__ float dval(float v) { return v; }
__device__ __forceinline__ double dval(double v) { return v; }
__device__ __forceinline__ float dval(__half v) { return __half2float(v); }
__device__ __forceinline__ float dval(__hip_bfloat16 v) { return __bfloat162float(v); }
// hi + lo of a split value: exact in FP32 (lo is below hi's last bit)
template <class VT, bool LO>
__device__ __forceinline__ auto dval2(VT hi, const __half* lo_p) {
    if constexpr (LO)
        return dval(hi) + __half2float(*lo_p);
    else
        return dval(hi);
}

template <class T>
struct SellView {
    const uint32_t* slice_ptr;
    const int32_t* slice_w;
    const T* val;
    const uint16_t* col;
    int64_t nslices;
    const __half* lo;   // FP16 residuals (same positions as val), or null
};

// Forward layout: in a slice of SLICE rows, entries come in groups of 4 of
// one row (slice width padded to a multiple of 4): entry k of lane l sits at
// base + (k / 4) * 4 * SLICE + 4 * l + k % 4, so one lane reads a group with
// one 4-element load and a wavefront instruction reads 4 * SLICE entries.
template <class T>
struct alignas(4 * sizeof(T)) Quad {
    T e[4];
};

// Lane `lane` of a wavefront: entries k0..k1-1 (multiples of 4) of its row in
// the slice that starts at entry `base`, visited in stored (ascending
// beamlet) order, with G groups of loads in flight per iteration.
// The first group of a lane's chunk, loaded ahead (before x is staged).
template <class T>
struct FirstGroup {
    Quad<T> v;
    Quad<uint16_t> c;
    Quad<__half> l;
};

template <class T, class XT, class Acc, bool LO, int G>
__device__ __forceinline__ Acc sell_dot(const T* __restrict__ val, const __half* __restrict__ lo,
                                        const uint16_t* __restrict__ col, uint32_t base, int k0, int k1,
                                        int lane, const XT* __restrict__ xs,
                                        const FirstGroup<T>* first = nullptr) {
    const int g0 = k0 >> 2, g1 = k1 >> 2;
    const size_t o = base + size_t(g0) * (4 * SLICE) + size_t(lane) * 4;
    Acc acc = Acc(0);
    int gs = g0;
    if (first && g0 < g1) {   // group g0 already loaded
#pragma unroll
        for (int q = 0; q < 4; ++q) acc += Acc(dval2<T, LO>(first->v.e[q], &first->l.e[q])) * Acc(xs[first->c.e[q]]);
        gs = g0 + 1;
    }
    for (int g = gs; g < g1; g += G) {
        Quad<T> v[G];
        Quad<uint16_t> c[G];
        Quad<__half> l[G];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const size_t e = o + size_t(g - g0 + u) * (4 * SLICE);
            if (G == 1 || g + u < g1) {
                v[u] = *reinterpret_cast<const Quad<T>*>(val + e);
                c[u] = *reinterpret_cast<const Quad<uint16_t>*>(col + e);
                if (LO) l[u] = *reinterpret_cast<const Quad<__half>*>(lo + e);
            }
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
            if (G == 1 || g + u < g1) {
#pragma unroll
                for (int q = 0; q < 4; ++q) acc += Acc(dval2<T, LO>(v[u].e[q], &l[u].e[q])) * Acc(xs[c[u].e[q]]);
            }
        }
    }
    return acc;
}

// As sell_dot for C chunks of the same row at once (chunk c: entries
// k0[c]..k1[c]-1), one group of each chunk per iteration, each chunk summed
// in its own accumulator in stored order (the same sums as C sell_dot calls).
template <class T, class XT, class Acc, bool LO, int C>
__device__ __forceinline__ void sell_dot_multi(const T* __restrict__ val, const __half* __restrict__ lo,
                                               const uint16_t* __restrict__ col, uint32_t base, const int* k0,
                                               const int* k1, int lane, const XT* __restrict__ xs, Acc* acc) {
    int n = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        acc[c] = Acc(0);
        n = max(n, (k1[c] - k0[c]) >> 2);
    }
    for (int g = 0; g < n; ++g) {
        Quad<T> v[C];
        Quad<uint16_t> cq[C];
        Quad<__half> l[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (g < ((k1[c] - k0[c]) >> 2)) {
                const size_t e = base + size_t((k0[c] >> 2) + g) * (4 * SLICE) + size_t(lane) * 4;
                v[c] = *reinterpret_cast<const Quad<T>*>(val + e);
                cq[c] = *reinterpret_cast<const Quad<uint16_t>*>(col + e);
                if (LO) l[c] = *reinterpret_cast<const Quad<__half>*>(lo + e);
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (g < ((k1[c] - k0[c]) >> 2)) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc[c] += Acc(dval2<T, LO>(v[c].e[q], &l[c].e[q])) * Acc(xs[cq[c].e[q]]);
            }
        }
    }
}

// Row sums of this workgroup's slab of SPBt slices (SLAB_THREADS threads).
// Every slice's entry groups are split into KSPLIT chunks whose partials
// meet in s_part (KSPLIT * SPBt * SLICE values) and are added in chunk
// order, whatever the geometry: with SPBt = SPB each wavefront sums one
// chunk; with more slices per slab each wavefront sums several chunks of
// its slice together (fewer workgroups, each staging x once for more rows;
// the same sums).  Returns the row sum in threads t < SPBt * SLICE (row
// blockIdx.x * SPBt * SLICE + t).
// Entry range [k0, k1) of chunk q of slice s (KSPLIT chunks of whole groups).
template <class T>
__device__ __forceinline__ void chunk_range(const SellView<T>& S, int64_t s, int q, int& k0, int& k1) {
    const int w = S.slice_w[s];   // a multiple of 4
    const int kc = ((w >> 2) + KSPLIT - 1) / KSPLIT * 4;
    k0 = min(w, q * kc);
    k1 = min(w, k0 + kc);
}

template <class T, class XT, class Acc, bool LO = false, int DEEP = 0, int SPBt = SPB>
__device__ __forceinline__ Acc slab_rows(const SellView<T>& S, const XT* __restrict__ xs, Acc* s_part,
                                         const FirstGroup<T>* first = nullptr) {
    constexpr int KSP = SPB * KSPLIT / SPBt;   // wavefronts per slice
    constexpr int CPW = KSPLIT / KSP;          // chunks per wavefront
    constexpr int SLABt = SPBt * SLICE;
    static_assert(KSP * CPW == KSPLIT && SPBt * KSP * WAVE == SLAB_THREADS, "slab geometry");
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int j = wave / KSP, kp = wave % KSP;
    const int64_t s = int64_t(blockIdx.x) * SPBt + j;
    Acc acc[CPW];
#pragma unroll
    for (int i = 0; i < CPW; ++i) acc[i] = Acc(0);
    if (s < S.nslices) {
        const int w = S.slice_w[s];   // a multiple of 4
        const int kc = ((w >> 2) + KSPLIT - 1) / KSPLIT * 4;
        if constexpr (CPW == 1) {
            int k0, k1;
            chunk_range(S, s, kp, k0, k1);
            constexpr int G = DEEP > 0 ? DEEP / 4 : 1;   // groups of loads in flight
            acc[0] = sell_dot<T, XT, Acc, LO, G>(S.val, S.lo, S.col, S.slice_ptr[s], k0, k1, lane, xs, first);
        } else {
            int k0[CPW], k1[CPW];
#pragma unroll
            for (int i = 0; i < CPW; ++i) {
                k0[i] = min(w, (kp * CPW + i) * kc);
                k1[i] = min(w, k0[i] + kc);
            }
            sell_dot_multi<T, XT, Acc, LO, CPW>(S.val, S.lo, S.col, S.slice_ptr[s], k0, k1, lane, xs, acc);
        }
    }
#pragma unroll
    for (int i = 0; i < CPW; ++i) s_part[(kp * CPW + i) * SLABt + j * SLICE + lane] = acc[i];
    __syncthreads();
    Acc sum = Acc(0);
    if (threadIdx.x < SLABt) {
#pragma unroll
        for (int q = 0; q < KSPLIT; ++q) sum += s_part[q * SLABt + threadIdx.x];
    }
    return sum;
}

// Row sums of the slab against the n-vector src: staged into LDS (times the
// per-beamlet scale when one is given) and gathered from there, or gathered
// from device memory when not staged.  The two gathers are separate code
// paths, so the staged one compiles to LDS reads rather than generic ones.
template <class VT, class XT, class Acc, bool LO = false, int DEEP = 0, int SPBt = SPB, class ST>
__device__ __forceinline__ Acc slab_rows_x(const SellView<VT>& S, const ST* __restrict__ src, int n, XT* lds,
                                           bool stage, const float* __restrict__ scale, Acc* s_part) {
    if (stage) {
        // one wavefront per chunk: load the chunk's first group before x is
        // staged, so that the two memory round trips overlap
        FirstGroup<VT> fg;
        constexpr bool PRE = SPBt == SPB;
        if (PRE) {
            const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
            const int64_t s = int64_t(blockIdx.x) * SPB + wave / KSPLIT;
            if (s < S.nslices) {
                int k0, k1;
                chunk_range(S, s, wave % KSPLIT, k0, k1);
                if (k0 < k1) {
                    const size_t e = S.slice_ptr[s] + size_t(k0 >> 2) * (4 * SLICE) + size_t(lane) * 4;
                    fg.v = *reinterpret_cast<const Quad<VT>*>(S.val + e);
                    fg.c = *reinterpret_cast<const Quad<uint16_t>*>(S.col + e);
                    if (LO) fg.l = *reinterpret_cast<const Quad<__half>*>(S.lo + e);
                }
            }
        }
        if (scale)
            for (int i = threadIdx.x; i < n; i += blockDim.x) lds[i] = XT(src[i]) * XT(scale[i]);
        else
            for (int i = threadIdx.x; i < n; i += blockDim.x) lds[i] = XT(src[i]);
        __syncthreads();
        return slab_rows<VT, XT, Acc, LO, DEEP, SPBt>(S, lds, s_part, PRE ? &fg : nullptr);
    }
    return slab_rows<VT, XT, Acc, LO, DEEP, SPBt>(S, reinterpret_cast<const XT*>(src), s_part);
}

// ---------------------------------------------------------------------------
// plain products and objective (C-ABI calls, round ends)
// ---------------------------------------------------------------------------

// d_ext[perm[r]] = (D x)_r for every row of the slab; x staged in LDS
// (times the per-beamlet scale of a 16-bit value format).  DEEP > 0 keeps
// DEEP entries per lane in flight, SPBt slices per workgroup (the autotuned
// variants; the same sums).
template <class T, class VT = T, bool LO = false, int DEEP = 0, int SPBt = SPB>
__global__ void __launch_bounds__(SLAB_THREADS) k_dose(SellView<VT> S, const int32_t* __restrict__ perm,
                                                       int64_t Vpad, const T* __restrict__ x, int N,
                                                       bool stage, const float* __restrict__ scale,
                                                       T* __restrict__ d_ext) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ T s_part[KSPLIT * SPBt * SLICE];
    const T sum =
        slab_rows_x<VT, T, T, LO, DEEP, SPBt>(S, x, N, reinterpret_cast<T*>(smem), stage, scale, s_part);
    const int64_t row = int64_t(blockIdx.x) * (SPBt * SLICE) + threadIdx.x;
    if (threadIdx.x < SPBt * SLICE && row < Vpad) {
        const int32_t j = perm[row];
        if (j >= 0) d_ext[j] = sum;
    }
}

// d_ext[perm[r]] = (D x)_r, whole rows per lane: a grid of a few
// workgroups per compute unit, each staging x (times the per-beamlet scale
// of a 16-bit format) in LDS once and then walking slices with the grid's
// stride (wavefront w of workgroup b: slices b * 4 + w, then every
// gridDim.x * 4 further).  The next slice's header is loaded while the
// current one is summed, and each lane issues GB groups of its row before
// adding them, so a whole row of the head-and-neck matrix is in flight at
// once.  The terms are added chunk by chunk exactly as the slab form adds
// them (the KSPLIT chunks of whole groups, each from 0 in stored order, then
// the chunk sums in order, empty chunks included), so the result is the
// same bit for bit.
//
// ORDERED: the slices of wavefront gw (of nw = gridDim.x * 4 in the grid) are
// order[k * nw + gw] for k = 0, 1, ... up to the first -1 (at most rounds),
// a list the host balances by slice width (the widest slices first, each to
// the wavefront with the least work so far): the length sort puts the widest
// slices at the start of every sort window, and a plain grid stride would
// give some wavefronts several of them.  Every row's sum is the same either
// way; only which wavefront computes it changes.
constexpr int ROWS_THREADS = 256;
template <class T, class VT = T, bool LO = false, int GB = 8, bool ORDERED = false>
__global__ void __launch_bounds__(ROWS_THREADS) k_dose_rows(SellView<VT> S, const int32_t* __restrict__ perm,
                                                            int64_t Vpad, const T* __restrict__ x, int N,
                                                            const float* __restrict__ scale, T* __restrict__ d_ext,
                                                            const int32_t* __restrict__ order = nullptr,
                                                            int rounds = 0) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* xs = reinterpret_cast<T*>(smem);
    constexpr int NW = ROWS_THREADS / WAVE;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int64_t stride = int64_t(gridDim.x) * NW;
    const int64_t gw = int64_t(blockIdx.x) * NW + wave;
    // slice of this wavefront's k-th turn (-1: none)
    auto slice_at = [&](int64_t k) -> int64_t {
        if (ORDERED) return k < rounds ? int64_t(order[k * stride + gw]) : -1;
        const int64_t sl = gw + k * stride;
        return sl < S.nslices ? sl : -1;
    };
    int64_t k = 0;
    int64_t s = slice_at(0);
    uint32_t nbase = 0;
    int nwid = 0;
    if (s >= 0) {
        nbase = S.slice_ptr[s];
        nwid = S.slice_w[s];
    }
    if (scale)
        for (int i = threadIdx.x; i < N; i += blockDim.x) xs[i] = T(x[i]) * T(scale[i]);
    else
        for (int i = threadIdx.x; i < N; i += blockDim.x) xs[i] = T(x[i]);
    __syncthreads();
    while (s >= 0) {
        const uint32_t base = nbase;
        const int w = nwid;   // a multiple of 4
        const int64_t s_next = slice_at(++k);
        if (s_next >= 0) {
            nbase = S.slice_ptr[s_next];
            nwid = S.slice_w[s_next];
        }
        const int ng = w >> 2;
        const int gpc = (ng + KSPLIT - 1) / KSPLIT;   // groups per chunk, as chunk_range
        const size_t o = size_t(base) + size_t(lane) * 4;
        T sum = T(0), cur = T(0);
        int q = 0;
        for (int g0 = 0; g0 < ng; g0 += GB) {
            Quad<VT> v[GB];
            Quad<uint16_t> c[GB];
            Quad<__half> l[GB];
#pragma unroll
            for (int u = 0; u < GB; ++u) {
                if (g0 + u < ng) {
                    const size_t e = o + size_t(g0 + u) * (4 * SLICE);
                    v[u] = *reinterpret_cast<const Quad<VT>*>(S.val + e);
                    c[u] = *reinterpret_cast<const Quad<uint16_t>*>(S.col + e);
                    if (LO) l[u] = *reinterpret_cast<const Quad<__half>*>(S.lo + e);
                }
            }
#pragma unroll
            for (int u = 0; u < GB; ++u) {
                if (g0 + u < ng) {
                    if ((g0 + u) / gpc != q) {   // the next chunk begins
                        sum += cur;
                        cur = T(0);
                        ++q;
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e) cur += T(dval2<VT, LO>(v[u].e[e], &l[u].e[e])) * xs[c[u].e[e]];
                }
            }
        }
        sum += cur;
        for (++q; q < KSPLIT; ++q) sum += T(0);   // the empty chunks
        const int64_t row = s * SLICE + lane;
        if (row < Vpad) {
            const int32_t j = perm[row];
            if (j >= 0) d_ext[j] = sum;
        }
        s = s_next;
    }
}

// The master dose from its intensities, in FP64 throughout: d[row] =
// (D x64)_row over internal rows, every product D_ij x_i and every sum in
// double (the stored D values are exact in double; a 16-bit format's scale
// multiplies x first).  Used at every round end, so that the prices of the
// sub-problem (eq. 8) see the dose of the current intensities rather than
// the master's incremental one, and on a state restore.
template <class VT, bool LO = false>
__global__ void __launch_bounds__(SLAB_THREADS) k_dose_exact(SellView<VT> S, int64_t Vpad,
                                                             const double* __restrict__ x64, int N, bool stage,
                                                             const float* __restrict__ scale,
                                                             const double* __restrict__ tau,
                                                             double* __restrict__ d) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double s_part[KSPLIT * SLAB];
    const double sum =
        slab_rows_x<VT, double, double, LO>(S, x64, N, reinterpret_cast<double*>(smem), stage, scale, s_part);
    const int64_t row = int64_t(blockIdx.x) * SLAB + threadIdx.x;
    // the master keeps the dose minus the per-voxel threshold shift
    if (threadIdx.x < SLAB && row < Vpad) d[row] = sum - tau_at(tau, row);
}

template <class T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

// out[i] = |in[i]|.
__global__ void k_abs_copy(const double* __restrict__ in, int64_t n, double* __restrict__ out) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        out[i] = fabs(in[i]);
}

// d[r] = -tau[r] (0 without shifts): the master's shifted form of zero dose.
__global__ void k_neg_or_zero(const double* __restrict__ tau, int64_t n, double* __restrict__ d) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        d[i] = -tau_at(tau, i);
}

// out[perm[r]] = in[r] + tau[r] for internal rows (caller order): the dose
// from the master's shifted dose, after a fill of out.
__global__ void k_scatter_shift(const double* __restrict__ in, const double* __restrict__ tau,
                                const int32_t* __restrict__ perm, int64_t n, double* __restrict__ out) {
    for (int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += int64_t(gridDim.x) * blockDim.x) {
        const int32_t j = perm[r];
        if (j >= 0) out[j] = in[r] + tau_at(tau, r);
    }
}

// out[perm[r]] = in[r] for internal rows (caller order), after a fill of out.
template <class TI, class TO>
__global__ void k_scatter(const TI* __restrict__ in, const int32_t* __restrict__ perm, int64_t n,
                          TO* __restrict__ out) {
    for (int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < n;
         r += int64_t(gridDim.x) * blockDim.x) {
        const int32_t j = perm[r];
        if (j >= 0) out[j] = TO(in[r]);
    }
}

// F over every caller voxel (eq. 9 + eq. 10); the last block writes *F_out.
// tau_ext: per-voxel threshold shifts in caller order (null: none).
// The class table (at most 256 records of 64 B) is copied to LDS first, so
// a voxel costs one round of independent loads (class index, dose, shift).
__device__ __forceinline__ void stage_classes(ObjClass* s_cl, const ObjClass* __restrict__ classes, int ncls) {
    for (int i = threadIdx.x; i < ncls; i += blockDim.x) s_cl[i] = classes[i];
    __syncthreads();
}

template <class T>
__global__ void __launch_bounds__(BLOCK) k_objective_ext(const T* __restrict__ d_ext,
                                                         const uint8_t* __restrict__ cls, int64_t V,
                                                         const ObjClass* __restrict__ classes, int ncls,
                                                         const double* __restrict__ tau_ext,
                                                         Rec* parts, Arrival* arr, double* F_out) {
    __shared__ ObjClass s_cl[MAX_CLASSES];
    stage_classes(s_cl, classes, ncls);
    Rec r = rec_identity();
    for (int64_t j = int64_t(blockIdx.x) * BLOCK + threadIdx.x; j < V; j += int64_t(gridDim.x) * BLOCK)
        r.s5 += obj_f(s_cl[cls[j]], double(d_ext[j]) - tau_at(tau_ext, j));
    Rec tot;
    const Rec mine = block_reduce(r);
    if (arrive_and_reduce(mine, parts, arr, &tot) && threadIdx.x == 0) *F_out = tot.s5;
}

// u[r] = dF/dz at the caller's dose of internal row r (0 on padding rows).
template <class T>
__global__ void k_gather_grad(const T* __restrict__ d_ext, const int32_t* __restrict__ perm,
                              const uint8_t* __restrict__ cls, int64_t Vpad,
                              const ObjClass* __restrict__ classes, const double* __restrict__ tau_int,
                              T* __restrict__ u) {
    for (int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < Vpad;
         r += int64_t(gridDim.x) * blockDim.x) {
        const int32_t j = perm[r];
        u[r] = j >= 0 ? T(grad_f(classes[cls[r]], double(d_ext[j]) - tau_at(tau_int, r))) : T(0);
    }
}

// u (ctx type) and optionally u64 (double) from the master dose d, plus
// F = F_const + sum f_j; the last block stores F in ms->F.
template <class T>
__global__ void __launch_bounds__(BLOCK) k_objective_int(const double* __restrict__ d,
                                                         const uint8_t* __restrict__ cls, int64_t Vpad,
                                                         const ObjClass* __restrict__ classes, int ncls,
                                                         T* __restrict__ u, double* __restrict__ u64,
                                                         Rec* parts, Arrival* arr, MasterState* ms) {
    __shared__ ObjClass s_cl[MAX_CLASSES];
    stage_classes(s_cl, classes, ncls);
    Rec r = rec_identity();
    for (int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x; i < Vpad;
         i += int64_t(gridDim.x) * BLOCK) {
        const ObjClass c = s_cl[cls[i]];
        const double z = d[i];
        const double gz = grad_f(c, z);
        u[i] = T(gz);
        if (u64) u64[i] = gz;
        r.s5 += obj_f(c, z);
    }
    Rec tot;
    const Rec mine = block_reduce(r);
    if (arrive_and_reduce(mine, parts, arr, &tot) && threadIdx.x == 0) ms->F = ms->F_const + tot.s5;
}

// Workgroups are handed to the 8 XCDs round-robin (workgroup b runs on XCD
// b mod 8), each XCD with its own L2.  xcd_block gives the workgroups of one
// XCD a contiguous range of [0, n): XCD x takes the x-th eighth.  A bijection
// of [0, n) for any n.
__device__ __forceinline__ int xcd_block(int b, int n) {
    constexpr int NX = 8;
    const int x = b % NX, k = b / NX;
    const int per = n / NX, rem = n % NX;   // XCD x runs per + (x < rem) workgroups
    return x * per + min(x, rem) + k;
}

// g_i = sum over beamlet i's entries of val * u[row]; one block per beamlet.
// Beamlets of one beam are adjacent and reach overlapping voxel rows, so
// each XCD takes a contiguous range of beamlets (xcd_block): its L2 then
// holds the u rows of a few beams instead of every XCD gathering all of u.
// GATED (the master's copy) runs only while a finished line search awaits
// its update (phase PH_UPD of an unfinished master), like k_update.  With a
// 16-bit value format the column sum is multiplied by the beamlet's scale.
template <class T, class UT, class Acc, class GT, bool GATED, bool LO = false, int PF = 4>
__global__ void __launch_bounds__(BLOCK) k_gradT(const int32_t* __restrict__ cptr,
                                                 const int32_t* __restrict__ crow,
                                                 const T* __restrict__ cval, const __half* __restrict__ clo,
                                                 const UT* __restrict__ u, GT* __restrict__ g,
                                                 const MasterState* gate, const float* __restrict__ scale) {
    if (GATED) {
        __shared__ int s_skip;
        if (threadIdx.x == 0) s_skip = (gate->done || gate->phase != PH_UPD);
        __syncthreads();
        if (s_skip) return;
    }
    const int i = xcd_block(blockIdx.x, gridDim.x);
    const int e0 = cptr[i], e1 = cptr[i + 1];
    Acc acc = Acc(0);
    int e = e0 + threadIdx.x;
    {
        // PF entries per thread in flight: rows and values, then the gathers
        // of u, then the products in entry order (the same sums).  Entries
        // past the column's end read its last entry (a valid address, no
        // branch around the load) and are left out of the sum, so the whole
        // batch is in flight at once
        for (; e < e1; e += PF * BLOCK) {
            int32_t r[PF];
            T v[PF];
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int ee = min(e + q * BLOCK, e1 - 1);
                r[q] = crow[ee];
                v[q] = cval[ee];
            }
            UT w[PF];
#pragma unroll
            for (int q = 0; q < PF; ++q) w[q] = u[r[q]];
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int ee = min(e + q * BLOCK, e1 - 1);
                const Acc term = Acc(dval2<T, LO>(v[q], clo + ee)) * Acc(w[q]);
                if (e + q * BLOCK < e1) acc += term;
            }
        }
    }
    for (; e < e1; e += BLOCK) acc += Acc(dval2<T, LO>(cval[e], clo + e)) * Acc(u[crow[e]]);
    acc = wave_sum(acc);
    __shared__ Acc s_w[BLOCK / WAVE];
    if ((threadIdx.x % WAVE) == 0) s_w[threadIdx.x / WAVE] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc t = Acc(0);
        for (int w = 0; w < BLOCK / WAVE; ++w) t += s_w[w];
        g[i] = GT(scale ? t * Acc(scale[i]) : t);
    }
}

// ---------------------------------------------------------------------------
// pricing: one wavefront per MLC row, last block picks the beam
// ---------------------------------------------------------------------------
struct RowRec {
    double v;        // best value (0 when closed)
    double second;   // best value among all other candidates
    int32_t L, R;
};

// the last block of k_price stages the row values and beam sums in LDS
// when they fit (otherwise it reads them from device memory)
constexpr int PRICE_ROWS_LDS = 4096;
constexpr int PRICE_BEAMS_LDS = 1024;

struct PriceGeom {
    const int32_t* row_start;
    const int32_t* row_len;
    const int32_t* beam_row0;
    int32_t R, B;
};

__global__ void __launch_bounds__(BLOCK) k_price(PriceGeom G, const double* __restrict__ g,
                                                 RowRec* __restrict__ rows, PriceResult* res,
                                                 Arrival* arr) {
    // prefix sums of each wave's row, accumulated sequentially so that a
    // beamlet priced exactly 0 leaves the prefix exactly unchanged (exact
    // ties such as leading or trailing zero-price beamlets stay ties)
    __shared__ double s_S[BLOCK / WAVE][WAVE + 1];
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int r = blockIdx.x * (BLOCK / WAVE) + wave;
    const bool have = r < G.R;
    const int n = have ? G.row_len[r] : 0;
    double* S = s_S[wave];
    // every lane loads its price (all loads in flight at once), then lane 0
    // forms the prefix sums in order from LDS
    S[lane + 1] = (have && lane < n) ? g[G.row_start[r] + lane] : 0.0;
    __syncthreads();
    if (lane == 0) {
        double acc = 0.0;
        S[0] = 0.0;
        for (int i = 0; i < WAVE; ++i) {
            if (i < n) acc += S[i + 1];
            S[i + 1] = acc;
        }
    }
    __syncthreads();
    if (have) {
        const double S1 = S[lane + 1];   // S_{i+1} = w_0 + ... + w_i
        const double S0 = S[lane];       // S_i
        // running maximum of S_0..S_i with the earliest index on ties
        double M = S0;
        int Mi = lane;
#pragma unroll
        for (int off = 1; off < WAVE; off <<= 1) {
            const double om = __shfl_up(M, off, WAVE);
            const int oi = __shfl_up(Mi, off, WAVE);
            if (lane >= off && !(M > om)) {
                M = om;
                Mi = oi;
            }
        }
        // best interval ending at right end i+1
        const bool valid = lane < n;
        const double c = valid ? S1 - M : INFINITY;
        // argmin over right ends, smallest right end on ties
        double bc = c;
        int bi = lane;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double oc = __shfl_xor(bc, off, WAVE);
            const int oi = __shfl_xor(bi, off, WAVE);
            if (oc < bc || (oc == bc && oi < bi)) {
                bc = oc;
                bi = oi;
            }
        }
        const bool open = bc < 0.0;
        const int Lb = __shfl(Mi, bi, WAVE);
        const int Rb = bi + 1;
        double second;
        if (!open) {
            second = wave_min(c);                 // every interval is a candidate
        } else {
            const double other_r = wave_min(lane == bi ? INFINITY : c);
            // runner-up left end for right end Rb: max S_l, l < Rb, l != Lb
            const double Sl = (lane < Rb && lane != Lb) ? S0 : -INFINITY;
            const double m2 = wave_max(Sl);
            const double SR = __shfl(S1, bi, WAVE);
            const double same_r = (m2 == -INFINITY) ? INFINITY : SR - m2;
            second = fmin(0.0, fmin(other_r, same_r));
        }
        if (lane == 0) {
            RowRec rr;
            rr.v = open ? bc : 0.0;
            rr.second = second;
            rr.L = open ? Lb : 0;
            rr.R = open ? Rb : 0;
            rows[r] = rr;
        }
    }
    // last block: per-beam sums (each beam's rows in order), the first
    // beam of smallest value, the smallest value among the other beams, and
    // the gap and leaves of the chosen beam's rows
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) s_last = arrive_last(arr);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    __shared__ double s_rv[PRICE_ROWS_LDS];    // row values
    __shared__ double s_bs[PRICE_BEAMS_LDS];   // beam sums
    __shared__ int s_best;
    __shared__ double s_bv, s_sv;
    const bool staged = G.R <= PRICE_ROWS_LDS && G.B <= PRICE_BEAMS_LDS;
    if (staged) {
        for (int rr = threadIdx.x; rr < G.R; rr += blockDim.x) s_rv[rr] = rows[rr].v;
        __syncthreads();
        for (int b = threadIdx.x; b < G.B; b += blockDim.x) {
            double sb = 0.0;
            for (int rr = G.beam_row0[b]; rr < G.beam_row0[b + 1]; ++rr) sb += s_rv[rr];
            s_bs[b] = sb;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int best = -1;
        double bv = INFINITY, sv = INFINITY;
        for (int b = 0; b < G.B; ++b) {
            double sb;
            if (staged) {
                sb = s_bs[b];
            } else {
                sb = 0.0;
                for (int rr = G.beam_row0[b]; rr < G.beam_row0[b + 1]; ++rr) sb += rows[rr].v;
            }
            if (best < 0 || sb < bv) {
                sv = bv;
                bv = sb;
                best = b;
            } else if (sb < sv) {
                sv = sb;
            }
        }
        s_best = best;
        s_bv = bv;
        s_sv = sv;
    }
    __syncthreads();
    // the chosen beam's rows, one per thread: leaves and the smallest row gap
    const int best = s_best;
    const int r0 = G.beam_row0[best], r1 = G.beam_row0[best + 1];
    double gap_t = INFINITY;
    for (int rr = r0 + int(threadIdx.x); rr < r1; rr += blockDim.x) {
        const RowRec x = rows[rr];
        gap_t = fmin(gap_t, x.second - x.v);
        res->leaves[2 * (rr - r0)] = int16_t(x.L);
        res->leaves[2 * (rr - r0) + 1] = int16_t(x.R);
    }
    __shared__ double s_gap[BLOCK / WAVE];
    gap_t = wave_min(gap_t);
    if (lane == 0) s_gap[wave] = gap_t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double gap = s_sv - s_bv;
        for (int w = 0; w < BLOCK / WAVE; ++w) gap = fmin(gap, s_gap[w]);
        res->beam = best;
        res->n_rows = r1 - r0;
        res->rc = s_bv;
        res->gap = gap;
    }
}

// ---------------------------------------------------------------------------
// gradient projection master (device-resident state machine)
//
// One step is the launch sequence
//   k_dir -> k_qstep -> k_lseval x slots -> k_update -> k_gradT.
// k_dir runs in PH_DIR (start of a solve) and PH_UPD (after an update); it
// sums the update's objective partials, tests KKT and builds the direction
// (-> PH_Q).  k_qstep and k_lseval evaluate the line search and decide in
// their last workgroup (-> PH_LS or, once final, PH_UPD).  k_update and
// k_gradT run in PH_UPD and leave the phase to the next k_dir.
// ---------------------------------------------------------------------------
struct PoolView {
    const int32_t* ap_beam;      // [Kmax]
    const int16_t* ap_lv;        // [Kmax * maxRB * 2]
    int32_t maxRB;
    const int32_t* blt_beam;     // [N]
    const int32_t* blt_row;      // [N]
    const int32_t* blt_pos;      // [N]
    const int32_t* beam_row0;    // [B + 1]
    const int32_t* row_start;    // [R]
    int32_t N;
};

// sum over the pool of v_k for apertures that open beamlet i (eq. 7), in
// pool order; `beam` and `lv` may point to LDS copies of the pool
__device__ __forceinline__ double pool_at_beamlet(const PoolView& P, int K, const int32_t* beam,
                                                  const int16_t* lv, const double* v, int i) {
    const int b = P.blt_beam[i];
    const int lr = P.blt_row[i] - P.beam_row0[b];
    const int pos = P.blt_pos[i];
    double acc = 0.0;
    for (int k = 0; k < K; ++k) {
        if (beam[k] != b) continue;
        const int16_t* l = lv + (size_t(k) * P.maxRB + lr) * 2;
        if (pos >= l[0] && pos < l[1]) acc += v[k];
    }
    return acc;
}

// x64[i] = sum over the pool of y_k for the apertures that open beamlet i
// (eq. 7), added in pool order.
__global__ void k_pool_x(PoolView P, int K, const double* __restrict__ y, double* __restrict__ x64) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P.N; i += gridDim.x * blockDim.x)
        x64[i] = pool_at_beamlet(P, K, P.ap_beam, P.ap_lv, y, i);
}

// Line-search history of a restored state (the first trial point of the
// next search is the step before the last).
__global__ void k_set_history(MasterState* ms, double last_step, double prev_step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ms->last_step = last_step;
        ms->prev_step = prev_step;
        ms->cg_valid = 0;
    }
}

// Direction step (single block of 1024 threads): objective of the last
// update, grad_y = A^T g, KKT test, projected direction p, longest feasible
// step t_max, dx = A p.  The pool and g are staged in LDS when they fit.
template <class T>
__global__ void __launch_bounds__(1024) k_dir(PoolView P, const T* __restrict__ g,
                                              double* __restrict__ y, double* __restrict__ p,
                                              double* __restrict__ grad, T* __restrict__ dx,
                                              MasterState* ms, CgMem* __restrict__ cgm,
                                              const Rec* __restrict__ upd_parts, int n_upd, bool stage) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_skip, s_go, s_upd, s_K;
    __shared__ double s_grad[MAX_APERTURES];
    __shared__ double s_p[MAX_APERTURES];
    __shared__ double s_y[MAX_APERTURES];
    __shared__ double s_r[MAX_APERTURES];
    __shared__ int32_t s_fr[MAX_APERTURES];
    __shared__ int32_t s_beam[MAX_APERTURES];
    __shared__ MasterState s_ms;
    ms_load(s_ms, ms);
    if (threadIdx.x == 0) {
        s_skip = s_ms.done || !(s_ms.phase == PH_DIR || s_ms.phase == PH_UPD);
        s_upd = s_ms.phase == PH_UPD;
        s_K = s_ms.K;
    }
    __syncthreads();
    if (s_skip) return;
    const int K = s_K;
    // objective after the update (fixed-order sum of the update's partials)
    if (s_upd) {
        Rec acc = rec_identity();
        const int per = (n_upd + blockDim.x - 1) / blockDim.x;
        const int b0 = threadIdx.x * per, b1 = min(n_upd, b0 + per);
        for (int b = b0; b < b1; ++b) acc.s5 += upd_parts[b].s5;
        const Rec t = block_reduce(acc);
        if (threadIdx.x == 0) s_ms.F = s_ms.F_const + t.s5;
    }
    // stage g and the pool
    T* gs_l = reinterpret_cast<T*>(smem);
    int16_t* lv_l = reinterpret_cast<int16_t*>(smem + ((size_t(P.N) * sizeof(T) + 15) & ~size_t(15)));
    const T* gs = g;
    const int16_t* lvs = P.ap_lv;
    if (stage) {
        for (int i = threadIdx.x; i < P.N; i += blockDim.x) gs_l[i] = g[i];
        const int nlv = K * P.maxRB * 2;
        for (int i = threadIdx.x; i < nlv; i += blockDim.x) lv_l[i] = P.ap_lv[i];
        gs = gs_l;
        lvs = lv_l;
    }
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        s_beam[k] = P.ap_beam[k];
        s_y[k] = y[k];
    }
    __syncthreads();
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
    const int nw = blockDim.x / WAVE;
    for (int k = wave; k < K; k += nw) {
        const int b = s_beam[k];
        const int r0 = P.beam_row0[b], nr = P.beam_row0[b + 1] - r0;
        double acc = 0.0;
        for (int lr = lane; lr < nr; lr += WAVE) {
            const int16_t* l = lvs + (size_t(k) * P.maxRB + lr) * 2;
            const int base = P.row_start[r0 + lr];
            double s = 0.0;
            for (int pos = l[0]; pos < l[1]; ++pos) s += double(gs[base + pos]);
            acc += s;
        }
        acc = wave_sum(acc);
        if (lane == 0) s_grad[k] = acc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double kkt = 0.0;
        for (int k = 0; k < K; ++k) kkt = fmax(kkt, fabs(fmin(s_y[k], s_grad[k])));
        s_ms.kkt = kkt;
        int go = 1;
        if (!(kkt > s_ms.tol)) {
            s_ms.stop_reason = 1;
            go = 0;
        } else if (s_ms.steps >= s_ms.max_steps) {
            s_ms.stop_reason = 2;
            go = 0;
        }
        double tmax = INFINITY, gp = 0.0;
        int any = 0;
        if (go) {
            // projected negative gradient r and free set; the conjugate
            // direction r + beta p_prev needs the last step's free set
            bool same = s_ms.conj && s_ms.cg_valid;
            for (int k = 0; k < K; ++k) {
                const bool fr = !(s_y[k] == 0.0 && s_grad[k] >= 0.0);
                s_r[k] = fr ? -s_grad[k] : 0.0;
                s_fr[k] = fr;
                if (fr != (cgm->free[k] != 0)) same = false;
                if (s_r[k] != 0.0) any = 1;
            }
            double beta = 0.0;
            if (same) {
                double num = 0.0, den = 0.0, gc = 0.0;
                for (int k = 0; k < K; ++k) {
                    num += s_r[k] * (s_r[k] - cgm->r[k]);
                    den += cgm->r[k] * cgm->r[k];
                }
                beta = den > 0.0 ? fmax(0.0, num / den) : 0.0;
                for (int k = 0; k < K; ++k) gc += s_grad[k] * (s_r[k] + beta * p[k]);
                if (!(gc < 0.0)) same = false;
            }
            for (int k = 0; k < K; ++k) s_p[k] = same ? s_r[k] + beta * p[k] : s_r[k];
            for (int k = 0; k < K; ++k) {
                const double pk = s_p[k];
                if (pk < 0.0) tmax = fmin(tmax, s_y[k] / (-pk));
                gp += s_grad[k] * pk;
            }
            if (!any) {
                s_ms.stop_reason = 3;
                go = 0;
            } else {
                for (int k = 0; k < K; ++k) {
                    p[k] = s_p[k];
                    grad[k] = s_grad[k];
                    cgm->r[k] = s_r[k];
                    cgm->free[k] = s_fr[k];
                }
            }
        }
        if (!go) {
            s_ms.done = 1;
            s_ms.phase = PH_DIR;
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
    __syncthreads();
    if (s_go) {
        for (int i = threadIdx.x; i < P.N; i += blockDim.x) dx[i] = T(pool_at_beamlet(P, K, s_beam, lvs, s_p, i));
        __syncthreads();
        if (threadIdx.x == 0) s_ms.phase = PH_Q;
    }
    ms_store(ms, s_ms);
}

// Line-search decision after an evaluation at m.t (on the MasterState or on
// any state with the same line-search fields).  Returns 1 when the step is
// final (m.t holds it), 0 when m.t holds the next trial point.
template <class S>
__device__ __forceinline__ int ls_decide(S& m, const Rec& e) {
    const double t = m.t, tmax = m.t_max;
    const double gphi = e.s0, s_r = 2.0 * e.s1, s_l = 2.0 * e.s2, nb = e.mn, pb = e.mx;
    m.ls_iter += 1;
    m.total_ls += 1;
    int fin = 0;
    double tf = 0.0, nxt = 0.0;
    if (gphi == 0.0) {
        fin = 1;
        tf = t;
    } else if (gphi < 0.0) {
        if (t >= tmax) {
            fin = 1;
            tf = tmax;
        } else {
            m.lo = t;
            const double tn = s_r > 0.0 ? t - gphi / s_r : INFINITY;
            if (tn <= nb) {
                fin = 1;
                tf = fmin(tn, tmax);
            } else if (nb >= tmax) {
                fin = 1;
                tf = tmax;
            } else {
                if (tn < m.hi)
                    nxt = tn;
                else if (!m.hi_known)
                    nxt = m.hi;
                else
                    nxt = 0.5 * (m.lo + m.hi);
                if (isinf(nxt)) nxt = nb;
            }
        }
    } else {
        m.hi = t;
        m.hi_known = 1;
        const double tn = s_l > 0.0 ? t - gphi / s_l : -INFINITY;
        if (tn >= pb) {
            fin = 1;
            tf = fmax(tn, m.lo);
        } else {
            nxt = tn > m.lo ? tn : 0.5 * (m.lo + m.hi);
        }
    }
    if (!fin && m.ls_iter >= LS_MAX_ITER) {
        fin = 1;
        tf = m.lo;
    }
    m.t = fin ? tf : nxt;
    return fin;
}

// Final step of a line search (all threads of the last block): y update with
// exact zeros for blocking apertures, step count, refresh of x = A y.
__device__ __forceinline__ void finish_step(const PoolView& P, MasterState& m, double* y,
                                            const double* p, double* x64, int fin) {
    __shared__ int s_refresh;
    __shared__ double s_y[MAX_APERTURES];
    if (!fin) return;
    const int K = m.K;
    const double t = m.t, tmax = m.t_max;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const double pk = p[k];
        const double ratio = pk < 0.0 ? y[k] / (-pk) : INFINITY;
        double yn = y[k] + t * pk;
        if (t == tmax && ratio == t) yn = 0.0;
        yn = fmax(yn, 0.0);
        y[k] = yn;
        s_y[k] = yn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        m.steps += 1;
        m.total_steps += 1;
        m.prev_step = m.last_step;
        m.last_step = t;
        m.refresh = (m.steps % m.refresh_every) == 0;
        // a step that blocks ends the conjugate sequence
        m.cg_valid = m.conj && !(t == tmax);
        m.cg_K = K;
        s_refresh = m.refresh;
    }
    __syncthreads();
    if (s_refresh)
        for (int i = threadIdx.x; i < P.N; i += blockDim.x)
            x64[i] = pool_at_beamlet(P, K, P.ap_beam, P.ap_lv, s_y, i);
    __syncthreads();
    if (threadIdx.x == 0) m.phase = PH_UPD;
}

// q = D dx and the first line-search evaluation (slab layout).
template <class T>
__global__ void __launch_bounds__(SLAB_THREADS) k_qstep(SellView<T> S, int64_t Vpad, const T* __restrict__ dx,
                                                        int N, bool stage, const double* __restrict__ d,
                                                        const uint8_t* __restrict__ cls,
                                                        const ObjClass* __restrict__ classes, int ncls,
                                                        T* __restrict__ q, Rec* parts, Arrival* arr,
                                                        MasterState* ms, PoolView P, double* y,
                                                        const double* p, double* x64) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_skip;
    __shared__ double s_t;
    __shared__ T s_part[KSPLIT * SLAB];
    if (threadIdx.x == 0) {
        s_skip = (ms->done || ms->phase != PH_Q);
        s_t = ms->t;
    }
    __syncthreads();
    if (s_skip) return;
    ObjClass* cl = reinterpret_cast<ObjClass*>(smem);
    for (int i = threadIdx.x; i < ncls; i += blockDim.x) cl[i] = classes[i];
    T* xs_l = reinterpret_cast<T*>(smem + sizeof(ObjClass) * ncls);
    __syncthreads();
    const T sum = slab_rows_x<T, T, T>(S, dx, N, xs_l, stage, nullptr, s_part);
    Rec r = rec_identity();
    const int64_t row = int64_t(blockIdx.x) * SLAB + threadIdx.x;
    if (threadIdx.x < SLAB && row < Vpad) {
        q[row] = sum;
        ls_voxel(cl[cls[row]], d[row], double(sum), s_t, r);
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
    finish_step(P, s_ms, y, p, x64, s_fin);
    ms_store(ms, s_ms);
}

// Further line-search evaluations at ms->t.
__global__ void __launch_bounds__(BLOCK) k_lseval(const double* __restrict__ d, const void* qv,
                                                  int q_is_f64, const uint8_t* __restrict__ cls,
                                                  int64_t Vpad, const ObjClass* __restrict__ classes,
                                                  int ncls, Rec* parts, Arrival* arr, MasterState* ms,
                                                  PoolView P, double* y, const double* p, double* x64) {
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
    const double t = s_t;
    Rec r = rec_identity();
    if (q_is_f64) {
        const double* q = static_cast<const double*>(qv);
        for (int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x; i < Vpad; i += int64_t(gridDim.x) * BLOCK)
            ls_voxel(cl[cls[i]], d[i], q[i], t, r);
    } else {
        const float* q = static_cast<const float*>(qv);
        for (int64_t i = int64_t(blockIdx.x) * BLOCK + threadIdx.x; i < Vpad; i += int64_t(gridDim.x) * BLOCK)
            ls_voxel(cl[cls[i]], d[i], double(q[i]), t, r);
    }
    Rec tot;
    const Rec mine = block_reduce(r);
    if (!arrive_and_reduce(mine, parts, arr, &tot)) return;
    __shared__ MasterState s_ms;
    __shared__ int s_fin;
    ms_load(s_ms, ms);
    if (threadIdx.x == 0) s_fin = ls_decide(s_ms, tot);
    __syncthreads();
    finish_step(P, s_ms, y, p, x64, s_fin);
    ms_store(ms, s_ms);
}

// Update (slab layout): d += t q (or d = D x64 on refresh steps),
// u = grad F(d), per-block objective partials for the next k_dir.
template <class T>
__global__ void __launch_bounds__(SLAB_THREADS) k_update(SellView<T> S, int64_t Vpad,
                                                         const double* __restrict__ x64, int N, bool stage,
                                                         double* __restrict__ d, const T* __restrict__ q,
                                                         const uint8_t* __restrict__ cls,
                                                         const ObjClass* __restrict__ classes, int ncls,
                                                         const double* __restrict__ tau,
                                                         T* __restrict__ u, Rec* upd_parts,
                                                         const MasterState* ms) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_skip, s_refresh;
    __shared__ double s_t;
    __shared__ double s_part[KSPLIT * SLAB];
    if (threadIdx.x == 0) {
        s_skip = (ms->done || ms->phase != PH_UPD);
        s_refresh = ms->refresh;
        s_t = ms->t;
    }
    __syncthreads();
    if (s_skip) return;
    ObjClass* cl = reinterpret_cast<ObjClass*>(smem);
    for (int i = threadIdx.x; i < ncls; i += blockDim.x) cl[i] = classes[i];
    double* xs_l = reinterpret_cast<double*>(smem + sizeof(ObjClass) * ncls);
    __syncthreads();
    double dn = 0.0;
    if (s_refresh) {
        dn = slab_rows_x<T, double, double>(S, x64, N, xs_l, stage, nullptr, s_part);
    }
    Rec r = rec_identity();
    const int64_t row = int64_t(blockIdx.x) * SLAB + threadIdx.x;
    if (threadIdx.x < SLAB && row < Vpad) {
        dn = s_refresh ? dn - tau_at(tau, row) : d[row] + s_t * double(q[row]);
        d[row] = dn;
        const ObjClass c = cl[cls[row]];
        u[row] = T(grad_f(c, dn));
        r.s5 = obj_f(c, dn);
    }
    const Rec mine = block_reduce(r);
    if (threadIdx.x == 0) upd_parts[blockIdx.x] = mine;
}

// Reset the master state machine for a new solve over a pool of K.
__global__ void k_master_init(MasterState* ms, int K, double tol, int max_steps) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ms->phase = PH_DIR;
        ms->done = 0;
        ms->steps = 0;
        ms->max_steps = max_steps;
        ms->K = K;
        ms->tol = tol;
        ms->stop_reason = 0;
        ms->ls_iter = 0;
        ms->refresh = 0;
        if (ms->cg_K != K) ms->cg_valid = 0;   // the pool changed since the last step
    }
}

// Append the last pricing result to the pool as aperture k with y_k = 0.
__global__ void k_add_from_price(const PriceResult* res, int k, int maxRB, int32_t* ap_beam,
                                 int16_t* ap_lv, double* y) {
    const int n = res->n_rows;
    for (int i = threadIdx.x; i < maxRB; i += blockDim.x) {
        ap_lv[(size_t(k) * maxRB + i) * 2] = i < n ? res->leaves[2 * i] : int16_t(0);
        ap_lv[(size_t(k) * maxRB + i) * 2 + 1] = i < n ? res->leaves[2 * i + 1] : int16_t(0);
    }
    if (threadIdx.x == 0) {
        ap_beam[k] = res->beam;
        y[k] = 0.0;
    }
}

}  // namespace dao
