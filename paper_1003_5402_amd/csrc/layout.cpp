// Host-side validation and layout construction (see layout.h).
#include "layout.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <queue>
#include <set>
#include <sstream>

namespace dao {

namespace {

constexpr int64_t SORT_WINDOW = 1024;   // rows sorted by length within windows of this size

template <class... A>
std::string cat(A&&... a) {
    std::ostringstream s;
    (s << ... << a);
    return s.str();
}

}  // namespace

namespace {
// RNE of |r| to a binary format with `mant` stored mantissa bits, exponent
// bias `bias` and `ebits` exponent bits; returns the magnitude bits.  Works
// on the IEEE bits of the double: the significand m (53 bits with the
// implicit one) is shifted right to the target's units, 2^(E - mant) for a
// normal result and 2^(1 - bias - mant) below the normal range, and the
// dropped bits round it to nearest, ties to an even result.
uint16_t enc_mag(double a, int mant, int bias, int ebits) {
    const int emax_field = (1 << ebits) - 1;   // all ones: infinity
    if (a == 0.0) return 0;
    if (std::isinf(a)) return uint16_t(emax_field << mant);
    uint64_t bits;
    std::memcpy(&bits, &a, sizeof bits);
    const int ef = int((bits >> 52) & 0x7FF);
    if (ef == 0) return 0;   // a subnormal double is far below half the smallest 16-bit unit
    const uint64_t m = (bits & ((uint64_t(1) << 52) - 1)) | (uint64_t(1) << 52);
    int E = ef - 1023;   // a = m 2^(E - 52)
    const bool normal = E >= 1 - bias;
    const int shift = (52 - mant) + (normal ? 0 : (1 - bias - E));
    if (shift >= 54) return 0;   // a < half a unit (m < 2^53)
    uint64_t q = m >> shift;
    const uint64_t rem = m & ((uint64_t(1) << shift) - 1), half = uint64_t(1) << (shift - 1);
    if (rem > half || (rem == half && (q & 1))) ++q;
    if (!normal) return uint16_t(q);   // 2^mant units is the smallest normal, encoded the same way
    if (q == (uint64_t(1) << (mant + 1))) {   // rounded up to the next binade
        E += 1;
        q = uint64_t(1) << mant;
    }
    if (E + bias >= emax_field) return uint16_t(emax_field << mant);
    return uint16_t(((E + bias) << mant) | int(q - (uint64_t(1) << mant)));
}
double dec_mag(uint16_t h, int mant, int bias, int ebits) {
    const int ef = (h >> mant) & ((1 << ebits) - 1), m = h & ((1 << mant) - 1);
    if (ef == (1 << ebits) - 1) return m ? NAN : INFINITY;
    if (ef == 0) return std::ldexp(double(m), 1 - bias - mant);
    return std::ldexp(double((1 << mant) + m), ef - bias - mant);
}
}  // namespace

uint16_t enc_f16(double r) {
    const uint16_t s = std::signbit(r) ? 0x8000 : 0;
    return uint16_t(s | enc_mag(std::fabs(r), 10, 15, 5));
}
uint16_t enc_bf16(double r) {
    const uint16_t s = std::signbit(r) ? 0x8000 : 0;
    return uint16_t(s | enc_mag(std::fabs(r), 7, 127, 8));
}
double dec_f16(uint16_t h) {
    const double v = dec_mag(uint16_t(h & 0x7FFF), 10, 15, 5);
    return (h & 0x8000) ? -v : v;
}
double dec_bf16(uint16_t h) {
    const double v = dec_mag(uint16_t(h & 0x7FFF), 7, 127, 8);
    return (h & 0x8000) ? -v : v;
}
void encode_value(int fmt, double r, uint16_t* hi, uint16_t* lo) {
    const uint16_t h = fmt == DAO_DFMT_BF16 ? enc_bf16(r) : enc_f16(r);
    *hi = h;
    if (lo) *lo = enc_f16(r - (fmt == DAO_DFMT_BF16 ? dec_bf16(h) : dec_f16(h)));
}

dao_status validate_inputs(const dao_matrix* D, const dao_beams* beams,
                           const dao_structures* structs, const dao_prescription* presc,
                           const dao_options* opt, std::string* err) {
    auto fail = [&](std::string m) { *err = std::move(m); return DAO_EINVAL; };
    if (!D || !beams || !structs || !opt || !err) return fail("null argument");
    if (D->n_vox <= 0 || D->n_blt <= 0 || D->nnz < 0) return fail("n_vox and n_blt must be positive, nnz >= 0");
    if (D->n_blt > 65535) return fail("n_blt above 65535 is not supported (16-bit column indices)");
    if (D->nnz >= (int64_t(1) << 31)) return fail("nnz must be below 2^31");
    if (D->n_vox >= (int64_t(1) << 31)) return fail("n_vox must be below 2^31");
    if (!D->row_ptr || (D->nnz > 0 && (!D->col || !D->val))) return fail("null CSR array");
    if (opt->dtype != DAO_F64 && opt->dtype != DAO_F32) return fail("dtype must be DAO_F64 or DAO_F32");
    if (opt->max_apertures < 1 || opt->max_apertures > MAX_APERTURES) return fail("max_apertures must be in [1, 256]");
    if (!(opt->eps > 0) || !std::isfinite(opt->eps)) return fail("eps must be positive");
    if (opt->max_steps < 1) return fail("max_steps must be >= 1");
    if (!(opt->tau_rel >= 0) || !std::isfinite(opt->tau_rel)) return fail("tau_rel must be >= 0");
    if (opt->max_tighten < 0) return fail("max_tighten must be >= 0");
    if (opt->refresh_every < 1) return fail("refresh_every must be >= 1");
    if (opt->ls_slots < 1 || opt->ls_slots > 16) return fail("ls_slots must be in [1, 16]");
    if (opt->mem_cap_bytes < 0) return fail("mem_cap_bytes must be >= 0");
    if (opt->master != DAO_MASTER_APERTURE && opt->master != DAO_MASTER_BEAMLET)
        return fail("master must be DAO_MASTER_APERTURE or DAO_MASTER_BEAMLET");
    if (opt->persistent < 0 || opt->persistent > 2) return fail("persistent must be 0, 1 or 2");
    if (opt->product_tune < 0 || opt->product_tune > 1) return fail("product_tune must be 0 or 1");
    if (opt->dose_variant < 0 || opt->dose_variant > 8) return fail("dose_variant must be in [0, 8]");
    if (opt->dose_variant == 2 && opt->d_format != DAO_DFMT_NATIVE)
        return fail("dose_variant 2 reads x unscaled: native d_format only");
    if (opt->gradient_depth != 4 && opt->gradient_depth != 8 && opt->gradient_depth != 16)
        return fail("gradient_depth must be 4, 8 or 16");
    if (opt->direction != DAO_DIR_STEEPEST && opt->direction != DAO_DIR_CONJUGATE)
        return fail("direction must be DAO_DIR_STEEPEST or DAO_DIR_CONJUGATE");
    if (opt->apertures_per_round < 1 || opt->apertures_per_round > 16)
        return fail("apertures_per_round must be in [1, 16]");
    if (opt->dk_format != DAO_DFMT_NATIVE && opt->dk_format != DAO_DFMT_F16 && opt->dk_format != DAO_DFMT_AUTO)
        return fail("dk_format must be DAO_DFMT_NATIVE, DAO_DFMT_F16 or DAO_DFMT_AUTO");
    if (opt->dk_format == DAO_DFMT_F16 && (opt->dtype != DAO_F32 || opt->master != DAO_MASTER_APERTURE))
        return fail("an FP16 aperture dose matrix needs dtype DAO_F32 and the aperture-matrix master");
    if (opt->d_format < DAO_DFMT_NATIVE || opt->d_format > DAO_DFMT_BF16)
        return fail("d_format must be DAO_DFMT_NATIVE, DAO_DFMT_F16 or DAO_DFMT_BF16");
    if (opt->d_residual < 0 || opt->d_residual > 2) return fail("d_residual must be 0, 1 or 2");
    if (opt->residual_rounds < 0) return fail("residual_rounds must be >= 0");
    if (opt->graphs < 0 || opt->graphs > 1) return fail("graphs must be 0 or 1");
    if (opt->d_format != DAO_DFMT_NATIVE) {
        if (opt->dtype != DAO_F32) return fail("a 16-bit d_format needs dtype DAO_F32");
        if (opt->master != DAO_MASTER_APERTURE) return fail("a 16-bit d_format needs the aperture-matrix master");
        if (D->n_blt > 12288) return fail("a 16-bit d_format needs n_blt <= 12288 (x staged on chip)");
    } else if (opt->d_residual) {
        return fail("d_residual needs a 16-bit d_format");
    }
    if (opt->master == DAO_MASTER_APERTURE && opt->max_apertures > KS)
        return fail("the aperture-matrix master holds at most 64 apertures (max_apertures)");

    const int64_t* rp = D->row_ptr;
    if (rp[0] != 0) return fail("row_ptr[0] must be 0");
    for (int64_t r = 0; r < D->n_vox; ++r) {
        if (rp[r + 1] < rp[r]) return fail(cat("row_ptr decreases at row ", r));
    }
    if (rp[D->n_vox] != D->nnz) return fail("row_ptr[n_vox] must equal nnz");
    for (int64_t r = 0; r < D->n_vox; ++r) {
        int32_t prev = -1;
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
            int32_t c = D->col[e];
            if (c < 0 || c >= D->n_blt) return fail(cat("column index out of range at entry ", e));
            if (c <= prev) return fail(cat("columns not strictly increasing in row ", r));
            prev = c;
            double v = D->val[e];
            if (!std::isfinite(v) || v < 0) return fail(cat("non-finite or negative value at entry ", e));
        }
    }

    if (beams->n_beams < 1 || !beams->rows_per_beam || !beams->row_len) return fail("beams: empty or null");
    int64_t R = 0;
    for (int b = 0; b < beams->n_beams; ++b) {
        if (beams->rows_per_beam[b] < 1 || beams->rows_per_beam[b] > 1024)
            return fail(cat("rows_per_beam[", b, "] must be in [1, 1024]"));
        R += beams->rows_per_beam[b];
    }
    int64_t Nsum = 0;
    for (int64_t r = 0; r < R; ++r) {
        if (beams->row_len[r] < 1 || beams->row_len[r] > MAX_ROW_LEN)
            return fail(cat("row_len[", r, "] must be in [1, 64]"));
        Nsum += beams->row_len[r];
    }
    if (Nsum != D->n_blt) return fail("sum of row_len must equal n_blt");

    if (structs->n_struct < 0 || structs->n_struct > 255) return fail("n_struct must be in [0, 255]");
    if (structs->n_struct > 0 && !presc) return fail("null prescriptions");
    if (!structs->vox_struct) return fail("null vox_struct");
    for (int64_t j = 0; j < D->n_vox; ++j) {
        int s = structs->vox_struct[j];
        if (s < -1 || s >= structs->n_struct) return fail(cat("structure id out of range at voxel ", j));
    }
    if (structs->vox_struct2) {
        std::set<std::pair<int, int>> pairs;
        for (int64_t j = 0; j < D->n_vox; ++j) {
            const int s2 = structs->vox_struct2[j];
            if (s2 < -1 || s2 >= structs->n_struct) return fail(cat("second structure id out of range at voxel ", j));
            if (s2 < 0) continue;
            const int s1 = structs->vox_struct[j];
            if (s1 < 0) return fail(cat("voxel ", j, " has a second structure but no first"));
            if (s1 == s2) return fail(cat("voxel ", j, " lists the same structure twice"));
            pairs.insert({s1, s2});
        }
        if (int64_t(structs->n_struct) + 1 + int64_t(pairs.size()) > MAX_CLASSES)
            return fail("more than 255 distinct structures and structure pairs");
    }
    if (structs->vox_shift) {
        for (int64_t j = 0; j < D->n_vox; ++j)
            if (!std::isfinite(structs->vox_shift[j])) return fail(cat("non-finite threshold shift at voxel ", j));
    }
    for (int s = 0; s < structs->n_struct; ++s) {
        const dao_prescription& p = presc[s];
        if (!std::isfinite(p.t_under) || !std::isfinite(p.t_over) || !std::isfinite(p.w_under) ||
            !std::isfinite(p.w_over))
            return fail(cat("non-finite prescription for structure ", s));
        if (p.w_under < 0 || p.w_over < 0) return fail(cat("negative weight for structure ", s));
        if (p.is_target && p.t_under > p.t_over) return fail(cat("target ", s, " has t_under > t_over"));
    }
    return DAO_OK;
}

void build_layout(const dao_matrix* D, const dao_beams* beams, const dao_structures* structs,
                  const dao_prescription* presc, HostLayout* L) {
    const int64_t V = D->n_vox, N = D->n_blt;
    const int64_t* rp = D->row_ptr;
    L->V = V;
    L->N = N;
    L->nnz = D->nnz;
    L->n_struct = structs->n_struct;

    // --- objective classes (eq. 9 and eq. 10) ------------------------------
    // |v_s| counts the voxels carrying s as first or second label; pairs of
    // overlapping structures get classes of their own after "none"
    const int ns = structs->n_struct;
    const int16_t* l1 = structs->vox_struct;
    const int16_t* l2 = structs->vox_struct2;
    std::vector<int64_t> size(ns, 0);
    for (int64_t j = 0; j < V; ++j) {
        if (l1[j] >= 0) size[l1[j]]++;
        if (l2 && l2[j] >= 0) size[l2[j]]++;
    }
    // the terms of structure s: (a, T-, b, T+), zero weights when empty
    auto terms = [&](int st, double* a, double* tu, double* b, double* to) {
        *a = *tu = *b = *to = 0.0;
        if (st < 0 || size[st] == 0) return;
        const dao_prescription& p = presc[st];
        if (p.is_target) {
            *a = p.w_under / double(size[st]);
            *tu = p.t_under;
        }
        *b = p.w_over / double(size[st]);
        *to = p.t_over;
    };
    const ObjClass zero{0, 0, 0, 0, 0, 0, 0, 0};
    L->classes.assign(ns + 1, zero);
    for (int st = 0; st < ns; ++st) {
        ObjClass& c = L->classes[st];
        terms(st, &c.a, &c.t_under, &c.b, &c.t_over);
    }
    const uint8_t none = uint8_t(ns);
    L->cls_ext.resize(V);
    std::map<std::pair<int, int>, int> pair_class;
    for (int64_t j = 0; j < V; ++j) {
        int cl = l1[j] < 0 ? int(none) : int(l1[j]);
        if (l2 && l2[j] >= 0) {
            const auto key = std::make_pair(int(l1[j]), int(l2[j]));
            auto it = pair_class.find(key);
            if (it == pair_class.end()) {
                ObjClass c = zero;
                terms(key.first, &c.a, &c.t_under, &c.b, &c.t_over);
                terms(key.second, &c.a2, &c.t_under2, &c.b2, &c.t_over2);
                it = pair_class.emplace(key, int(L->classes.size())).first;
                L->classes.push_back(c);
            }
            cl = it->second;
        }
        L->cls_ext[j] = uint8_t(cl);
    }

    // --- internal row order: non-empty rows, sorted by length (descending)
    //     inside windows so that slices carry little padding ---------------
    std::vector<int32_t> rows;
    rows.reserve(V);
    for (int64_t j = 0; j < V; ++j)
        if (rp[j + 1] > rp[j]) rows.push_back(int32_t(j));
    L->Vnz = int64_t(rows.size());
    for (size_t w0 = 0; w0 < rows.size(); w0 += SORT_WINDOW) {
        size_t w1 = std::min(rows.size(), w0 + size_t(SORT_WINDOW));
        std::stable_sort(rows.begin() + w0, rows.begin() + w1, [&](int32_t a, int32_t b) {
            return (rp[a + 1] - rp[a]) > (rp[b + 1] - rp[b]);
        });
    }
    L->nslices = (L->Vnz + SLICE - 1) / SLICE;
    L->Vpad = L->nslices * SLICE;
    L->perm.assign(L->Vpad, -1);
    std::copy(rows.begin(), rows.end(), L->perm.begin());
    std::vector<int32_t> inv(V, -1);
    for (int64_t r = 0; r < L->Vnz; ++r) inv[L->perm[r]] = int32_t(r);

    L->cls_int.assign(L->Vpad, none);
    for (int64_t r = 0; r < L->Vnz; ++r) L->cls_int[r] = L->cls_ext[L->perm[r]];

    // per-voxel threshold shifts: caller order and internal row order
    // (padding rows 0)
    if (structs->vox_shift) {
        L->tau_ext.assign(structs->vox_shift, structs->vox_shift + V);
        L->tau_int.assign(L->Vpad, 0.0);
        for (int64_t r = 0; r < L->Vnz; ++r) L->tau_int[r] = structs->vox_shift[L->perm[r]];
    }

    // objective of voxels that no beamlet reaches (their dose is always 0;
    // with shifted thresholds the terms see 0 - tau_j against unshifted ones)
    {
        double acc = 0.0;
        for (int64_t j = 0; j < V; ++j) {
            if (rp[j + 1] > rp[j]) continue;
            const ObjClass& c = L->classes[L->cls_ext[j]];
            const double z = structs->vox_shift ? -structs->vox_shift[j] : 0.0;
            const double un = std::max(0.0, c.t_under - z), ov = std::max(0.0, z - c.t_over);
            const double un2 = std::max(0.0, c.t_under2 - z), ov2 = std::max(0.0, z - c.t_over2);
            acc += c.a * un * un + c.b * ov * ov + c.a2 * un2 * un2 + c.b2 * ov2 * ov2;
        }
        L->F_const = acc;
    }

    // --- sliced ELL ------------------------------------------------------
    L->slice_ptr.assign(L->nslices + 1, 0);
    L->slice_w.assign(L->nslices, 0);
    for (int64_t s = 0; s < L->nslices; ++s) {
        int64_t w = 0;
        for (int l = 0; l < SLICE; ++l) {
            int32_t j = L->perm[s * SLICE + l];
            if (j >= 0) w = std::max<int64_t>(w, rp[j + 1] - rp[j]);
        }
        w = (w + 3) / 4 * 4;   // groups of 4 entries per row
        L->slice_w[s] = int32_t(w);
        L->slice_ptr[s + 1] = L->slice_ptr[s] + uint32_t(w * SLICE);
    }
    const uint32_t total = L->slice_ptr[L->nslices];
    L->sell_col.assign(total, 0);
    L->sell_val.assign(total, 0.0);
    for (int64_t s = 0; s < L->nslices; ++s) {
        for (int l = 0; l < SLICE; ++l) {
            int32_t j = L->perm[s * SLICE + l];
            if (j < 0) continue;
            int64_t len = rp[j + 1] - rp[j];
            for (int64_t k = 0; k < len; ++k) {
                uint32_t e = L->slice_ptr[s] + uint32_t((k / 4) * 4 * SLICE + 4 * l + k % 4);
                L->sell_col[e] = uint16_t(D->col[rp[j] + k]);
                L->sell_val[e] = D->val[rp[j] + k];
            }
        }
    }

    // --- beamlet-major copy over internal row numbers ----------------------
    L->csc_ptr.assign(N + 1, 0);
    for (int64_t e = 0; e < D->nnz; ++e) L->csc_ptr[D->col[e] + 1]++;
    for (int64_t i = 0; i < N; ++i) L->csc_ptr[i + 1] += L->csc_ptr[i];
    L->csc_row.assign(D->nnz, 0);
    L->csc_val.assign(D->nnz, 0.0);
    {
        std::vector<int32_t> fill(L->csc_ptr.begin(), L->csc_ptr.end() - 1);
        for (int64_t r = 0; r < L->Vnz; ++r) {          // internal order: rows ascending
            int32_t j = L->perm[r];
            for (int64_t e = rp[j]; e < rp[j + 1]; ++e) {
                int32_t c = D->col[e];
                L->csc_row[fill[c]] = int32_t(r);
                L->csc_val[fill[c]] = D->val[e];
                fill[c]++;
            }
        }
    }

    // per-beamlet scale of the 16-bit value formats: the column maximum
    L->col_scale.assign(N, 1.0f);
    for (int64_t i = 0; i < N; ++i) {
        double mx = 0.0;
        for (int32_t e = L->csc_ptr[i]; e < L->csc_ptr[i + 1]; ++e) mx = std::max(mx, L->csc_val[e]);
        if (mx > 0.0) L->col_scale[i] = float(mx);
    }

    // --- MLC geometry -----------------------------------------------------
    L->B = beams->n_beams;
    L->beam_row0.assign(L->B + 1, 0);
    for (int b = 0; b < L->B; ++b) {
        L->beam_row0[b + 1] = L->beam_row0[b] + beams->rows_per_beam[b];
        L->max_rows_per_beam = std::max(L->max_rows_per_beam, beams->rows_per_beam[b]);
    }
    L->R = L->beam_row0[L->B];
    L->row_start.assign(L->R, 0);
    L->row_len.assign(beams->row_len, beams->row_len + L->R);
    L->blt_beam.assign(N, 0);
    L->blt_row.assign(N, 0);
    L->blt_pos.assign(N, 0);
    int32_t i = 0;
    for (int b = 0; b < L->B; ++b) {
        for (int r = L->beam_row0[b]; r < L->beam_row0[b + 1]; ++r) {
            L->row_start[r] = i;
            for (int p = 0; p < L->row_len[r]; ++p, ++i) {
                L->blt_beam[i] = b;
                L->blt_row[i] = r;
                L->blt_pos[i] = p;
            }
        }
    }
}

void balanced_slice_order(const std::vector<int32_t>& slice_w, int64_t nwaves, std::vector<int32_t>& order,
                          int& rounds) {
    const int64_t ns = int64_t(slice_w.size());
    std::vector<int32_t> idx(static_cast<size_t>(ns));
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return slice_w[a] > slice_w[b]; });
    using Item = std::pair<int64_t, int64_t>;   // (work so far, wavefront)
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    for (int64_t g = 0; g < nwaves; ++g) heap.push({0, g});
    std::vector<std::vector<int32_t>> lists(size_t(nwaves > 0 ? nwaves : 0));
    for (int32_t sl : idx) {
        Item it = heap.top();
        heap.pop();
        lists[size_t(it.second)].push_back(sl);
        it.first += int64_t(slice_w[size_t(sl)]) + 4;
        heap.push(it);
    }
    rounds = 0;
    for (auto& l : lists) {
        std::sort(l.begin(), l.end());
        rounds = std::max(rounds, int(l.size()));
    }
    order.assign(size_t(rounds) * size_t(nwaves > 0 ? nwaves : 0), -1);
    for (int64_t g = 0; g < nwaves; ++g)
        for (size_t k = 0; k < lists[size_t(g)].size(); ++k) order[k * size_t(nwaves) + size_t(g)] = lists[size_t(g)][k];
}

}  // namespace dao
