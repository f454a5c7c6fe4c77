// Host-side checks of the library's input validation and layout construction,
// built by tests/test_host_sanitized.py with AddressSanitizer and
// UndefinedBehaviorSanitizer (g++, no HIP): every array the layout builder
// writes is read back here, so an out-of-bounds or uninitialised access in
// it, or undefined arithmetic, ends the run.
//
// Input file (little endian): int64 V, N, nnz, B, n_struct; int64 row_ptr[V+1];
// int32 col[nnz]; double val[nnz]; int32 rows_per_beam[B]; int32 row_len[R];
// int16 vox_struct[V]; per structure int32 is_target and 4 doubles
// (t_under, t_over, w_under, w_over).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "layout.h"

using namespace dao;

namespace {

template <class T>
std::vector<T> read_vec(FILE* f, int64_t n) {
    std::vector<T> v(size_t(n > 0 ? n : 0));
    if (n > 0 && std::fread(v.data(), sizeof(T), size_t(n), f) != size_t(n)) {
        std::fprintf(stderr, "short read\n");
        std::exit(2);
    }
    return v;
}

int64_t read_i64(FILE* f) { return read_vec<int64_t>(f, 1)[0]; }

int failures = 0;
void expect(bool ok, const std::string& what) {
    if (!ok) {
        std::fprintf(stderr, "FAIL: %s\n", what.c_str());
        ++failures;
    }
}

struct Problem {
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    std::vector<int32_t> rows_per_beam, row_len;
    std::vector<int16_t> vox_struct;
    std::vector<dao_prescription> presc;
    int64_t V = 0, N = 0, nnz = 0;

    dao_matrix m() const { return dao_matrix{V, N, nnz, row_ptr.data(), col.data(), val.data()}; }
    dao_beams b() const {
        return dao_beams{int32_t(rows_per_beam.size()), rows_per_beam.data(), row_len.data()};
    }
    dao_structures s() const { return dao_structures{int32_t(presc.size()), vox_struct.data()}; }
};

dao_status validate(const Problem& p, const dao_options& o) {
    std::string err;
    const dao_matrix M = p.m();
    const dao_beams Bm = p.b();
    const dao_structures S = p.s();
    return validate_inputs(&M, &Bm, &S, p.presc.data(), &o, &err);
}

}  // namespace

int main(int argc, char** argv) {
    if (argc != 2) {
        std::fprintf(stderr, "usage: %s problem.bin\n", argv[0]);
        return 2;
    }
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    Problem p;
    p.V = read_i64(f);
    p.N = read_i64(f);
    p.nnz = read_i64(f);
    const int64_t B = read_i64(f), ns = read_i64(f);
    p.row_ptr = read_vec<int64_t>(f, p.V + 1);
    p.col = read_vec<int32_t>(f, p.nnz);
    p.val = read_vec<double>(f, p.nnz);
    p.rows_per_beam = read_vec<int32_t>(f, B);
    int64_t R = 0;
    for (int32_t r : p.rows_per_beam) R += r;
    p.row_len = read_vec<int32_t>(f, R);
    p.vox_struct = read_vec<int16_t>(f, p.V);
    for (int64_t s = 0; s < ns; ++s) {
        dao_prescription q{};
        q.is_target = read_vec<int32_t>(f, 1)[0];
        const auto d = read_vec<double>(f, 4);
        q.t_under = d[0];
        q.t_over = d[1];
        q.w_under = d[2];
        q.w_over = d[3];
        p.presc.push_back(q);
    }
    std::fclose(f);

    dao_options o;
    std::memset(&o, 0, sizeof(o));
    o.dtype = DAO_F32;
    o.max_apertures = 64;
    o.eps = 1e-6;
    o.max_steps = 500;
    o.tau_rel = 1e-10;
    o.max_tighten = 3;
    o.refresh_every = 50;
    o.ls_slots = 2;
    o.master = DAO_MASTER_APERTURE;
    o.persistent = 2;
    o.product_tune = 1;
    o.gradient_depth = 4;
    o.direction = DAO_DIR_CONJUGATE;
    o.apertures_per_round = 1;
    o.dk_format = DAO_DFMT_NATIVE;
    o.residual_rounds = 5;
    o.graphs = 0;
    expect(validate(p, o) == DAO_OK, "valid problem accepted");

    // ---- the persistent master's dealt row batches: every batch owned by
    // exactly one workgroup, each workgroup's count as coop_nbatches says,
    // never more than the LDS sizing's ceil(batches / workgroups), and a
    // workgroup's local batches in increasing order
    for (int64_t nbat : {int64_t(1), int64_t(7), int64_t(255), int64_t(256), int64_t(257), int64_t(1651),
                         int64_t(11236), int64_t(20000)}) {
        for (uint32_t gn : {1u, 3u, 64u, 255u, 256u}) {
            std::vector<int> owner(size_t(nbat), 0);
            const int64_t most = (nbat + gn - 1) / gn;
            for (uint32_t b = 0; b < gn; ++b) {
                const int64_t n = coop_nbatches(nbat, b, gn);
                expect(n <= most, "no workgroup owns more batches than the LDS holds");
                int64_t prev = -1;
                for (int64_t lb = 0; lb < n; ++lb) {
                    const int64_t bt = coop_batch(lb, b, gn);
                    expect(bt >= 0 && bt < nbat && bt > prev, "dealt batch in range and in order");
                    if (bt >= 0 && bt < nbat) ++owner[size_t(bt)];
                    prev = bt;
                }
            }
            for (int64_t bt = 0; bt < nbat; ++bt) expect(owner[size_t(bt)] == 1, "every batch dealt once");
        }
    }

    // ---- balanced slice lists: every slice once, -1 only past a list's end,
    // each list ascending, and no wavefront's work above the average plus the
    // widest slice (the greedy bound)
    {
        std::mt19937 g(7);
        for (int64_t nw : {int64_t(1), int64_t(5), int64_t(64), int64_t(2048)}) {
            std::vector<int32_t> w(size_t(3000));
            for (auto& x : w) x = 4 * int32_t(1 + g() % 18);
            std::vector<int32_t> order;
            int rounds = 0;
            balanced_slice_order(w, nw, order, rounds);
            expect(int64_t(order.size()) == int64_t(rounds) * nw, "slice lists size");
            std::vector<int> seen(w.size(), 0);
            int64_t total = 0, widest = 0, worst = 0;
            for (auto x : w) { total += x + 4; widest = std::max<int64_t>(widest, x + 4); }
            for (int64_t gw = 0; gw < nw; ++gw) {
                int64_t work = 0, prev = -1;
                bool ended = false;
                for (int k = 0; k < rounds; ++k) {
                    const int32_t sl = order[size_t(k) * size_t(nw) + size_t(gw)];
                    if (sl < 0) { ended = true; continue; }
                    expect(!ended && sl < int32_t(w.size()) && sl > prev, "list entry in range, ascending, unbroken");
                    if (sl >= 0 && sl < int32_t(w.size())) { ++seen[size_t(sl)]; work += w[size_t(sl)] + 4; }
                    prev = sl;
                }
                worst = std::max(worst, work);
            }
            for (int v : seen) expect(v == 1, "every slice in one list");
            expect(worst <= total / nw + widest, "greedy balance bound");
        }
    }

    // ---- the layouts
    const dao_matrix M = p.m();
    const dao_beams Bm = p.b();
    const dao_structures S = p.s();
    HostLayout L;
    build_layout(&M, &Bm, &S, p.presc.data(), &L);
    expect(L.V == p.V && L.N == p.N && L.nnz == p.nnz, "sizes");
    expect(int64_t(L.perm.size()) == L.Vpad && L.Vpad % SLICE == 0, "perm covers the padded rows");
    std::vector<int> seen(size_t(p.V), 0);
    int64_t nonempty = 0;
    for (int64_t v = 0; v < p.V; ++v) nonempty += p.row_ptr[v + 1] > p.row_ptr[v];
    expect(L.Vnz == nonempty, "non-empty row count");
    for (int64_t r = 0; r < L.Vpad; ++r) {
        const int32_t v = L.perm[size_t(r)];
        if (v < 0) continue;
        expect(v < p.V, "perm in range");
        if (v < p.V) ++seen[size_t(v)];
    }
    for (int64_t v = 0; v < p.V; ++v)
        expect(seen[size_t(v)] == (p.row_ptr[v + 1] > p.row_ptr[v] ? 1 : 0), "each non-empty voxel once");
    // forward layout: row r of slice s holds its CSR row, in order, then zeros
    expect(int64_t(L.slice_ptr.size()) == L.nslices + 1, "slice pointers");
    int64_t sell_nz = 0;
    for (int64_t r = 0; r < L.Vpad; ++r) {
        const int64_t s = r / SLICE, l = r % SLICE;
        const int32_t v = L.perm[size_t(r)];
        const int64_t w = L.slice_w[size_t(s)];
        expect(w % 4 == 0, "slice width a multiple of 4");
        const int64_t n = v >= 0 ? p.row_ptr[v + 1] - p.row_ptr[v] : 0;
        expect(n <= w, "row fits its slice");
        for (int64_t k = 0; k < w; ++k) {
            const size_t at = size_t(L.slice_ptr[size_t(s)] + (k / 4) * 256 + 4 * l + k % 4);
            expect(at < L.sell_val.size() && at < L.sell_col.size(), "forward entry in range");
            if (at >= L.sell_val.size()) continue;
            if (k < n) {
                const int64_t e = p.row_ptr[v] + k;
                expect(L.sell_col[at] == uint16_t(p.col[size_t(e)]) && L.sell_val[at] == p.val[size_t(e)],
                       "forward entry equals the CSR entry");
                ++sell_nz;
            } else {
                expect(L.sell_val[at] == 0.0, "forward padding is zero");
            }
        }
    }
    expect(sell_nz == p.nnz, "every CSR entry in the forward layout");
    // transposed layout: column i lists the internal rows of its CSR entries
    expect(int64_t(L.csc_ptr.size()) == p.N + 1 && L.csc_ptr[size_t(p.N)] == p.nnz, "column pointers");
    std::vector<int32_t> inv(size_t(p.V), -1);
    for (int64_t r = 0; r < L.Vpad; ++r)
        if (L.perm[size_t(r)] >= 0) inv[size_t(L.perm[size_t(r)])] = int32_t(r);
    double csr_sum = 0.0, csc_sum = 0.0;
    for (int64_t e = 0; e < p.nnz; ++e) csr_sum += p.val[size_t(e)];
    for (int64_t i = 0; i < p.N; ++i) {
        for (int32_t e = L.csc_ptr[size_t(i)]; e < L.csc_ptr[size_t(i + 1)]; ++e) {
            const int32_t r = L.csc_row[size_t(e)];
            expect(r >= 0 && r < L.Vpad && L.perm[size_t(r)] >= 0, "transposed row in range");
            csc_sum += L.csc_val[size_t(e)];
        }
        float mx = 0.0f;
        for (int32_t e = L.csc_ptr[size_t(i)]; e < L.csc_ptr[size_t(i + 1)]; ++e)
            mx = std::fmax(mx, float(L.csc_val[size_t(e)]));
        expect(L.col_scale[size_t(i)] >= mx * (1.0f - 1e-6f), "column scale covers the column");
    }
    expect(std::fabs(csr_sum - csc_sum) <= 1e-9 * std::fabs(csr_sum), "transposed values sum");
    // objective classes: one per structure plus "none"
    expect(int64_t(L.classes.size()) == int64_t(p.presc.size()) + 1, "class table");
    for (int64_t v = 0; v < p.V; ++v) {
        const int s = p.vox_struct[size_t(v)];
        expect(L.cls_ext[size_t(v)] == uint8_t(s < 0 ? p.presc.size() : size_t(s)), "caller-order class");
        if (inv[size_t(v)] >= 0) expect(L.cls_int[size_t(inv[size_t(v)])] == L.cls_ext[size_t(v)], "internal class");
    }
    // MLC geometry
    int64_t start = 0;
    for (int64_t r = 0; r < R; ++r) {
        expect(L.row_start[size_t(r)] == start && L.row_len[size_t(r)] == p.row_len[size_t(r)], "row geometry");
        for (int32_t q = 0; q < p.row_len[size_t(r)]; ++q) {
            expect(L.blt_row[size_t(start + q)] == r && L.blt_pos[size_t(start + q)] == q, "beamlet position");
        }
        start += p.row_len[size_t(r)];
    }

    // ---- malformed inputs, each rejected before any device call
    auto rejected = [&](const char* what, auto&& mutate) {
        Problem q = p;
        mutate(q);
        expect(validate(q, o) == DAO_EINVAL, std::string("rejects ") + what);
    };
    int64_t r2 = 0;
    while (r2 < p.V && p.row_ptr[r2 + 1] - p.row_ptr[r2] < 2) ++r2;
    rejected("decreasing row_ptr", [&](Problem& q) { q.row_ptr[1] = q.row_ptr[2] + 1; });
    rejected("column out of range", [&](Problem& q) { q.col[0] = int32_t(q.N); });
    rejected("negative column", [&](Problem& q) { q.col[0] = -1; });
    if (r2 < p.V) {
        rejected("duplicate column", [&](Problem& q) { q.col[size_t(q.row_ptr[r2] + 1)] = q.col[size_t(q.row_ptr[r2])]; });
        rejected("unsorted columns", [&](Problem& q) { std::swap(q.col[size_t(q.row_ptr[r2])], q.col[size_t(q.row_ptr[r2] + 1)]); });
    }
    rejected("negative value", [&](Problem& q) { q.val[0] = -1.0; });
    rejected("NaN value", [&](Problem& q) { q.val[0] = std::nan(""); });
    rejected("row lengths not summing to N", [&](Problem& q) { q.row_len[0] += 1; });
    rejected("structure id out of range", [&](Problem& q) { q.vox_struct[0] = int16_t(q.presc.size()); });
    rejected("negative weight", [&](Problem& q) { q.presc[0].w_over = -1.0; });
    rejected("target with t_under > t_over", [&](Problem& q) {
        q.presc[0].is_target = 1;
        q.presc[0].t_under = q.presc[0].t_over + 1.0;
    });
    {
        dao_options bad = o;
        bad.direction = 7;
        expect(validate(p, bad) == DAO_EINVAL, "rejects an unknown direction");
    }

    // ---- 16-bit encoders: nearest value, residual exact in FP64
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> u(-14.0, 15.0);
    for (int t = 0; t < 20000; ++t) {
        const double r = std::ldexp(1.0 + (rng() >> 11) * 0x1p-53, int(std::floor(u(rng))));
        for (int fmt : {int(DAO_DFMT_F16), int(DAO_DFMT_BF16)}) {
            uint16_t hi = 0, lo = 0;
            encode_value(fmt, r, &hi, &lo);
            const double h = fmt == DAO_DFMT_BF16 ? dec_bf16(hi) : dec_f16(hi);
            const double ulp = fmt == DAO_DFMT_BF16 ? 0x1p-7 : 0x1p-10;
            expect(std::fabs(h - r) <= 0.5 * ulp * std::ldexp(1.0, int(std::floor(std::log2(r)))) * (1 + 1e-12),
                   "encoder rounds to nearest");
            expect(std::fabs(h + dec_f16(lo) - r) <= std::fabs(h - r), "residual does not add error");
        }
    }

    if (failures) {
        std::fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    std::printf("OK V=%lld N=%lld nnz=%lld slices=%lld\n", (long long)p.V, (long long)p.N, (long long)p.nnz,
                (long long)L.nslices);
    return 0;
}
