// Host-side validation of the C-ABI inputs and construction of the device
// layouts.  Pure C++ (no HIP): everything here runs before the first device
// call, so malformed inputs are rejected without touching the GPU.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/dao.h"
#include "dao_common.h"

namespace dao {

struct HostLayout {
    int64_t V = 0, N = 0, nnz = 0;
    int64_t Vnz = 0;            // voxel rows with at least one entry
    int64_t nslices = 0;        // ceil(Vnz / SLICE)
    int64_t Vpad = 0;           // nslices * SLICE
    int32_t B = 0, R = 0, max_rows_per_beam = 0, n_struct = 0;

    // forward layout: sliced ELL, 64 rows per slice, each row's entries in
    // groups of 4 (slice width padded to a multiple of 4): entry k of row l
    // of a slice at (k / 4) * 256 + 4 * l + k % 4 from the slice's start
    std::vector<int32_t> perm;        // [Vpad] internal row -> caller voxel (-1: padding)
    std::vector<uint32_t> slice_ptr;  // [nslices + 1] first entry of each slice
    std::vector<int32_t> slice_w;     // [nslices] entries per row in the slice
    std::vector<uint16_t> sell_col;   // [slice_ptr[nslices]]
    std::vector<double> sell_val;     // [slice_ptr[nslices]]

    // transposed layout: beamlet-major (CSC) over internal row numbers
    std::vector<int32_t> csc_ptr;     // [N + 1]
    std::vector<int32_t> csc_row;     // [nnz]
    std::vector<double> csc_val;      // [nnz]
    std::vector<float> col_scale;     // [N] per-beamlet scale of the 16-bit formats (max of the column)

    // objective classes
    std::vector<uint8_t> cls_int;     // [Vpad] class of each internal row
    std::vector<uint8_t> cls_ext;     // [V] class of each caller voxel
    std::vector<ObjClass> classes;    // [n_struct + 1 + structure pairs]
    double F_const = 0.0;             // objective of unreachable voxels at dose 0
    // per-voxel threshold shifts (empty when none): the master keeps the
    // shifted dose d - tau in internal row order
    std::vector<double> tau_ext;      // [V] caller order
    std::vector<double> tau_int;      // [Vpad] internal row order (padding 0)

    // MLC geometry
    std::vector<int32_t> row_start;   // [R] first beamlet of each row
    std::vector<int32_t> row_len;     // [R]
    std::vector<int32_t> beam_row0;   // [B + 1] first row of each beam
    std::vector<int32_t> blt_beam;    // [N]
    std::vector<int32_t> blt_row;     // [N] global row of each beamlet
    std::vector<int32_t> blt_pos;     // [N] position within the row
};

// Round-to-nearest-even encoders of the 16-bit value formats (sign kept,
// overflow to infinity, subnormals exact) and their exact decoders.
uint16_t enc_f16(double r);
uint16_t enc_bf16(double r);
double dec_f16(uint16_t h);
double dec_bf16(uint16_t h);
// hi in `fmt` (DAO_DFMT_F16 / DAO_DFMT_BF16) and the FP16 residual lo.
void encode_value(int fmt, double r, uint16_t* hi, uint16_t* lo);

// Check every input (returns DAO_EINVAL with a message on the first problem).
dao_status validate_inputs(const dao_matrix* D, const dao_beams* beams,
                           const dao_structures* structs, const dao_prescription* presc,
                           const dao_options* opt, std::string* err);

// Build the layouts (inputs must have passed validate_inputs).
void build_layout(const dao_matrix* D, const dao_beams* beams, const dao_structures* structs,
                  const dao_prescription* presc, HostLayout* L);

// Slice lists of the whole-rows forward product for nwaves wavefronts: the
// widest slices first, each to the wavefront with the least work so far
// (ties: the lowest wavefront), work = slice width + 4; each list ascending.
// order[k * nwaves + g] is the k-th slice of wavefront g, -1 past its list;
// rounds = the longest list.
void balanced_slice_order(const std::vector<int32_t>& slice_w, int64_t nwaves, std::vector<int32_t>& order,
                          int& rounds);

}  // namespace dao
