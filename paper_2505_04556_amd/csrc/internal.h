// Internal interfaces between the library's translation units.  Not installed;
// the public ABI is include/pstat.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pstat {

// Label value used for padding rows, columns and permutation lanes; it never
// equals a real label (real labels are < 65535).
constexpr uint16_t kPadLabel = 0xFFFF;
constexpr int kMaxGroups = 65535;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Number of tiles of an upper-triangular tiling with nt tiles per side.
inline int64_t tri_count(int64_t nt) { return nt * (nt + 1) / 2; }

// Upper-triangle tile t (row-major over tile rows I, J = I .. nt-1) -> (I, J).
__device__ inline void tri_decode(int64_t t, int64_t nt, int64_t &I, int64_t &J) {
    const double b = 2.0 * (double)nt + 1.0;
    int64_t r = (int64_t)((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
    if (r < 0) r = 0;
    if (r > nt - 1) r = nt - 1;
    auto off = [nt](int64_t x) { return x * nt - x * (x - 1) / 2; };
    while (r > 0 && off(r) > t) --r;
    while (r + 1 < nt && off(r + 1) <= t) ++r;
    I = r;
    J = r + (t - off(r));
}

// Layouts of D in device memory: the row-major n x n square (packed == 0),
// or only its strict upper triangle, row after row (packed != 0: row i holds
// columns i + 1 .. n - 1 and starts at i (2n - i - 1) / 2; n (n - 1) / 2
// floats in all).  Every kernel reads D only at j > i.
__host__ __device__ inline int64_t d_row_base(int64_t i, int64_t n, int packed) {
    // index of element (i, j) = d_row_base(i) + j
    return packed ? i * (2 * n - i - 1) / 2 - i - 1 : i * n;
}
__host__ __device__ inline int64_t d_index(int64_t i, int64_t j, int64_t n, int packed) {
    return d_row_base(i, n, packed) + j;
}

// ---- staging (k_stage.hip) ------------------------------------------------
// int32 [.][n] -> u16 [n_pad][P_pad] (object-major), pads with kPadLabel;
// staged permutation q is row rows[q] of g (row q when rows is NULL).
// Labels outside [0, limit) set bad_perm[q] = 1 and *err_flag |= 1.
void launch_stage_labels_om(const int32_t *g, const int32_t *rows, int64_t n, int64_t P,
                            int64_t n_pad, int64_t P_pad, int32_t limit, uint16_t *out,
                            uint8_t *bad_perm, int32_t *err_flag, hipStream_t s);
// Range check and maximum of `count` int32 labels (no staging); *max_label
// receives the largest label (atomicMax; the caller sets it to -1 first).
void launch_scan_labels(const int32_t *g, int64_t count, int32_t limit, int32_t *err_flag,
                        int32_t *max_label, hipStream_t s);
// int32 [P][n] -> u16 [P_pad][n_pad] (permutation-major), same checks.
void launch_stage_labels_pm(const int32_t *g, int64_t n, int64_t P, int64_t n_pad,
                            int64_t P_pad, int32_t limit, uint16_t *out, uint8_t *bad_perm,
                            int32_t *err_flag, hipStream_t s);
void launch_fill_u8(uint8_t *p, int64_t count, uint8_t v, hipStream_t s);
void launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s);
void launch_group_weights(const int32_t *grouping, int64_t n, int32_t k, uint32_t *counts,
                          double *inv, hipStream_t s);
// s_T: per-block FP64 partial sums of d^2 over the strict upper triangle,
// then a fixed-order final sum divided by n.
int64_t sT_partials_count(int64_t n);
void launch_sT(const float *mat, int64_t n, double *partials, double *sT, hipStream_t s,
               int packed = 0);
// s_T = (sum of count partials, fixed order) / n
void launch_sT_final(const double *partials, int64_t count, int64_t n, double *sT, hipStream_t s);

// ---- plain kernel (k_plain.hip) -------------------------------------------
struct PlainPlan {
    int tile;        // square tile edge T
    int lanes;       // permutation lanes per work-group (64 * waves)
    int64_t n_t;     // tiles per side
    int64_t n_tiles; // upper-triangle tiles
    int64_t chunks;  // tile chunks (one partial row each)
    int64_t tiles_per_chunk;
    int64_t pgroups; // permutation groups
    int64_t P_pad;   // permutations rounded up to `lanes`
    int64_t n_pad;   // n rounded up to T
};
PlainPlan plain_plan(int64_t n, int64_t P, int tile, int lanes, int n_cu);

// Work-list execution (the serving rounds): fixed tile and lanes.
constexpr int kServeTile = 32;
constexpr int kServeLanes = 256;
struct JobDesc {              // one staged problem, device-resident
    // plain form
    const float *mat;         // D in the layout `packed` names
    int32_t packed;
    const uint16_t *lab;      // u16 [n_pad][P_pad], object-major
    const double *w;
    double *partial;          // [chunks][P_pad]
    int64_t n, nt, n_tiles, tiles_per_chunk, P_pad;
    int32_t k, kind;          // kind: 0 plain FP32, 1 / 2 MFMA split BF16 (512 / 256 columns)
    // MFMA form (split BF16, 512 columns per work-group)
    const void *tiles;        // pre-squared tiles
    const uint16_t *lab_pm;   // u16 [P_pad_m][n_pad_m], permutation-major
    const int32_t *tab;       // work-item table
    float *z;                 // [items][R][k], complement form [items][R][k-1][2]
    int64_t comp_units, kb_total, n_pad_m, R;
    int32_t cx;               // complement form (group *Lp has no columns)
    const int32_t *Lp;
};
struct UnitDesc {             // one work-group's share of one job: plain
    int32_t job, chunk, pgroup;   // (tile chunk, permutation group); MFMA
};                                // (work item, column block)
// FP64 s_W of m groupings (rows[q] of g, [*][n] int32, labels in [0, k)) in
// one pass over D: out[q] for q < m.  partial: few_partial_bytes(n, m) bytes.
size_t few_partial_bytes(int64_t n, int64_t m);
void launch_sw_few(const float *mat, int64_t n, const int32_t *g, const int32_t *rows, int64_t m,
                   int32_t k, const double *w, double *partial, double *out, hipStream_t s,
                   int packed = 0);
// The same with the groupings as u16 rows of `stride` entries (the MFMA
// forms' staged labels).
void launch_sw_few_u16(const float *mat, int64_t n, const uint16_t *g, int64_t stride,
                       const int32_t *rows, int64_t m, int32_t k, const double *w, double *partial,
                       double *out, hipStream_t s, int packed = 0);
// out[q] = sum over r < runs, ascending, of partial[r * stride + q], q < m.
void launch_reduce_partials(const double *partial, int64_t runs, int64_t stride, int64_t m,
                            double *out, hipStream_t s);
void launch_plain_worklist(const JobDesc *jobs, const UnitDesc *units, const int32_t *count,
                           int64_t max_units, hipStream_t s);
// ncols: the column count (512 or 256) every job of the unit list was planned with
void launch_mfma_worklist(const JobDesc *jobs, const UnitDesc *units, const int32_t *count,
                          int64_t max_units, hipStream_t s, int ncols = 512);
// partial[chunk][P_pad] FP64 from u16 [n_pad][P_pad] labels.  Perm lane q of
// the label table is permutation q.  f64 selects the FP64 instantiation.
int launch_plain(const PlainPlan &pl, bool f64, const float *mat, int64_t n,
                 const uint16_t *lab_om, const double *w, int32_t k, double *partial,
                 hipStream_t s, int packed = 0);

// ---- MFMA kernels (k_mfma.hip) ---------------------------------------------
struct MfmaPlan {
    int dtype;        // 0 bf16, 1 f16, 2 split bf16 (hi, lo)
    int64_t n_pad;    // n rounded up to 128 (panel height)
    int64_t panels;   // row panels of 128 rows
    int64_t kb_total; // 64-column K blocks in a row: n_pad / 64
    int64_t kchunk;   // K blocks per work item
    int64_t items;    // (panel, K chunk) work items
    int ncols;        // N columns per work-group
    int64_t N;        // k * P (columns)
    int64_t nblocks;  // ceil(N / ncols)
    int64_t P_pad;    // permutation rows of the staged label table
    size_t tile_bytes;// bytes of the pre-squared tile storage (all components)
    bool cx;          // complement form: one group (the largest) gets no columns
    int32_t kcol;     // columns per grouping: k, or k - 1 in the complement form
};
// cx asks for the complement form (taken when its label staging fits in LDS).
MfmaPlan mfma_plan(int64_t n, int64_t P, int32_t k, int dtype, int kchunk_cols, int ncols,
                   int n_cu, bool cx = false);
size_t mfma_tile_bytes(int64_t n, int dtype);
// FP16 form: the squares are multiplied by 2^e, a power of two chosen from the
// largest |d| of the strict upper triangle so that the largest square lands
// in [2^14, 2^15) (FP16 is finite below 65,504 and has full precision above
// 2^-14: scaling keeps big inputs finite and small ones normal); the FP64
// reduction multiplies by 2^-e.  Both are exact.  The bits of that largest
// |d| sit in a 32-bit cell after the FP16 tiles (f16_max_cell).
const uint32_t *f16_max_cell(const void *tiles, int64_t n);
__device__ inline int f16_scale_exp(uint32_t maxabs_bits) {
    const float d = __builtin_bit_cast(float, maxabs_bits);
    const float m = d * d;   // the same FP32 product as each square
    if (!(m > 0.0f) || !__builtin_isfinite(m)) return 0;
    int E = 0;
    (void)frexpf(m, &E);     // m < 2^E
    const int e = 15 - E;
    return e < -126 ? -126 : e > 127 ? 127 : e;
}
// Pre-pass: strict-upper d^2 of 128-row panels into MFMA fragment order.
// FP64 s_W of rows 0 .. m-1 (m <= kRecheckRows) of a staged u16 label table
// (rows of `stride` entries), computed inside the MFMA pre-pass; part holds
// prepass_blocks(n) * kRecheckRows doubles, out[q] receives row q's s_W.
constexpr int kRecheckRows = 8;
struct PrepassRecheck {
    const uint16_t *lab = nullptr;
    int64_t stride = 0;
    int32_t m = 0;
    const double *w = nullptr;
    int32_t k = 0;
    double *part = nullptr;
    double *out = nullptr;
};
// Pre-squares the strict upper triangle into MFMA fragment order; with
// sT_part (sT_partials_count(n) doubles) set it also leaves s_T in *sT, with
// rc the FP64 s_W of rc->m staged label rows in rc->out, and with rcs
// (complement_part_doubles(n)) the FP64 row and column sums of each unit's
// stored values.
void launch_mfma_prepass(const float *mat, int64_t n, int dtype, void *tiles, hipStream_t s,
                         double *sT_part = nullptr, double *sT = nullptr,
                         const PrepassRecheck *rc = nullptr, double *rcs = nullptr,
                         int packed = 0);
int64_t prepass_blocks(int64_t n);
size_t mfma_table_bytes(const MfmaPlan &pl);
void launch_item_table(const MfmaPlan &pl, int32_t *tab, hipStream_t s);
// z[item][P][k] FP32 sums of the (G^T U G) diagonal per (panel, K chunk) item;
// tab is scratch for the item table (mfma_table_bytes).  Complement form
// (pl.cx): z[item][P][k - 1][2], per column the rows of its group and the
// rows not in group *Lp.
// lab4: the same labels packed four bits each (launch_pack_nibbles; k <= 15),
// or NULL to read the u16 table.
int launch_mfma(const MfmaPlan &pl, const void *tiles, int64_t n, const uint16_t *lab_pm,
                int32_t k, int64_t P, int32_t *tab, float *z, hipStream_t s,
                const int32_t *Lp = nullptr, const uint32_t *lab4 = nullptr);
// Whether launch_mfma should be given the labels packed four bits each for
// this plan (k <= 15; not the three-part split, whose A blocks leave the
// u16 label buffers room).
bool mfma_use_nibbles(const MfmaPlan &pl, int32_t k);
// out (count / 8 dwords) = the u16 label table lab (count entries, a multiple
// of 8, every real label below 15) packed four bits per label, padding as 15.
void launch_pack_nibbles(const uint16_t *lab, int64_t count, uint32_t *out, hipStream_t s);

// ---- complement form (k_reduce.hip) ------------------------------------------
// Device state of one complement-form evaluation.
struct Complement {
    int32_t *L = nullptr;     // [1] the group without columns (the largest)
    double *rcs = nullptr;    // complement_part_doubles(n): per-unit row/column sums
    double *slices = nullptr; // complement_slice_doubles(n): partial sums of rcs
    double *v = nullptr;      // [n_pad] row + column sums of the stored U
    double *r = nullptr;      // [n_pad] row sums
    double *S = nullptr;      // [1] sum of the stored U
    double *vnot = nullptr;   // [P] sum of v over the objects not in L, per grouping
};
int64_t complement_part_doubles(int64_t n);
int64_t complement_slice_doubles(int64_t n);
// *L = the lowest index of the largest count
void launch_largest_group(const uint32_t *counts, int32_t k, int32_t *L, hipStream_t s);
// v, r and S from the pre-pass's per-unit sums.
void launch_complement_sums(const Complement &cx, int64_t n, hipStream_t s);
// vnot[p] = sum over i < n with lab[p * stride + i] != *L of v[i], p < P
// (stride a multiple of 128, rows padded with a label other than *L).
void launch_vnot(const Complement &cx, const uint16_t *lab, int64_t stride, int64_t n, int64_t P,
                 hipStream_t s);

// ---- reductions (k_reduce.hip) ---------------------------------------------
// out[p] = sum_chunk partial[chunk][p] (fixed order); NaN where bad_perm[p].
void launch_reduce_plain(const double *partial, int64_t chunks, int64_t P_pad, int64_t P,
                         const uint8_t *bad_perm, double *out, hipStream_t s);
// out[p] = sum_g w[g] * sum_item z[item][p][g] (FP64, fixed order); tmp holds
// reduce_tmp_doubles(items, P, k) doubles.
size_t reduce_tmp_doubles(int64_t items, int64_t P, int32_t k);
// f16max: the FP16 form's scale cell (f16_max_cell), NULL for the other forms;
// cx: the complement form's state (z then holds k - 1 column pairs per
// grouping, and tmp reduce_tmp_doubles(items, P, 2 (k - 1)) doubles).
void launch_reduce_mfma(const float *z, int64_t items, int64_t P, int32_t k, const double *w,
                        const uint8_t *bad_perm, double *tmp, double *out, hipStream_t s,
                        const uint32_t *f16max = nullptr, const Complement *cx = nullptr);
void launch_F(const double *sW, int64_t count, const double *sT, int64_t n, int32_t k,
              double *F, hipStream_t s);
void launch_pvalue(const double *sW_obs, const double *sW_perm, int64_t P, double *p,
                   hipStream_t s);
// Rows q in [q0, R) of sW_all with sW_all[0] (1 - *band) <= sW_all[q] <=
// sW_all[0] (1 + PSTAT_TIE_RTOL + *band) (sW_all[0] >= 0) go to list (row
// indices): every row whose side of the p-value's edge could be wrong by
// *band; *count (zeroed by the caller) = number flagged.
void launch_flag_ties(const double *sW_all, int64_t q0, int64_t R, const double *band,
                      int32_t *list, int32_t *count, hipStream_t s);
// *band = margin * max_j |fast[j] - exact[j]| / |exact[0]|, j < S, floor 1e-13.
void launch_tie_band(const double *fast, const double *exact, int64_t S, double margin,
                     double *band, hipStream_t s);
void launch_iota(int32_t *list, int64_t m, hipStream_t s);
void launch_scatter(const double *vals, const int32_t *list, int64_t m, double *sW_all,
                    hipStream_t s);
// result = [F_obs, p, s_W_obs, s_T]; with counts (group sizes, [k]) F counts
// only the non-empty groups.
void launch_pack_result(const double *sW_all, const double *sT, int64_t n, int32_t k,
                        const uint32_t *counts, const double *p, double *result, hipStream_t s);

// ---- permutation generator (k_permute.hip) -----------------------------------
// lds_limit: LDS bytes a work-group may use; n_cu: compute units (the lanes
// per permutation depend on whether every permutation runs at once).
int launch_permute(const int32_t *base, int64_t n, int64_t P, uint64_t seed, int32_t max_label,
                   int32_t *out, size_t lds_limit, int n_cu, hipStream_t s);
// The same permutations written as u16 rows of `stride` entries (row p at
// out + p * stride), padded with kPadLabel: the MFMA forms' staged layout.
// Returns nonzero (nothing launched) when no LDS-resident form fits.
int launch_permute_u16(const int32_t *base, int64_t n, int64_t P, uint64_t seed, int32_t max_label,
                       uint16_t *out, int64_t stride, size_t lds_limit, int n_cu, hipStream_t s);

} // namespace pstat
