// Dense-contraction (MFMA) form of s_W.
//
// With U the strict upper triangle of D∘D (u_ij = d_ij^2 for j > i, else 0) and
// G_p the n x k one-hot matrix of permutation p's labels,
//     s_W[p] = sum_g w_g (G_p^T U G_p)_gg,
// which is exactly Algorithm 1's sum (section 2) regrouped: (G^T U G)_gg adds
// u_ij over the pairs i < j that both carry label g.  G is 0/1, so it is exact
// in any input type; only U is rounded (to BF16, FP16, or BF16 hi + BF16 lo),
// or split without rounding into BF16 hi + mid + lo: an FP32 square has 24
// significant bits and each BF16 part takes 8 of them (below).
//
// Blocking.  Rows are cut into 128-row panels and columns into 64-column K
// blocks.  A pre-pass writes, for each panel I, its K blocks from the diagonal
// (block 2I) to the end, each as 128 x 64 values in MFMA fragment order, with
// the entries j <= i of the diagonal blocks set to zero.  The main kernel
// computes Y = U_panel * G over a K range for 256 or 512 columns (p, g) of G at
// a time with v_mfma_f32_32x32x16_{bf16,f16} (FP32 accumulation), staging the
// K blocks of U in LDS and building the one-hot B fragments in registers from
// the staged labels (u16, or four bits each for k <= 15), and in its epilogue
// keeps
// for each column (p, g) only the rows i whose label is g:
//     z[item][p][g] = sum_{i in panel, g_p(i) = g} Y[i][(p, g)].
// Each (panel, K chunk) work item writes its own z; they are summed in FP64 and
// weighted by w_g in FP64 afterwards, so FP32 only ever accumulates one K
// chunk.
//
// Complement form (the whole test and serving jobs, where every grouping is a
// permutation of the observed one and so has its group sizes).  One group L
// (the largest) gets no columns: with e_L = 1 - sum of
// the other one-hot columns,
//     e_L^T U e_L = S - sum_{i: g(i) != L} v_i + sum_{g != L} N_g,
// where S is the sum of U, v_i its row plus column sums, and
// N_g = sum_{i: g(i) != L} (U e_g)_i, which the epilogue gets next to the
// diagonal term at no extra MFMA cost.  k - 1 columns per grouping instead
// of k.  S and v are FP64 sums of the values the MFMAs see (the rounded
// squares), so the identity holds for them exactly; only the FP32
// accumulation error of the N_g is scaled up, by (n - n_L)^2 / (n n_L)
// relative to s_W.
#include <hip/hip_bf16.h>

#include <type_traits>

#include "internal.h"
#include "lane_mask.h"

namespace pstat {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kPanel = 128;      // rows per panel
constexpr int kKBlock = 64;      // columns per K block
constexpr int kUnitU4 = 1024;    // uint4 per (panel, K block) unit per component (16 KB)
// s_waitcnt operand that waits for LDS/scalar loads only: lgkmcnt(0), with the
// vector-memory (vmcnt 63) and export (expcnt 7) fields left at their maxima
constexpr int kLgkmOnly = 0xC07F;

// bits of 1.0 in the MFMA input type
template <int DT>
struct One;
template <>
struct One<0> { static constexpr uint32_t v = 0x3F80u; };  // bf16
template <>
struct One<1> { static constexpr uint32_t v = 0x3C00u; };  // f16

__device__ inline uint16_t to_bf16_bits(float x) {
    __bf16 h = (__bf16)x;  // round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
__device__ inline float bf16_bits_to_float(uint16_t b) {
    return __builtin_bit_cast(float, (uint32_t)b << 16);
}
__device__ inline uint16_t to_f16_bits(float x) {
    _Float16 h = (_Float16)x;  // round to nearest even, subnormals kept
    return __builtin_bit_cast(uint16_t, h);
}

// ---- pre-pass --------------------------------------------------------------
// Unit (I, kb), kb >= 2I: the 128 x 64 block of rows 128I.., columns 64kb..
// of the strict upper triangle.  A work-group walks units blockIdx.x,
// blockIdx.x + gridDim.x, ...: it loads the FP32 block (16-byte row reads when
// every row is 16-byte aligned), squares it into LDS, then writes 1024 uint4
// per component in fragment order: uint4 index ((rb * 4 + s) * 64 + lane)
// holds row rb*32 + lane%32, columns 32*(lane/32) + 8*s + 0..7 of the block.
// With sT_part set it also sums d^2 in FP64 over the same strict upper
// triangle (the s_T numerator) and writes one partial per work-group: threads
// in unit order, then a butterfly over each wave, then the four waves in order.
__device__ inline int64_t unit_panel(int64_t unit, int64_t kb_total) {
    // first unit of panel I: I * (kb_total - I + 1)
    const double b = (double)(kb_total + 1);
    int64_t I = (int64_t)((b - sqrt(b * b - 4.0 * (double)unit)) * 0.5);
    if (I < 0) I = 0;
    while (I > 0 && I * (kb_total - I + 1) > unit) --I;
    while ((I + 1) * (kb_total - I) <= unit) ++I;
    return I;
}

// With RC the same pass also takes the FP64 s_W of the first rc.m (<= 16)
// rows of the staged label table -- the observed grouping and the first
// permutations, which the p-value recheck needs anyway -- so D is read once
// for both.  Each thread holds its 8 x 4 block entries as exact FP64 squares;
// per grouping and column it adds the squares of the rows whose label equals
// the column's (masked adds, rows in order), times the column label's weight,
// into one running FP64 sum per grouping; the sums are reduced like s_T and
// written as one partial per work-group and grouping.
//
// With rcs set (the complement form) each unit also leaves the FP64 sums of
// its 128 rows and 64 columns of the stored values -- hi + lo, hi + mid + lo,
// the BF16 value, or the scaled FP16 value, each exact in FP32 -- at
// rcs[unit * 192 + row] and rcs[unit * 192 + 128 + column], in a fixed order.
// The writer loop leaves those values in LDS; they are summed after the next
// unit's loads are issued (or after the last unit).
__device__ inline void unit_sums(const float (*sm)[kKBlock + 1], double *__restrict__ out,
                                 int tid) {
    // rows: two threads per row, 32 columns each, then their sum
    const int rr = tid >> 1, rh = tid & 1;
    double a = 0.0;
    for (int c = 0; c < 32; c++) a += (double)sm[rr][rh * 32 + c];
    a += __shfl_xor(a, 1);
    if (rh == 0) out[rr] = a;
    // columns: four threads per column, 32 rows each, then in pairs
    const int cc = tid >> 2, c4 = tid & 3;
    double b = 0.0;
    for (int r = 0; r < 32; r++) b += (double)sm[c4 * 32 + r][cc];
    b += __shfl_xor(b, 1);
    b += __shfl_xor(b, 2);
    if (c4 == 0) out[128 + cc] = b;
}

// Loads of one unit into registers: thread t reads rows 16 ps + t / 16
// (ps < 8) at the four columns 4 (t % 16) .. + 3 of the block, 0 outside the
// matrix; with RC also 8 row labels of grouping t / 16 (t < 16 Q) and, for
// t < 8 Q, 8 column labels of grouping t / 8 (16-byte reads; the staged label
// rows are padded to a multiple of 128 entries, so these reads stay inside
// them).
struct PrepassLoads {
    float d[8][4];
    uint4 lr, lc;
};

template <bool RC, int Q>
__device__ __attribute__((always_inline)) inline void prepass_fetch(
    const float *__restrict__ mat, int64_t n, int64_t kb_total, int vec, int packed,
    const PrepassRecheck &rc, int64_t unit, int tid, PrepassLoads &L) {
    const int64_t I = unit_panel(unit, kb_total);
    const int64_t kb = 2 * I + (unit - I * (kb_total - I + 1));
    const int64_t r0 = I * kPanel, c0 = kb * kKBlock;
    const int cq = (tid % 16) * 4, rq = tid / 16;
    // blocks inside the square layout need no per-element test (the same
    // answer for the whole work-group)
    if (vec && r0 + kPanel <= n && c0 + kKBlock <= n) {
        const float *base = mat + (uint64_t)(r0 + rq) * (uint64_t)n + (c0 + cq);
#pragma unroll
        for (int ps = 0; ps < 8; ps++) {
            const float4 v = *reinterpret_cast<const float4 *>(base + (uint64_t)(16 * ps) * n);
            L.d[ps][0] = v.x;
            L.d[ps][1] = v.y;
            L.d[ps][2] = v.z;
            L.d[ps][3] = v.w;
        }
    } else {
#pragma unroll
        for (int ps = 0; ps < 8; ps++) {
            const int64_t i = r0 + ps * 16 + rq, j0 = c0 + cq;
            if (vec && i < n && j0 + 3 < n) {
                const float4 v =
                    *reinterpret_cast<const float4 *>(mat + (uint64_t)i * (uint64_t)n + j0);
                L.d[ps][0] = v.x;
                L.d[ps][1] = v.y;
                L.d[ps][2] = v.z;
                L.d[ps][3] = v.w;
            } else {
                // (the packed layout has no entries at j <= i)
#pragma unroll
                for (int e = 0; e < 4; e++)
                    L.d[ps][e] = (i < n && j0 + e < n && (!packed || j0 + e > i))
                                     ? mat[d_index(i, j0 + e, n, packed)]
                                     : 0.0f;
            }
        }
    }
    L.lr = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
    L.lc = L.lr;
    if constexpr (RC) {
        const int qr = tid / 16, qc = tid / 8;
        if (qr < rc.m)
            L.lr = *reinterpret_cast<const uint4 *>(rc.lab + qr * rc.stride + r0 + (tid % 16) * 8);
        if (tid < 8 * Q && qc < rc.m)
            L.lc = *reinterpret_cast<const uint4 *>(rc.lab + qc * rc.stride + c0 + (tid % 8) * 8);
    }
}

template <int DT, bool RC>
__global__ __launch_bounds__(256) void k_prepass(const float *__restrict__ mat, int64_t n,
                                                 int64_t kb_total, int64_t comp_units, int vec,
                                                 uint4 *__restrict__ tiles,
                                                 double *__restrict__ sT_part, PrepassRecheck rc,
                                                 const uint32_t *__restrict__ f16max,
                                                 double *__restrict__ rcs, int packed) {
    constexpr int Q = RC ? kRecheckRows : 1;
    // FP16: the power of two that brings the largest square into [2^14, 2^15)
    float f16sc = 1.0f;
    if constexpr (DT == 1) f16sc = ldexpf(1.0f, f16_scale_exp(*f16max));
    __shared__ float sm[kPanel][kKBlock + 1];
    __shared__ double sred[4];
    // recheck labels: rows as [grouping][row % 16][row / 16] (a thread's 8
    // rows are contiguous), columns and their weights as [grouping][column]
    __shared__ __align__(16) uint32_t rrow[Q][16][8];
    __shared__ __align__(16) uint32_t rcol[Q][kKBlock];
    __shared__ __align__(16) double rw[Q][kKBlock];
    __shared__ double rred[RC ? 4 : 1][Q];
    const int tid = threadIdx.x;
    const int cq = (tid % 16) * 4;   // four columns of the block
    const int rq = tid / 16;         // row within each pass of 16 rows
    double st = 0.0;
    double acc[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) acc[q] = 0.0;
    int64_t prev = -1;   // the unit whose stored values LDS holds
    for (int64_t unit = blockIdx.x; unit < comp_units; unit += gridDim.x) {
        const int64_t I = unit_panel(unit, kb_total);
        const int64_t kb = 2 * I + (unit - I * (kb_total - I + 1));
        const int64_t r0 = I * kPanel, c0 = kb * kKBlock;
        PrepassLoads cur;
        prepass_fetch<RC, Q>(mat, n, kb_total, vec, packed, rc, unit, tid, cur);
        if (rcs && prev >= 0) {
            __syncthreads();   // the previous unit's stored values are in LDS
            unit_sums(sm, rcs + prev * 192, tid);
        }
        prev = unit;
        __syncthreads();   // the previous unit's LDS reads are done
        // squares: FP32 into LDS for the fragments; exact FP64 for s_T and
        // the recheck; 0 off the strict upper triangle.  Only the diagonal
        // blocks and the matrix's edge need that test, so the work-group
        // takes one of two versions of this part per unit (EDGE or not): in
        // block coordinates an entry is kept when row < lim_r, column <
        // lim_c and column + delta > row.
        const int lim_r = (int)(n - r0 < kPanel ? n - r0 : kPanel);
        const int lim_c = (int)(n - c0 < kKBlock ? n - c0 : kKBlock);
        const int delta = (int)(c0 - r0 < 2 * kPanel ? c0 - r0 : 2 * kPanel);
        const bool edge = lim_r < kPanel || lim_c < kKBlock || delta < kPanel;
        auto squares = [&](auto edge_tag) {
            constexpr bool EDGE = decltype(edge_tag)::value;
            auto kept = [&](int ps, int e) {
                const int r = ps * 16 + rq, c = cq + e;
                return !EDGE || (r < lim_r && c < lim_c && c + delta > r);
            };
#pragma unroll
            for (int ps = 0; ps < 8; ps++) {
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const float x = cur.d[ps][e];
                    const bool keep = kept(ps, e);
                    sm[ps * 16 + rq][cq + e] = keep ? x * x : 0.0f;
                    if constexpr (!RC) st += keep ? (double)x * (double)x : 0.0;
                }
            }
            if constexpr (RC) {
                const uint32_t l8[4] = {cur.lr.x, cur.lr.y, cur.lr.z, cur.lr.w};
                const int qr = tid / 16, rb = (tid % 16) * 8;
                if (qr < Q) {
#pragma unroll
                    for (int e = 0; e < 8; e++) {
                        const int r = rb + e;
                        rrow[qr][r % 16][r / 16] = (l8[e / 2] >> (16 * (e % 2))) & 0xFFFFu;
                    }
                }
                if (tid < 8 * Q) {
                    const uint32_t c8[4] = {cur.lc.x, cur.lc.y, cur.lc.z, cur.lc.w};
                    const int qc = tid / 8, cb = (tid % 8) * 8;
#pragma unroll
                    for (int e = 0; e < 8; e++) {
                        const uint32_t l = (c8[e / 2] >> (16 * (e % 2))) & 0xFFFFu;
                        rcol[qc][cb + e] = l;
                        rw[qc][cb + e] = (l < (uint32_t)rc.k) ? rc.w[l] : 0.0;
                    }
                }
            }
            __syncthreads();
            if constexpr (RC) {
                // one column at a time: its 8 exact FP64 squares (which also
                // go into s_T), then every grouping's masked sum of them
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    double d2[8];
#pragma unroll
                    for (int ps = 0; ps < 8; ps++) {
                        const float x = cur.d[ps][e];
                        d2[ps] = kept(ps, e) ? (double)x * (double)x : 0.0;
                        st += d2[ps];
                    }
                    static_assert(Q % 2 == 0, "groupings in pairs");
#pragma unroll
                    for (int q = 0; q < Q; q += 2) {
                        const uint4 ra = *reinterpret_cast<const uint4 *>(&rrow[q][rq][0]);
                        const uint4 rb = *reinterpret_cast<const uint4 *>(&rrow[q][rq][4]);
                        const uint4 sa = *reinterpret_cast<const uint4 *>(&rrow[q + 1][rq][0]);
                        const uint4 sb = *reinterpret_cast<const uint4 *>(&rrow[q + 1][rq][4]);
                        const uint32_t rl0[8] = {ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, rb.w};
                        const uint32_t rl1[8] = {sa.x, sa.y, sa.z, sa.w, sb.x, sb.y, sb.z, sb.w};
                        double s0 = 0.0, s1 = 0.0;
                        masked_add8_pair(s0, rcol[q][cq + e], rl0, s1, rcol[q + 1][cq + e], rl1, d2);
                        acc[q] = __builtin_fma(s0, rw[q][cq + e], acc[q]);
                        acc[q + 1] = __builtin_fma(s1, rw[q + 1][cq + e], acc[q + 1]);
                    }
                }
            }
        };
        if (edge)
            squares(std::integral_constant<bool, true>{});
        else
            squares(std::integral_constant<bool, false>{});
        const int64_t off = unit;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int idx = tid + 256 * q;
            const int rb = idx / 256, s = (idx / 64) % 4, lane = idx % 64;
            const int r = rb * 32 + (lane % 32);
            const int cb = 32 * (lane / 32) + 8 * s;
            uint32_t hw[4], lw[4], tw[4];
#pragma unroll
            for (int e2 = 0; e2 < 4; e2++) {
                const float x0 = sm[r][cb + 2 * e2], x1 = sm[r][cb + 2 * e2 + 1];
                float s0, s1;   // the values the MFMAs will see
                if (DT == 1) {
                    const uint16_t h0 = to_f16_bits(x0 * f16sc), h1 = to_f16_bits(x1 * f16sc);
                    hw[e2] = (uint32_t)h0 | ((uint32_t)h1 << 16);
                    s0 = (float)__builtin_bit_cast(_Float16, h0);
                    s1 = (float)__builtin_bit_cast(_Float16, h1);
                } else {
                    const uint16_t h0 = to_bf16_bits(x0), h1 = to_bf16_bits(x1);
                    hw[e2] = (uint32_t)h0 | ((uint32_t)h1 << 16);
                    // x - hi is exact in FP32 (hi is x rounded to 8 bits, so
                    // they share the exponent range); for DT 3 the remainder
                    // is split once more and the last remainder, at most 8
                    // significant bits, is exact in BF16 (normal range)
                    const float r0f = x0 - bf16_bits_to_float(h0);
                    const float r1f = x1 - bf16_bits_to_float(h1);
                    const uint16_t l0 = to_bf16_bits(r0f), l1 = to_bf16_bits(r1f);
                    lw[e2] = (uint32_t)l0 | ((uint32_t)l1 << 16);
                    s0 = bf16_bits_to_float(h0);
                    s1 = bf16_bits_to_float(h1);
                    if (DT >= 2) {   // hi + lo has at most 24 significant bits
                        s0 += bf16_bits_to_float(l0);
                        s1 += bf16_bits_to_float(l1);
                    }
                    if (DT == 3) {
                        const uint16_t t0 = to_bf16_bits(r0f - bf16_bits_to_float(l0));
                        const uint16_t t1 = to_bf16_bits(r1f - bf16_bits_to_float(l1));
                        tw[e2] = (uint32_t)t0 | ((uint32_t)t1 << 16);
                        s0 += bf16_bits_to_float(t0);
                        s1 += bf16_bits_to_float(t1);
                    }
                }
                // each element is read and rewritten by this thread only
                if (rcs) {
                    sm[r][cb + 2 * e2] = s0;
                    sm[r][cb + 2 * e2 + 1] = s1;
                }
            }
            tiles[off * kUnitU4 + idx] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
            if (DT >= 2)
                tiles[(comp_units + off) * kUnitU4 + idx] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
            if (DT == 3)
                tiles[(2 * comp_units + off) * kUnitU4 + idx] = make_uint4(tw[0], tw[1], tw[2], tw[3]);
        }
    }
    if (rcs && prev >= 0) {
        __syncthreads();
        unit_sums(sm, rcs + prev * 192, tid);
    }
    if (sT_part) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) st += __shfl_xor(st, o);
        if (tid % 64 == 0) sred[tid / 64] = st;
        __syncthreads();
        if (tid == 0) sT_part[blockIdx.x] = ((sred[0] + sred[1]) + sred[2]) + sred[3];
    }
    if constexpr (RC) {
#pragma unroll
        for (int q = 0; q < Q; q++) {
            double v = acc[q];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
            if (tid % 64 == 0) rred[tid / 64][q] = v;
        }
        __syncthreads();
        if (tid < Q)
            rc.part[(int64_t)blockIdx.x * Q + tid] =
                ((rred[0][tid] + rred[1][tid]) + rred[2][tid]) + rred[3][tid];
    }
}

// Largest |d| over the strict upper triangle, as float bits (non-negative
// floats order like their bit patterns; a NaN orders above infinity), folded
// into *cell with one atomicMax per work-group.  Work-group b takes rows b,
// b + gridDim.x, ...
__global__ __launch_bounds__(256) void k_max_abs_upper(const float *__restrict__ mat, int64_t n,
                                                       uint32_t *__restrict__ cell, int packed) {
    __shared__ uint32_t red[4];
    uint32_t m = 0;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int64_t rb = d_row_base(i, n, packed);
        for (int64_t j = i + 1 + threadIdx.x; j < n; j += 256) {
            const uint32_t b = __builtin_bit_cast(uint32_t, mat[rb + j]) & 0x7FFFFFFFu;
            m = b > m ? b : m;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint32_t v = (uint32_t)__shfl_xor((int)m, o);
        m = v > m ? v : m;
    }
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t r = red[0];
        for (int q = 1; q < 4; q++) r = red[q] > r ? red[q] : r;
        atomicMax(cell, r);
    }
}

// ---- labels packed four bits each ------------------------------------------------
// out dword e = the 8 u16 labels e*8 .. e*8+7 of the staged table, label i in
// bits 4i .. 4i+3 (every label below 15, the padding 0xFFFF becomes 15).
__global__ __launch_bounds__(256) void k_pack_nibbles(const uint4 *__restrict__ lab,
                                                      int64_t words, uint32_t *__restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < words;
         e += (int64_t)gridDim.x * 256) {
        const uint4 v = lab[e];
        const uint32_t h[4] = {v.x, v.y, v.z, v.w};
        uint32_t w = 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const uint32_t lo = h[q] & 0xFFFFu, hi = h[q] >> 16;
            w |= ((lo < 15u ? lo : 15u) | ((hi < 15u ? hi : 15u) << 4)) << (8 * q);
        }
        out[e] = w;
    }
}

// ---- work items ---------------------------------------------------------------
// tab[3*item] = panel I, tab[3*item+1] = first K block, tab[3*item+2] = end.
// Items in panel order, K chunks ascending; thread I writes panel I's items
// after counting those of the panels before it.
__global__ __launch_bounds__(256) void k_item_table(int64_t panels, int64_t kb_total,
                                                    int64_t kchunk, int32_t *__restrict__ tab) {
    const int64_t I = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (I >= panels) return;
    int64_t it = 0;
    for (int64_t J = 0; J < I; J++) it += (kb_total - 2 * J + kchunk - 1) / kchunk;
    for (int64_t kb = 2 * I; kb < kb_total; kb += kchunk) {
        const int64_t e = kb + kchunk < kb_total ? kb + kchunk : kb_total;
        tab[3 * it] = (int32_t)I;
        tab[3 * it + 1] = (int32_t)kb;
        tab[3 * it + 2] = (int32_t)e;
        it++;
    }
}

// One-hot of 8 labels against g: 1.0 where label == g, else 0, two 16-bit
// lanes per dword: x = labels ^ (g, g) is 0 exactly where they match;
// saturating (1, 1) - x is then 1 there and 0 elsewhere; times the bits of 1.0.
// Written as packed 16-bit instructions (ALU only) so that each dword costs
// three VALU operations.
template <int DT>
__device__ inline uint4 onehot8(uint4 L, uint32_t gg) {
    const uint32_t one1 = 0x00010001u;
    const uint32_t onev = One<DT>::v | (One<DT>::v << 16);
    uint32_t in[4] = {L.x, L.y, L.z, L.w};
    uint32_t out[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint32_t x = in[q] ^ gg;
        uint32_t t, o;
        asm("v_pk_sub_u16 %0, %1, %2 clamp" : "=v"(t) : "v"(one1), "v"(x));
        asm("v_pk_mul_lo_u16 %0, %1, %2" : "=v"(o) : "v"(t), "v"(onev));
        out[q] = o;
    }
    return make_uint4(out[0], out[1], out[2], out[3]);
}

// The same from 8 labels packed four bits each (label i in bits 4i .. 4i+3):
// y = labels ^ (g in every nibble) is 0 in exactly the matching nibbles; a
// byte permute puts byte q (labels 2q, 2q+1) in both 16-bit halves, the mask
// keeps the low nibble in the low half and the high nibble (times 16) in the
// high one, and the saturating subtract and multiply follow as above: four
// VALU operations per dword, and one per eight labels for the xor.
template <int DT>
__device__ inline uint4 onehot8_nib(uint32_t L, uint32_t gg) {
    const uint32_t one1 = 0x00010001u;
    const uint32_t onev = One<DT>::v | (One<DT>::v << 16);
    const uint32_t y = L ^ ((gg & 0xFu) * 0x11111111u);
    uint32_t out[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        // selector bytes: q, zero, q, zero (0x0C selects the constant 0)
        const uint32_t sel = (uint32_t)q | 0x0C00u | ((uint32_t)q << 16) | 0x0C000000u;
        const uint32_t v = __builtin_amdgcn_perm(0u, y, sel) & 0x00F0000Fu;
        uint32_t t, o;
        asm("v_pk_sub_u16 %0, %1, %2 clamp" : "=v"(t) : "v"(one1), "v"(v));
        asm("v_pk_mul_lo_u16 %0, %1, %2" : "=v"(o) : "v"(t), "v"(onev));
        out[q] = o;
    }
    return make_uint4(out[0], out[1], out[2], out[3]);
}

// zs += y[b] where lab[b] == g, zn += y[b] where lab[b] != L, for b = 0..3
// in order: eight compares write lane masks, then each add runs under its
// mask in EXEC (the sums are those of the selects, term by term).  Every lane
// must be active on entry.
__device__ inline void masked_pair4(float &zs, float &zn, uint32_t g, uint32_t L,
                                    const uint32_t *lab, const float *y) {
    uint64_t e0, e1, e2, e3, m0, m1, m2, m3, sv;
    asm volatile(
        "v_cmp_eq_u32_e64 %[e0], %[g], %[l0]\n"
        "v_cmp_eq_u32_e64 %[e1], %[g], %[l1]\n"
        "v_cmp_eq_u32_e64 %[e2], %[g], %[l2]\n"
        "v_cmp_eq_u32_e64 %[e3], %[g], %[l3]\n"
        "v_cmp_ne_u32_e64 %[m0], %[L], %[l0]\n"
        "v_cmp_ne_u32_e64 %[m1], %[L], %[l1]\n"
        "v_cmp_ne_u32_e64 %[m2], %[L], %[l2]\n"
        "v_cmp_ne_u32_e64 %[m3], %[L], %[l3]\n"
        "s_mov_b64 %[sv], exec\n"
        "s_mov_b64 exec, %[e0]\n"
        "v_add_f32 %[zs], %[zs], %[y0]\n"
        "s_mov_b64 exec, %[m0]\n"
        "v_add_f32 %[zn], %[zn], %[y0]\n"
        "s_mov_b64 exec, %[e1]\n"
        "v_add_f32 %[zs], %[zs], %[y1]\n"
        "s_mov_b64 exec, %[m1]\n"
        "v_add_f32 %[zn], %[zn], %[y1]\n"
        "s_mov_b64 exec, %[e2]\n"
        "v_add_f32 %[zs], %[zs], %[y2]\n"
        "s_mov_b64 exec, %[m2]\n"
        "v_add_f32 %[zn], %[zn], %[y2]\n"
        "s_mov_b64 exec, %[e3]\n"
        "v_add_f32 %[zs], %[zs], %[y3]\n"
        "s_mov_b64 exec, %[m3]\n"
        "v_add_f32 %[zn], %[zn], %[y3]\n"
        "s_mov_b64 exec, %[sv]\n"
        : [zs] "+v"(zs), [zn] "+v"(zn), [e0] "=&s"(e0), [e1] "=&s"(e1), [e2] "=&s"(e2),
          [e3] "=&s"(e3), [m0] "=&s"(m0), [m1] "=&s"(m1), [m2] "=&s"(m2), [m3] "=&s"(m3),
          [sv] "=&s"(sv)
        : [g] "v"(g), [L] "v"(L), [l0] "v"(lab[0]), [l1] "v"(lab[1]), [l2] "v"(lab[2]),
          [l3] "v"(lab[3]), [y0] "v"(y[0]), [y1] "v"(y[1]), [y2] "v"(y[2]), [y3] "v"(y[3]));
}

template <int DT>
__device__ inline f32x16 mma(uint4 a, uint4 b, f32x16 c) {
    if (DT == 1)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// DT: 0 bf16, 1 f16, 2 split bf16 (hi and lo MFMAs into one accumulator),
// 3 three-part split bf16 (hi, mid, lo).
// NF: 32-column fragments per wave; a work-group of 4 waves covers 128 rows x
// (4 * NF * 32) columns.
//
// Pipeline.  Each K block is copied global -> LDS by the direct-to-LDS load
// (no registers): the block of A (the pre-squared tiles) and the 64 labels of
// every permutation the work-group's columns belong to.  The copy of block
// kb + 1 is issued before block kb is computed and waited for at the barrier
// that ends block kb, so it has a whole block of MFMA work to land.  All
// operands of the MFMAs then come from LDS, none from global memory: the
// vector-memory counter retires in issue order, so waiting for any global load
// issued after the copy would also wait for the copy.  Two LDS buffers of each
// kind are separate variables and the loop is unrolled by two (items have an
// even number of K blocks), so every access names its buffer statically and
// the compiler can see that reads of one buffer do not depend on the copy into
// the other.
// cx: complement form -- kcol = k - 1 columns per grouping, for the groups
// other than Lg; the epilogue writes two sums per column (rows of the
// column's group, rows not in Lg).  Otherwise kcol = k.
// NIB: the labels come from the table packed four bits per label (k <= 15,
// padding 15): per permutation and K block two 16-byte chunks, no pad
// chunk; a K step reads one dword (8 labels) instead of 16 bytes.
template <int DT, int NF, int LQ, bool NIB>
__device__ __attribute__((always_inline)) inline void mfma_unit(
    const uint4 *__restrict__ tiles, int64_t comp_units, int64_t kb_total,
    const int32_t *__restrict__ tab, int64_t item, int64_t nb, const uint16_t *__restrict__ lab,
    const uint32_t *__restrict__ lab4, int64_t n_pad, bool cx, int32_t kcol, int32_t Lg, int64_t P,
    float *__restrict__ z) {
    constexpr int BT = DT == 1 ? 1 : 0;     // operand type of the MFMA
    constexpr int NC = DT == 3 ? 3 : DT == 2 ? 2 : 1;   // A components (hi, [mid,] lo)
    constexpr int UNIT = NC * kUnitU4;      // uint4 of one staged K block
    constexpr int COLS = 4 * NF * 32;       // columns per work-group
    // Labels of one K block: per permutation 8 chunks of 8 u16 (16 bytes) and
    // one pad chunk (a stride of 9 chunks spreads neighbouring permutations
    // over the LDS banks); LQ * 256 slots hold the (COLS - 1) / k + 2
    // permutations a work-group's columns can touch (the launch picks LQ).
    constexpr int kLStride = NIB ? 2 : 9;   // 16-byte slots per permutation
    constexpr int LSLOTS = LQ * 256;
    __shared__ uint4 sA0[UNIT];
    __shared__ uint4 sA1[UNIT];
    __shared__ uint4 sL0[LSLOTS];
    __shared__ uint4 sL1[LSLOTS];
    __shared__ uint4 sE0[NIB ? LSLOTS : 1];
    __shared__ uint4 sE1[NIB ? LSLOTS : 1];
    const int64_t I = tab[3 * item], kb0 = tab[3 * item + 1], kb1 = tab[3 * item + 2];
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int half = lane / 32, col = lane % 32;
    // permutations of this work-group's columns (p_hi < the padded count)
    const int64_t p_lo = nb * COLS / kcol;
    const int64_t p_hi = (nb * COLS + COLS - 1) / kcol;

    // Per column fragment: its group (both 16-bit halves) and the LDS label
    // slot of its permutation (everything else is derived from these two).
    uint32_t gg[NF];
    int lslot[NF];
#pragma unroll
    for (int nf = 0; nf < NF; nf++) {
        const int64_t c = nb * COLS + wave * (NF * 32) + nf * 32 + col;
        const int64_t p = c / kcol;
        uint32_t g = (uint32_t)(c - p * kcol);
        if (cx && g >= (uint32_t)Lg) g++;   // the column's group skips Lg
        gg[nf] = g | (g << 16);
        // K step s of a block uses rows 8s + 32*half + 0..7: chunk s + 4*half
        // (u16: 16-byte slot; NIB: dword, 8 per permutation)
        lslot[nf] = NIB ? (int)(p - p_lo) * 8 + 4 * half : (int)(p - p_lo) * kLStride + 4 * half;
    }

    f32x16 acc[4][NF];
#pragma unroll
    for (int rb = 0; rb < 4; rb++)
#pragma unroll
        for (int nf = 0; nf < NF; nf++)
#pragma unroll
            for (int v = 0; v < 16; v++) acc[rb][nf][v] = 0.0f;

    const int64_t panel_off = I * kb_total - I * (I - 1);
    // Copy of K block kb: lane l of wave w moves uint4 number q*256 + 64w + l
    // (A: both sides in fragment order; labels: slot j = 9 * perm + chunk,
    // the pad chunk repeating chunk 0 and slots past the last permutation
    // repeating it, so every source address is inside the label array).
    auto stage_labels = [&](int64_t kb, uint4 *dL) {
#pragma unroll
        for (int q = 0; q < LQ; q++) {
            const int j = q * 256 + tid;
            const int pr = j / kLStride;
            int ch = j - pr * kLStride;
            if (!NIB && ch == kLStride - 1) ch = 0;
            int64_t p = p_lo + pr;
            if (p > p_hi) p = p_hi;
            // NIB rows hold n_pad / 2 bytes, 32 per K block
            const void *src = NIB ? (const void *)((const char *)lab4 + p * (n_pad / 2) +
                                                   kb * (kKBlock / 2) + ch * 16)
                                  : (const void *)(lab + p * n_pad + kb * kKBlock + ch * 8);
            __builtin_amdgcn_global_load_lds(
                (__attribute__((address_space(1))) void *)src,
                (__attribute__((address_space(3))) void *)&dL[q * 256 + wave * 64], 16, 0, 0);
        }
    };
    auto stage = [&](int64_t kb, uint4 *dA, uint4 *dL) {
#pragma unroll
        for (int q = 0; q < UNIT / 256; q++) {
            const uint4 *src = tiles + ((int64_t)(q / 4) * comp_units + panel_off + (kb - 2 * I)) *
                                           kUnitU4 + (q % 4) * 256 + tid;
            __builtin_amdgcn_global_load_lds(
                (__attribute__((address_space(1))) void *)src,
                (__attribute__((address_space(3))) void *)&dA[q * 256 + wave * 64], 16, 0, 0);
        }
        stage_labels(kb, dL);
    };
    // Software pipeline over K steps: the A fragments and labels of step t+1
    // are read from LDS before the MFMAs of step t are issued, and B(t+1) is
    // built from those labels while the second half of step t's MFMAs run.
    // Scheduling barriers pin this order (left to itself the compiler reads
    // each A fragment just before its MFMAs, exposing the LDS latency).
    uint4 Ac[4][NC], An[4][NC];
    uint4 Ln[NF], BX[2][NF];   // one-hot fragments of alternate K steps
    uint32_t Lw[NF];
    auto load_step = [&](const uint4 *cA, const uint4 *cL, int s) {
#pragma unroll
        for (int rb = 0; rb < 4; rb++)
#pragma unroll
            for (int c = 0; c < NC; c++) An[rb][c] = cA[c * kUnitU4 + (rb * 4 + s) * 64 + lane];
#pragma unroll
        for (int nf = 0; nf < NF; nf++) {
            if constexpr (NIB)
                Lw[nf] = reinterpret_cast<const uint32_t *>(cL)[lslot[nf] + s];
            else
                Ln[nf] = cL[lslot[nf] + s];
        }
    };
    auto build_b = [&](uint4 *B) {
#pragma unroll
        for (int nf = 0; nf < NF; nf++)
            B[nf] = NIB ? onehot8_nib<BT>(Lw[nf], gg[nf]) : onehot8<BT>(Ln[nf], gg[nf]);
    };
    // One dword (two 16-bit one-hot values) of the next step's fragment nf.
    auto onehot_piece = [&](uint4 *Bn, int nf, int q, uint32_t y) {
        const uint32_t one1 = 0x00010001u;
        const uint32_t onev = One<BT>::v | (One<BT>::v << 16);
        uint32_t x;
        if constexpr (NIB) {
            const uint32_t sel = (uint32_t)q | 0x0C00u | ((uint32_t)q << 16) | 0x0C000000u;
            x = __builtin_amdgcn_perm(0u, y, sel) & 0x00F0000Fu;
        } else {
            const uint32_t in[4] = {Ln[nf].x, Ln[nf].y, Ln[nf].z, Ln[nf].w};
            x = in[q] ^ gg[nf];
        }
        uint32_t t, o;
        asm("v_pk_sub_u16 %0, %1, %2 clamp" : "=v"(t) : "v"(one1), "v"(x));
        asm("v_pk_mul_lo_u16 %0, %1, %2" : "=v"(o) : "v"(t), "v"(onev));
        if (q == 0) Bn[nf].x = o;
        if (q == 1) Bn[nf].y = o;
        if (q == 2) Bn[nf].z = o;
        if (q == 3) Bn[nf].w = o;
    };
    // MFMAs of the current step (one-hot fragments Bc), with the VALU that
    // builds the next step's fragments (into Bn, the other buffer) placed one
    // dword after each MFMA from the fifth on, so the MFMA pipe never waits
    // for a run of VALU; then A of the next step.  Scheduling barriers pin
    // the order (left to itself the compiler issues most MFMAs first).
    auto step = [&](const uint4 *Bc, uint4 *Bn) {
        constexpr int NP = 4 * NF;   // dwords of the next fragments
        uint32_t y[NF];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int rb = 0; rb < 4; rb++)
#pragma unroll
            for (int c = 0; c < NC; c++)
#pragma unroll
                for (int nf = 0; nf < NF; nf++) {
                    const int i = (rb * NC + c) * NF + nf;
                    acc[rb][nf] = mma<BT>(Ac[rb][c], Bc[nf], acc[rb][nf]);
                    const int p = i - 4;
                    if (p >= 0 && p < NP) {
                        const int pf = p / 4, pq = p % 4;
                        if constexpr (NIB)
                            if (pq == 0) y[pf] = Lw[pf] ^ ((gg[pf] & 0xFu) * 0x11111111u);
                        onehot_piece(Bn, pf, pq, NIB ? y[pf] : 0u);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
        for (int p = 4 * NC * NF - 4; p < NP; p++) {   // left over when NC = 1
            const int pf = p / 4, pq = p % 4;
            if constexpr (NIB)
                if (pq == 0) y[pf] = Lw[pf] ^ ((gg[pf] & 0xFu) * 0x11111111u);
            onehot_piece(Bn, pf, pq, NIB ? y[pf] : 0u);
        }
#pragma unroll
        for (int rb = 0; rb < 4; rb++)
#pragma unroll
            for (int c = 0; c < NC; c++) Ac[rb][c] = An[rb][c];
        __builtin_amdgcn_sched_barrier(0);
    };
    // Block kb from (cA, cL); the copy of block kb + 1 into (nA, nL) was
    // issued one block earlier.  The barrier sits before the last step: by
    // then every read of (cA, cL) has been issued and waited for, so the copy
    // of block kb + 2 may reuse them, and the next block's first operands are
    // read while the last step's MFMAs run.  Past the item's last block the
    // copy repeats that block and the reads of the next one are not used:
    // every address stays in range and the code stays branch-free.
    auto block = [&](int64_t kb, uint4 *cA, uint4 *cL, const uint4 *nA, const uint4 *nL) {
        load_step(cA, cL, 1);
        step(BX[0], BX[1]);
        load_step(cA, cL, 2);
        step(BX[1], BX[0]);
        load_step(cA, cL, 3);
        step(BX[0], BX[1]);
        __builtin_amdgcn_s_waitcnt(0);   // this wave's copies have landed
        __syncthreads();                 // ... and every wave's; reads of cA done
        stage(kb + 2 < kb1 ? kb + 2 : kb1 - 1, cA, cL);
        load_step(nA, nL, 0);
        step(BX[1], BX[0]);
        // The next block's A fragments were read a whole step ago; saying so
        // here keeps the wait for them out of the loop's first MFMAs (the
        // compiler cannot track LDS reads across the loop's back edge).
        __builtin_amdgcn_s_waitcnt(kLgkmOnly);
    };

    stage(kb0, sA0, sL0);
    if constexpr (NIB) {
        stage_labels(2 * I, sE0);
        stage_labels(2 * I + 1, sE1);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    stage(kb0 + 1, sA1, sL1);
    load_step(sA0, sL0, 0);
    build_b(BX[0]);
#pragma unroll
    for (int rb = 0; rb < 4; rb++)
#pragma unroll
        for (int c = 0; c < NC; c++) Ac[rb][c] = An[rb][c];
    __builtin_amdgcn_s_waitcnt(kLgkmOnly);
    for (int64_t kb = kb0; kb < kb1; kb += 2) {
        block(kb, sA0, sL0, sA1, sL1);
        block(kb + 1, sA1, sL1, sA0, sL0);
    }
    // the last copy (a repeat) must land before the work-group ends
    __builtin_amdgcn_s_waitcnt(0);

    // Epilogue: keep the rows whose label equals the column's group.  The
    // panel's 128 rows are K blocks 2I and 2I + 1, so their labels are copied
    // in the same layout as in the loop: with packed labels into two buffers
    // of their own together with the first K block (their wait then falls on
    // the prologue's, which is exposed anyway: 1% of the kernel at n =
    // 100,000), with u16 labels (no room for two more buffers) into the
    // loop's label buffers once the loop is done.
    if constexpr (!NIB) {
        __syncthreads();                 // every wave is done with the buffers
        stage_labels(2 * I, sL0);
        stage_labels(2 * I + 1, sL1);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    const uint4 *E0 = NIB ? sE0 : sL0, *E1 = NIB ? sE1 : sL1;
#pragma unroll
    for (int nf = 0; nf < NF; nf++) {
        // Derived again from the loop's two registers (an empty asm hides
        // their origin), so nothing else stays live across the K loop.
        int sl = lslot[nf];
        uint32_t gv = gg[nf];
        asm volatile("" : "+v"(sl), "+v"(gv));
        const int slot0 = sl - 4 * half;   // chunk 0 of this permutation
        const uint32_t g = gv & 0xFFFFu;
        uint2 l4[4][4];
#pragma unroll
        for (int rb = 0; rb < 4; rb++) {
            const uint2 *L2 = reinterpret_cast<const uint2 *>(rb < 2 ? E0 : E1);
            const uint32_t *L1 = reinterpret_cast<const uint32_t *>(rb < 2 ? E0 : E1);
#pragma unroll
            for (int a = 0; a < 4; a++) {
                // rows rb*32 + 8a + 4*half + 0..3 of the panel: chunk
                // (rb % 2) * 4 + a of its K block, bytes 8*half .. 8*half + 7
                // (NIB: dword (rb % 2) * 4 + a, bits 16*half .. 16*half + 15)
                if constexpr (NIB)
                    l4[rb][a].x = L1[slot0 + (rb % 2) * 4 + a] >> (16 * half);
                else
                    l4[rb][a] = L2[(slot0 + (rb % 2) * 4 + a) * 2 + half];
            }
        }
        float zs = 0.0f, zn = 0.0f;
#pragma unroll
        for (int rb = 0; rb < 4; rb++) {
#pragma unroll
            for (int a = 0; a < 4; a++) {
                uint32_t lab4[4];
                if constexpr (NIB) {
#pragma unroll
                    for (int b = 0; b < 4; b++) lab4[b] = (l4[rb][a].x >> (4 * b)) & 0xFu;
                } else {
                    lab4[0] = l4[rb][a].x & 0xFFFFu;
                    lab4[1] = l4[rb][a].x >> 16;
                    lab4[2] = l4[rb][a].y & 0xFFFFu;
                    lab4[3] = l4[rb][a].y >> 16;
                }
                const float y4[4] = {acc[rb][nf][4 * a], acc[rb][nf][4 * a + 1],
                                     acc[rb][nf][4 * a + 2], acc[rb][nf][4 * a + 3]};
                masked_pair4(zs, zn, g, (uint32_t)Lg, lab4, y4);
            }
        }
        zs += __shfl_xor(zs, 32);
        const int64_t p = p_lo + slot0 / (NIB ? 8 : kLStride);   // slot0 is in dwords for NIB
        if (cx) {
            zn += __shfl_xor(zn, 32);
            const uint32_t gc = g - (g > (uint32_t)Lg ? 1u : 0u);   // column within p
            if (half == 0 && p < P)
                *reinterpret_cast<float2 *>(&z[((item * P + p) * kcol + gc) * 2]) =
                    make_float2(zs, zn);
        } else if (half == 0 && p < P) {
            z[(item * P + p) * kcol + g] = zs;
        }
    }
}

template <int DT, int NF, int LQ, bool NIB>
__global__ __launch_bounds__(256) void k_mfma(
    const uint4 *__restrict__ tiles, int64_t comp_units, int64_t kb_total,
    const int32_t *__restrict__ tab, int64_t grid_real, int64_t nblocks,
    const uint16_t *__restrict__ lab, const uint32_t *__restrict__ lab4, int64_t n_pad, int cx,
    int32_t kcol, const int32_t *__restrict__ Lp, int64_t P, float *__restrict__ z) {
    const int64_t gpad = gridDim.x;
    const int64_t bid = blockIdx.x;
    const int64_t logical = (bid & 7) * (gpad >> 3) + (bid >> 3);
    if (logical >= grid_real) return;
    const int32_t Lg = cx ? *Lp : 0;
    mfma_unit<DT, NF, LQ, NIB>(tiles, comp_units, kb_total, tab, logical / nblocks,
                               logical % nblocks, lab, lab4, n_pad, cx != 0, kcol, Lg, P, z);
}

// Label-copy rounds for the permutations that COLS columns of k columns per
// grouping can touch ((COLS - 1) / k + 2, 9 slots each, 256 per round),
// rounded up to the instantiated counts.
constexpr int kLqBins[5] = {2, 4, 5, 7, 10};
// Static LDS of k_mfma<DT, NF, LQ, NIB>: two buffers of A (one 16 KB block
// per component) and two of labels, with packed labels two more for the
// epilogue's; gfx950 gives a work-group 160 KB.
constexpr bool mfma_lds_fits(int dt, int nf, int lq, bool nib = false) {
    (void)nf;
    return 2 * (dt == 3 ? 3 : dt == 2 ? 2 : 1) * kUnitU4 * 16 + (nib ? 4 : 2) * lq * 256 * 16 <=
           160 * 1024;
}
int lq_bin(int cols, int32_t k) {
    const int64_t need = ceil_div(((int64_t)(cols - 1) / k + 2) * 9, 256);
    for (int b : kLqBins)
        if (need <= b) return b;
    return -1;
}
// The same for labels packed four bits each (2 slots per permutation).  The
// copy shrinks by 4.5x (at k = 3, 512 columns: 257 permutations, 37 KB of u16
// labels per K block beside 32 KB of A); the one-hot work grows from three
// to four operations per dword.  Measured on one device: n = 100,000, k = 3
// 30.9 ms against 34.0; n = 10,000, k = 5 6.15 ms against 6.25.
constexpr int kLqNibBins[3] = {1, 2, 3};
static_assert(mfma_lds_fits(2, 4, 3, true) && mfma_lds_fits(0, 4, 3, true),
              "packed-label kernels fit in LDS");
int lq_bin_nib(int cols, int32_t k) {
    const int64_t need = ceil_div(((int64_t)(cols - 1) / k + 2) * 2, 256);
    for (int b : kLqNibBins)
        if (need <= b) return b;
    return -1;
}

// Work-list form (serving): block b runs unit units[b] = (job, item, column
// block) of a split-BF16 job in the job table; NF = 4 for the jobs planned
// with 512 columns per work-group, 2 for those with 256 (labels staged for
// any number of columns per grouping those plans allow).
template <int NF>
__global__ __launch_bounds__(256) void k_mfma_worklist(const JobDesc *__restrict__ jobs,
                                                      const UnitDesc *__restrict__ units,
                                                      const int32_t *__restrict__ count) {
    const int64_t gpad = gridDim.x;
    const int64_t bid = blockIdx.x;
    const int64_t logical = (bid & 7) * (gpad >> 3) + (bid >> 3);
    if (logical >= *count) return;
    const UnitDesc u = units[logical];
    const JobDesc &j = jobs[u.job];
    const bool cx = j.cx != 0;
    mfma_unit<2, NF, 10, false>((const uint4 *)j.tiles, j.comp_units, j.kb_total, j.tab, u.chunk,
                         u.pgroup, j.lab_pm, nullptr, j.n_pad_m, cx, cx ? j.k - 1 : j.k, cx ? *j.Lp : 0,
                         j.R, j.z);
}

} // namespace

size_t mfma_tile_bytes(int64_t n, int dtype) {
    const int64_t panels = ceil_div(n, kPanel);
    const int64_t units = panels * (panels + 1);
    // FP16: one 256-byte slot after the tiles for the scale cell
    return (size_t)units * kUnitU4 * 16 * (dtype == 3 ? 3 : dtype == 2 ? 2 : 1) +
           (dtype == 1 ? 256 : 0);
}

const uint32_t *f16_max_cell(const void *tiles, int64_t n) {
    return (const uint32_t *)((const char *)tiles + mfma_tile_bytes(n, 1) - 256);
}

MfmaPlan mfma_plan(int64_t n, int64_t P, int32_t k, int dtype, int kchunk_cols, int ncols,
                   int n_cu, bool cx) {
    (void)n_cu;
    MfmaPlan pl{};
    pl.dtype = dtype;
    pl.n_pad = round_up(n, kPanel);
    pl.panels = pl.n_pad / kPanel;
    pl.kb_total = pl.n_pad / kKBlock;
    // Default K chunk: 2,048 columns from 128 to 1,023 row panels (16,256 <
    // n <= 130,944), where halving the per-item epilogues outweighs the FP64
    // recheck of the few more near ties the longer FP32 sums bring (whole
    // tests at n = 25,000 and 100,000: 4% and 3% faster); 1,536 from 64 to
    // 127 panels (8,064 < n <= 16,256; at n = 10,000 2% faster than 1,024,
    // 2,048 slower again); else 1,024: at n = 229,376 the wider band doubled
    // the near ties (49 against 28 groupings rechecked) and their FP64
    // passes cost more than the kernel saved (355 against ~320 ms)
    int64_t kc = kchunk_cols > 0 ? kchunk_cols / kKBlock
                 : pl.panels >= 1024 ? 16
                 : pl.panels >= 128  ? 32
                 : pl.panels >= 64   ? 24
                                     : 16;
    // the kernel takes K blocks in pairs: every item's length is even
    // (each panel's range [2I, kb_total) has even length)
    if (kc < 2) kc = 2;
    kc += kc & 1;
    pl.kchunk = kc;
    int64_t items = 0;
    for (int64_t I = 0; I < pl.panels; I++) items += ceil_div(pl.kb_total - 2 * I, kc);
    pl.items = items;
    pl.ncols = (ncols == 256) ? 256 : 512;
    // The labels of the permutations a work-group's columns touch must fit in
    // LDS beside the A blocks: fewer columns per work-group when they do not
    // (three A components, or one or two columns per permutation), and the
    // full form when not even 256 columns fit.
    auto fits = [&](int cols, int32_t kc) {
        const int lq = lq_bin(cols, kc);
        return lq > 0 && mfma_lds_fits(dtype, cols / 128, lq);
    };
    pl.cx = cx && k >= 2 && (fits(pl.ncols, k - 1) || fits(256, k - 1));
    pl.kcol = pl.cx ? k - 1 : k;
    if (!fits(pl.ncols, pl.kcol)) pl.ncols = 256;
    pl.N = (int64_t)pl.kcol * P;
    pl.nblocks = ceil_div(pl.N > 0 ? pl.N : 1, pl.ncols);
    pl.P_pad = ceil_div(pl.nblocks * pl.ncols, pl.kcol);
    if (pl.P_pad < P) pl.P_pad = P;
    pl.tile_bytes = mfma_tile_bytes(n, dtype);
    return pl;
}

size_t mfma_table_bytes(const MfmaPlan &pl) { return (size_t)pl.items * 3 * sizeof(int32_t); }

void launch_mfma_prepass(const float *mat, int64_t n, int dtype, void *tiles, hipStream_t s,
                         double *sT_part, double *sT, const PrepassRecheck *rc, double *rcs,
                         int packed) {
    const int64_t panels = ceil_div(n, kPanel);
    const int64_t kb_total = panels * 2;
    const int64_t comp_units = panels * (panels + 1);
    // one s_T partial per work-group: no more work-groups than partial slots
    const int64_t blocks = prepass_blocks(n);
    // 16-byte row reads where every row of the square is 16-byte aligned;
    // packed rows start at any element and are read element by element
    // (measured faster than 16/8/4-byte reads chosen by each row's alignment)
    const int vec = !packed && (n % 4 == 0) && ((uintptr_t)mat % 16 == 0);
    const dim3 grid((unsigned)blocks);
    uint4 *t = (uint4 *)tiles;
    const PrepassRecheck none{};
    uint32_t *cell = nullptr;
    if (dtype == 1) {
        cell = const_cast<uint32_t *>(f16_max_cell(tiles, n));
        launch_fill_i32((int32_t *)cell, 1, 0, s);
        const int64_t mb = n < 2048 ? n : 2048;
        hipLaunchKernelGGL(k_max_abs_upper, dim3((unsigned)mb), dim3(256), 0, s, mat, n, cell,
                           packed);
    }
#define PSTAT_PREPASS(DT_, RC_)                                                                   \
    hipLaunchKernelGGL((k_prepass<DT_, RC_>), grid, dim3(256), 0, s, mat, n, kb_total, comp_units, \
                       vec, t, sT_part, rc ? *rc : none, cell, rcs, packed)
    if (rc) {
        if (dtype == 0) PSTAT_PREPASS(0, true);
        else if (dtype == 1) PSTAT_PREPASS(1, true);
        else if (dtype == 3) PSTAT_PREPASS(3, true);
        else PSTAT_PREPASS(2, true);
    } else {
        if (dtype == 0) PSTAT_PREPASS(0, false);
        else if (dtype == 1) PSTAT_PREPASS(1, false);
        else if (dtype == 3) PSTAT_PREPASS(3, false);
        else PSTAT_PREPASS(2, false);
    }
#undef PSTAT_PREPASS
    if (sT_part) launch_sT_final(sT_part, blocks, n, sT, s);
    if (rc) launch_reduce_partials(rc->part, blocks, kRecheckRows, rc->m, rc->out, s);
}

// Work-groups of the pre-pass: what stays resident on the device (two
// per CU), never more than the units or the s_T partial slots.  A function of
// n alone, so every caller reduces the partials in the same order.
constexpr int64_t kPrepassBlocks = 512;
int64_t prepass_blocks(int64_t n) {
    const int64_t panels = ceil_div(n, kPanel);
    const int64_t comp_units = panels * (panels + 1);
    int64_t b = sT_partials_count(n);
    if (b > kPrepassBlocks) b = kPrepassBlocks;
    return b < comp_units ? b : comp_units;
}

template <int DT, int NF, int LQ, bool NIB>
void launch_mfma_t(const MfmaPlan &pl, const uint4 *t, int64_t comp_units, const int32_t *tab,
                   int64_t grid_real, int64_t gpad, const uint16_t *lab, const int32_t *Lp,
                   int64_t P, float *z, hipStream_t s, const uint32_t *lab4 = nullptr) {
    hipLaunchKernelGGL((k_mfma<DT, NF, LQ, NIB>), dim3((unsigned)gpad), dim3(256), 0, s, t,
                       comp_units, pl.kb_total, tab, grid_real, pl.nblocks, lab, lab4, pl.n_pad,
                       pl.cx ? 1 : 0, pl.kcol, Lp, P, z);
}

template <int DT, int NF>
int launch_mfma_lq(const MfmaPlan &pl, const uint4 *t, int64_t comp_units, const int32_t *tab,
                   int64_t grid_real, int64_t gpad, const uint16_t *lab, const int32_t *Lp,
                   int64_t P, float *z, hipStream_t s, const uint32_t *lab4) {
    if constexpr (DT != 3) {
        // labels packed four bits each when the table was given (k <= 15)
        if (lab4) {
            switch (lq_bin_nib(4 * NF * 32, pl.kcol)) {
            case 1: launch_mfma_t<DT, NF, 1, true>(pl, t, comp_units, tab, grid_real, gpad, lab, Lp, P, z, s, lab4); return 0;
            case 2: launch_mfma_t<DT, NF, 2, true>(pl, t, comp_units, tab, grid_real, gpad, lab, Lp, P, z, s, lab4); return 0;
            case 3: launch_mfma_t<DT, NF, 3, true>(pl, t, comp_units, tab, grid_real, gpad, lab, Lp, P, z, s, lab4); return 0;
            }
        }
    }
    switch (lq_bin(4 * NF * 32, pl.kcol)) {
    case 2: launch_mfma_t<DT, NF, 2, false>(pl, t, comp_units, tab, grid_real, gpad, lab, Lp, P, z, s); return 0;
    case 4: launch_mfma_t<DT, NF, 4, false>(pl, t, comp_units, tab, grid_real, gpad, lab, Lp, P, z, s); return 0;
    case 5: launch_mfma_t<DT, NF, 5, false>(pl, t, comp_units, tab, grid_real, gpad, lab, Lp, P, z, s); return 0;
    case 7: launch_mfma_t<DT, NF, 7, false>(pl, t, comp_units, tab, grid_real, gpad, lab, Lp, P, z, s); return 0;
    case 10:
        if constexpr (mfma_lds_fits(DT, NF, 10)) {
            launch_mfma_t<DT, NF, 10, false>(pl, t, comp_units, tab, grid_real, gpad, lab, Lp, P, z, s);
            return 0;
        }
        return -1;
    }
    return -1;
}

int launch_mfma(const MfmaPlan &pl, const void *tiles, int64_t n, const uint16_t *lab_pm,
                int32_t k, int64_t P, int32_t *tab, float *z, hipStream_t s, const int32_t *Lp,
                const uint32_t *lab4) {
    (void)n;
    if (pl.ncols != 256 && pl.ncols != 512) return -1;
    if (k < 2 || (pl.kchunk & 1)) return -1;
    if (pl.cx && (!Lp || pl.kcol != k - 1)) return -1;
    hipLaunchKernelGGL(k_item_table, dim3((unsigned)ceil_div(pl.panels, 256)), dim3(256), 0, s,
                       pl.panels, pl.kb_total, pl.kchunk, tab);
    const int64_t grid_real = pl.items * pl.nblocks;
    const int64_t gpad = round_up(grid_real, 8);
    const int64_t comp_units = pl.panels * (pl.panels + 1);
    const uint4 *t = (const uint4 *)tiles;
#define PSTAT_MFMA_CASE(DT_)                                                                      \
    if (pl.dtype == DT_) {                                                                        \
        if (pl.ncols == 512)                                                                      \
            return launch_mfma_lq<DT_, 4>(pl, t, comp_units, tab, grid_real, gpad, lab_pm, Lp, P, z, \
                                          s, lab4);                                               \
        return launch_mfma_lq<DT_, 2>(pl, t, comp_units, tab, grid_real, gpad, lab_pm, Lp, P, z, s, \
                                      lab4);                                                      \
    }
    PSTAT_MFMA_CASE(0)
    PSTAT_MFMA_CASE(1)
    PSTAT_MFMA_CASE(2)
    PSTAT_MFMA_CASE(3)
#undef PSTAT_MFMA_CASE
    return -1;
}

bool mfma_use_nibbles(const MfmaPlan &pl, int32_t k) {
    return k <= 15 && pl.dtype != 3 && lq_bin_nib(pl.ncols, pl.kcol) > 0;
}
void launch_pack_nibbles(const uint16_t *lab, int64_t count, uint32_t *out, hipStream_t s) {
    const int64_t words = count / 8;
    if (words <= 0) return;
    int64_t blocks = ceil_div(words, 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_pack_nibbles, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const uint4 *)lab, words, out);
}
void launch_mfma_worklist(const JobDesc *jobs, const UnitDesc *units, const int32_t *count,
                          int64_t max_units, hipStream_t s, int ncols) {
    const int64_t gpad = round_up(max_units > 0 ? max_units : 1, 8);
    if (ncols == 256)
        hipLaunchKernelGGL(k_mfma_worklist<2>, dim3((unsigned)gpad), dim3(256), 0, s, jobs, units,
                           count);
    else
        hipLaunchKernelGGL(k_mfma_worklist<4>, dim3((unsigned)gpad), dim3(256), 0, s, jobs, units,
                           count);
}

void launch_item_table(const MfmaPlan &pl, int32_t *tab, hipStream_t s) {
    hipLaunchKernelGGL(k_item_table, dim3((unsigned)ceil_div(pl.panels, 256)), dim3(256), 0, s,
                       pl.panels, pl.kb_total, pl.kchunk, tab);
}

} // namespace pstat
