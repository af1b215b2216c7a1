// Dense-contraction (MFMA) form of s_W.
//
// With U the strict upper triangle of D∘D (u_ij = d_ij^2 for j > i, else 0) and
// G_p the n x k one-hot matrix of permutation p's labels,
//     s_W[p] = sum_g w_g (G_p^T U G_p)_gg,
// which is exactly Algorithm 1's sum (section 2) regrouped: (G^T U G)_gg adds
// u_ij over the pairs i < j that both carry label g.  G is 0/1, so it is exact
// in any input type; only U is rounded (to BF16, FP16, or BF16 hi + BF16 lo).
//
// Blocking.  Rows are cut into 128-row panels and columns into 64-column K
// blocks.  A pre-pass writes, for each panel I, its K blocks from the diagonal
// (block 2I) to the end, each as 128 x 64 values in MFMA fragment order, with
// the entries j <= i of the diagonal blocks set to zero.  The main kernel
// computes Y = U_panel * G over a K range for 256 or 512 columns (p, g) of G at
// a time with v_mfma_f32_32x32x16_{bf16,f16} (FP32 accumulation), staging the
// K blocks of U in LDS and building the one-hot B fragments in registers from
// u16 labels, and in its epilogue keeps
// for each column (p, g) only the rows i whose label is g:
//     z[item][p][g] = sum_{i in panel, g_p(i) = g} Y[i][(p, g)].
// Each (panel, K chunk) work item writes its own z; they are summed in FP64 and
// weighted by w_g in FP64 afterwards, so FP32 only ever accumulates one K
// chunk.
#include <hip/hip_bf16.h>

#include "internal.h"

namespace pstat {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kPanel = 128;      // rows per panel
constexpr int kKBlock = 64;      // columns per K block
constexpr int kUnitU4 = 1024;    // uint4 per (panel, K block) unit per component (16 KB)

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
// Block (kb, I): unit (I, kb) for kb >= 2I.  Stages the 128 x 64 FP32 block in
// LDS (coalesced row reads), then writes 1024 uint4 per component in fragment
// order: uint4 index ((rb * 4 + s) * 64 + lane) holds row rb*32 + lane%32,
// columns 32*(lane/32) + 8*s + 0..7 of the block.
template <int DT>
__global__ __launch_bounds__(256) void k_prepass(const float *__restrict__ mat, int64_t n,
                                                 int64_t kb_total, int64_t comp_units,
                                                 uint4 *__restrict__ tiles) {
    const int64_t kb = blockIdx.x, I = blockIdx.y;
    if (kb < 2 * I) return;
    __shared__ float sm[kPanel][kKBlock + 1];
    const int tid = threadIdx.x;
    const int64_t r0 = I * kPanel, c0 = kb * kKBlock;
    for (int idx = tid; idx < kPanel * kKBlock; idx += 256) {
        const int r = idx / kKBlock, c = idx % kKBlock;
        const int64_t i = r0 + r, j = c0 + c;
        float x = 0.0f;
        if (i < n && j < n && j > i) {
            const float d = mat[(uint64_t)i * (uint64_t)n + j];
            x = d * d;
        }
        sm[r][c] = x;
    }
    __syncthreads();
    const int64_t unit = I * kb_total - I * (I - 1) + (kb - 2 * I);
    for (int q = 0; q < 4; q++) {
        const int idx = tid + 256 * q;
        const int rb = idx / 256, s = (idx / 64) % 4, lane = idx % 64;
        const int r = rb * 32 + (lane % 32);
        const int cb = 32 * (lane / 32) + 8 * s;
        uint32_t hw[4], lw[4];
        for (int e2 = 0; e2 < 4; e2++) {
            const float x0 = sm[r][cb + 2 * e2], x1 = sm[r][cb + 2 * e2 + 1];
            if (DT == 1) {
                hw[e2] = (uint32_t)to_f16_bits(x0) | ((uint32_t)to_f16_bits(x1) << 16);
            } else {
                const uint16_t h0 = to_bf16_bits(x0), h1 = to_bf16_bits(x1);
                hw[e2] = (uint32_t)h0 | ((uint32_t)h1 << 16);
                if (DT == 2) {
                    const uint16_t l0 = to_bf16_bits(x0 - bf16_bits_to_float(h0));
                    const uint16_t l1 = to_bf16_bits(x1 - bf16_bits_to_float(h1));
                    lw[e2] = (uint32_t)l0 | ((uint32_t)l1 << 16);
                }
            }
        }
        tiles[unit * kUnitU4 + idx] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
        if (DT == 2)
            tiles[(comp_units + unit) * kUnitU4 + idx] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    }
}

// ---- work items ---------------------------------------------------------------
// tab[3*item] = panel I, tab[3*item+1] = first K block, tab[3*item+2] = end.
__global__ void k_item_table(int64_t panels, int64_t kb_total, int64_t kchunk,
                             int32_t *__restrict__ tab) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t it = 0;
    for (int64_t I = 0; I < panels; I++) {
        for (int64_t kb = 2 * I; kb < kb_total; kb += kchunk) {
            const int64_t e = kb + kchunk < kb_total ? kb + kchunk : kb_total;
            tab[3 * it] = (int32_t)I;
            tab[3 * it + 1] = (int32_t)kb;
            tab[3 * it + 2] = (int32_t)e;
            it++;
        }
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

template <int DT>
__device__ inline f32x16 mma(uint4 a, uint4 b, f32x16 c) {
    if (DT == 1)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// DT: 0 bf16, 1 f16, 2 split bf16 (hi and lo MFMAs into one accumulator).
// NF: 32-column fragments per wave; a work-group of 4 waves covers 128 rows x
// (4 * NF * 32) columns.  The K blocks of A (the pre-squared tiles) are staged
// once per work-group in double-buffered LDS and read by all four waves; each
// wave builds its own one-hot B fragments from u16 labels, one K step ahead.
template <int DT, int NF>
__device__ __attribute__((always_inline)) inline void mfma_unit(const uint4 *__restrict__ tiles, int64_t comp_units,
                                 int64_t kb_total, const int32_t *__restrict__ tab, int64_t item,
                                 int64_t nb, const uint16_t *__restrict__ lab, int64_t n_pad,
                                 int32_t k, int64_t P, float *__restrict__ z) {
    constexpr int BT = DT == 1 ? 1 : 0;     // operand type of the MFMA
    constexpr int NC = DT == 2 ? 2 : 1;     // A components (hi, lo)
    constexpr int UNIT = NC * kUnitU4;      // uint4 of one staged K block
    constexpr int COLS = 4 * NF * 32;       // columns per work-group
    __shared__ uint4 sA[2][UNIT];
    const int64_t I = tab[3 * item], kb0 = tab[3 * item + 1], kb1 = tab[3 * item + 2];
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int half = lane / 32, col = lane % 32;
    const int64_t NK = (int64_t)k * P;

    int64_t cidx[NF], pcol[NF];
    int32_t gcol[NF];
    uint32_t gg[NF];
    const uint16_t *labrow[NF];
#pragma unroll
    for (int nf = 0; nf < NF; nf++) {
        cidx[nf] = nb * COLS + wave * (NF * 32) + nf * 32 + col;
        pcol[nf] = cidx[nf] / k;
        gcol[nf] = (int32_t)(cidx[nf] % k);
        gg[nf] = (uint32_t)gcol[nf] | ((uint32_t)gcol[nf] << 16);
        labrow[nf] = lab + pcol[nf] * n_pad + 32 * half;
    }

    f32x16 acc[4][NF];
#pragma unroll
    for (int rb = 0; rb < 4; rb++)
#pragma unroll
        for (int nf = 0; nf < NF; nf++)
#pragma unroll
            for (int v = 0; v < 16; v++) acc[rb][nf][v] = 0.0f;

    const int64_t panel_off = I * kb_total - I * (I - 1);
    // Direct global -> LDS copy of one staged K block: lane l of wave w moves
    // uint4 number q*256 + 64w + l of the block (both sides in fragment order).
    auto stage = [&](int64_t kb, int buf) {
#pragma unroll
        for (int q = 0; q < UNIT / 256; q++) {
            const uint4 *src = tiles + ((int64_t)(q / 4) * comp_units + panel_off + (kb - 2 * I)) *
                                           kUnitU4 + (q % 4) * 256 + tid;
            __builtin_amdgcn_global_load_lds(
                (__attribute__((address_space(1))) void *)src,
                (__attribute__((address_space(3))) void *)&sA[buf][q * 256 + wave * 64], 16, 0, 0);
        }
    };
    stage(kb0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    uint4 L[NF];
#pragma unroll
    for (int nf = 0; nf < NF; nf++) L[nf] = *(const uint4 *)(labrow[nf] + kb0 * kKBlock);

    for (int64_t kb = kb0; kb < kb1; kb++) {
        const int buf = (int)((kb - kb0) & 1);
        const bool more = kb + 1 < kb1;
        // The other buffer was last read before the previous barrier.
        if (more) stage(kb + 1, buf ^ 1);
#pragma unroll
        for (int s = 0; s < 4; s++) {
            uint4 B[NF];
#pragma unroll
            for (int nf = 0; nf < NF; nf++) B[nf] = onehot8<BT>(L[nf], gg[nf]);
            // labels of the next K step (or the next K block's first step)
            if (s < 3) {
#pragma unroll
                for (int nf = 0; nf < NF; nf++)
                    L[nf] = *(const uint4 *)(labrow[nf] + kb * kKBlock + 8 * (s + 1));
            } else if (more) {
#pragma unroll
                for (int nf = 0; nf < NF; nf++)
                    L[nf] = *(const uint4 *)(labrow[nf] + (kb + 1) * kKBlock);
            }
#pragma unroll
            for (int rb = 0; rb < 4; rb++) {
#pragma unroll
                for (int c = 0; c < NC; c++) {
                    const uint4 A = sA[buf][c * kUnitU4 + (rb * 4 + s) * 64 + lane];
#pragma unroll
                    for (int nf = 0; nf < NF; nf++) acc[rb][nf] = mma<BT>(A, B[nf], acc[rb][nf]);
                }
            }
        }
        // the next block's copy has landed in LDS for every wave
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }

    // Epilogue: keep the rows whose label equals the column's group.
    const int64_t i0 = I * kPanel;
#pragma unroll
    for (int nf = 0; nf < NF; nf++) {
        const uint16_t *lr = lab + pcol[nf] * n_pad + i0;
        float zs = 0.0f;
#pragma unroll
        for (int rb = 0; rb < 4; rb++) {
#pragma unroll
            for (int a = 0; a < 4; a++) {
                // rows rb*32 + 8a + 4*half + 0..3 of the panel
                const uint2 l4 = *(const uint2 *)(lr + rb * 32 + 8 * a + 4 * half);
                const uint32_t lab4[4] = {l4.x & 0xFFFFu, l4.x >> 16, l4.y & 0xFFFFu, l4.y >> 16};
#pragma unroll
                for (int b = 0; b < 4; b++)
                    zs += (lab4[b] == (uint32_t)gcol[nf]) ? acc[rb][nf][4 * a + b] : 0.0f;
            }
        }
        zs += __shfl_xor(zs, 32);
        if (half == 0 && cidx[nf] < NK) z[(item * P + pcol[nf]) * k + gcol[nf]] = zs;
    }
}

template <int DT, int NF>
__global__ __launch_bounds__(256) void k_mfma(
    const uint4 *__restrict__ tiles, int64_t comp_units, int64_t kb_total,
    const int32_t *__restrict__ tab, int64_t grid_real, int64_t nblocks,
    const uint16_t *__restrict__ lab, int64_t n_pad, int32_t k, int64_t P,
    float *__restrict__ z) {
    const int64_t gpad = gridDim.x;
    const int64_t bid = blockIdx.x;
    const int64_t logical = (bid & 7) * (gpad >> 3) + (bid >> 3);
    if (logical >= grid_real) return;
    mfma_unit<DT, NF>(tiles, comp_units, kb_total, tab, logical / nblocks, logical % nblocks,
                      lab, n_pad, k, P, z);
}

// Work-list form (serving): block b runs unit units[b] = (job, item, column
// block) of a split-BF16 job in the job table.
__global__ __launch_bounds__(256) void k_mfma_worklist(const JobDesc *__restrict__ jobs,
                                                      const UnitDesc *__restrict__ units,
                                                      const int32_t *__restrict__ count) {
    const int64_t gpad = gridDim.x;
    const int64_t bid = blockIdx.x;
    const int64_t logical = (bid & 7) * (gpad >> 3) + (bid >> 3);
    if (logical >= *count) return;
    const UnitDesc u = units[logical];
    const JobDesc &j = jobs[u.job];
    mfma_unit<2, 4>((const uint4 *)j.tiles, j.comp_units, j.kb_total, j.tab, u.chunk, u.pgroup,
                    j.lab_pm, j.n_pad_m, j.k, j.R, j.z);
}

} // namespace

size_t mfma_tile_bytes(int64_t n, int dtype) {
    const int64_t panels = ceil_div(n, kPanel);
    const int64_t units = panels * (panels + 1);
    return (size_t)units * kUnitU4 * 16 * (dtype == 2 ? 2 : 1);
}

MfmaPlan mfma_plan(int64_t n, int64_t P, int32_t k, int dtype, int kchunk_cols, int ncols,
                   int n_cu) {
    (void)n_cu;
    MfmaPlan pl{};
    pl.dtype = dtype;
    pl.n_pad = round_up(n, kPanel);
    pl.panels = pl.n_pad / kPanel;
    pl.kb_total = pl.n_pad / kKBlock;
    int64_t kc = kchunk_cols > 0 ? kchunk_cols / kKBlock : 16;
    if (kc < 1) kc = 1;
    pl.kchunk = kc;
    int64_t items = 0;
    for (int64_t I = 0; I < pl.panels; I++) items += ceil_div(pl.kb_total - 2 * I, kc);
    pl.items = items;
    pl.ncols = (ncols == 256) ? 256 : 512;
    pl.N = (int64_t)k * P;
    pl.nblocks = ceil_div(pl.N > 0 ? pl.N : 1, pl.ncols);
    pl.P_pad = ceil_div(pl.nblocks * pl.ncols, k);
    if (pl.P_pad < P) pl.P_pad = P;
    pl.tile_bytes = mfma_tile_bytes(n, dtype);
    return pl;
}

size_t mfma_table_bytes(const MfmaPlan &pl) { return (size_t)pl.items * 3 * sizeof(int32_t); }

void launch_mfma_prepass(const float *mat, int64_t n, int dtype, void *tiles, hipStream_t s) {
    const int64_t panels = ceil_div(n, kPanel);
    const int64_t kb_total = panels * 2;
    const int64_t comp_units = panels * (panels + 1);
    dim3 grid((unsigned)kb_total, (unsigned)panels);
    uint4 *t = (uint4 *)tiles;
    if (dtype == 0) hipLaunchKernelGGL(k_prepass<0>, grid, dim3(256), 0, s, mat, n, kb_total, comp_units, t);
    else if (dtype == 1) hipLaunchKernelGGL(k_prepass<1>, grid, dim3(256), 0, s, mat, n, kb_total, comp_units, t);
    else hipLaunchKernelGGL(k_prepass<2>, grid, dim3(256), 0, s, mat, n, kb_total, comp_units, t);
}

template <int DT, int NF>
void launch_mfma_t(const MfmaPlan &pl, const uint4 *t, int64_t comp_units, const int32_t *tab,
                   int64_t grid_real, int64_t gpad, const uint16_t *lab, int32_t k, int64_t P,
                   float *z, hipStream_t s) {
    hipLaunchKernelGGL((k_mfma<DT, NF>), dim3((unsigned)gpad), dim3(256), 0, s, t, comp_units,
                       pl.kb_total, tab, grid_real, pl.nblocks, lab, pl.n_pad, k, P, z);
}

int launch_mfma(const MfmaPlan &pl, const void *tiles, int64_t n, const uint16_t *lab_pm,
                int32_t k, int64_t P, int32_t *tab, float *z, hipStream_t s) {
    (void)n;
    if (pl.ncols != 256 && pl.ncols != 512) return -1;
    hipLaunchKernelGGL(k_item_table, dim3(1), dim3(64), 0, s, pl.panels, pl.kb_total, pl.kchunk, tab);
    const int64_t grid_real = pl.items * pl.nblocks;
    const int64_t gpad = round_up(grid_real, 8);
    const int64_t comp_units = pl.panels * (pl.panels + 1);
    const uint4 *t = (const uint4 *)tiles;
#define PSTAT_MFMA_CASE(DT_)                                                                   \
    if (pl.dtype == DT_) {                                                                     \
        if (pl.ncols == 512)                                                                   \
            launch_mfma_t<DT_, 4>(pl, t, comp_units, tab, grid_real, gpad, lab_pm, k, P, z, s); \
        else                                                                                   \
            launch_mfma_t<DT_, 2>(pl, t, comp_units, tab, grid_real, gpad, lab_pm, k, P, z, s); \
        return 0;                                                                              \
    }
    PSTAT_MFMA_CASE(0)
    PSTAT_MFMA_CASE(1)
    PSTAT_MFMA_CASE(2)
#undef PSTAT_MFMA_CASE
    return -1;
}

void launch_mfma_worklist(const JobDesc *jobs, const UnitDesc *units, const int32_t *count,
                          int64_t max_units, hipStream_t s) {
    const int64_t gpad = round_up(max_units > 0 ? max_units : 1, 8);
    hipLaunchKernelGGL(k_mfma_worklist, dim3((unsigned)gpad), dim3(256), 0, s, jobs, units, count);
}

void launch_item_table(const MfmaPlan &pl, int32_t *tab, hipStream_t s) {
    hipLaunchKernelGGL(k_item_table, dim3(1), dim3(64), 0, s, pl.panels, pl.kb_total, pl.kchunk, tab);
}

} // namespace pstat
