// FP64 s_W of a few groupings (the tie recheck and the samples of the plain
// forms), in one pass over the strict upper triangle of D for all of them.

#include "internal.h"
#include "lane_mask.h"

namespace pstat {

namespace {

// With only a handful of groupings the lane-per-permutation form leaves most
// lanes idle and re-walks each tile per lane.  Here the lanes run over pairs
// instead: for each 64 x 64 tile of the triangle, each thread takes 16 of its
// pairs (one column, every fourth row), holds their d^2 in FP64 registers, and
// for each of EQ groupings adds the d^2 of its pairs whose two labels agree,
// times that label's weight (Algorithm 1's sum, split by column).  D is read
// once for all EQ groupings.  A pair counts through an add that runs under
// the lane mask of its label compare (two vector operations), and each thread
// keeps one running FP64 sum per grouping over the whole run of tiles; the
// cross-lane sums happen once per work-group.  The D entries and labels of
// the next tile are loaded while the current one is computed.  Every sum has
// a fixed order (rows within a tile, tiles of the run, a butterfly over the
// wave, the four waves in order, then the runs in order), so results are
// reproducible.
constexpr int kFT = 64;               // tile edge
constexpr int64_t kFewChunks = 4096;  // work-groups (tile runs) per launch
constexpr int64_t kFewMaxM = 1024;    // groupings per launch
constexpr int kFewWLds = 1024;        // weights kept in LDS up to this many groups

template <int EQ, typename LT>
__global__ __launch_bounds__(256) void k_sw_few(const float *__restrict__ mat, int64_t n,
                                                int64_t nt, int64_t tiles, int64_t tpc,
                                                const LT *__restrict__ g, int64_t gstride,
                                                const int32_t *__restrict__ rows, int64_t m,
                                                int32_t k, const double *__restrict__ w,
                                                double *__restrict__ partial, int64_t m_pad,
                                                int packed) {
    static_assert(EQ % 2 == 0, "two groupings per label round");
    constexpr int LR = EQ / 2;   // label loads per thread and tile
    // row labels as [grouping][row % 4][row / 4], so the 16 rows of a thread
    // (wave + 4u) are four 16-byte reads; column labels and their weights
    __shared__ __align__(16) int32_t srow[EQ][4][16];
    __shared__ int32_t scol[EQ][kFT];
    __shared__ double swc[EQ][kFT];
    __shared__ double sred[4][EQ];
    __shared__ double sw[kFewWLds];
    const int tid = threadIdx.x;
    const int wave = tid / 64, c = tid % 64;
    // label round r of this thread: grouping wave / 2 + 2r, rows (even waves)
    // or columns (odd waves), tile position c
    const int side = wave % 2;
    const int64_t q0 = (int64_t)blockIdx.y * EQ;
    const bool wl = k <= kFewWLds;
    if (wl)
        for (int e = tid; e < k; e += 256) sw[e] = w[e];
    int64_t gb[LR];
#pragma unroll
    for (int r = 0; r < LR; r++) {
        const int64_t q = q0 + wave / 2 + 2 * r;
        gb[r] = q < m ? (int64_t)rows[q] * gstride : -1;
    }
    double acc[EQ];
#pragma unroll
    for (int q = 0; q < EQ; q++) acc[q] = 0.0;
    const int64_t t0 = (int64_t)blockIdx.x * tpc;
    const int64_t t_end = t0 + tpc < tiles ? t0 + tpc : tiles;

    float dn[16];        // D entries of the next tile (0 off the strict triangle)
    int32_t ln[LR];      // labels of the next tile (padding never matches)
    auto fetch = [&](int64_t t) {
        int64_t I, J;
        tri_decode(t, nt, I, J);
        const int64_t j = J * kFT + c;
        if (I < J && (J + 1) * kFT <= n) {
            // every pair of the tile is in the strict triangle and inside
            // the matrix: one base and fixed row steps, no per-entry test
            // (3.7 ms instead of 4.4 for one pass at n = 100,000)
            const int64_t i0 = I * kFT + wave;
            if (packed) {
#pragma unroll
                for (int u = 0; u < 16; u++) dn[u] = mat[d_index(i0 + 4 * u, j, n, 1)];
            } else {
                const float *b = mat + (uint64_t)i0 * (uint64_t)n + (uint64_t)j;
#pragma unroll
                for (int u = 0; u < 16; u++) dn[u] = b[(uint64_t)(4 * u) * (uint64_t)n];
            }
        } else {
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const int64_t i = I * kFT + wave + 4 * u;
                dn[u] = (j < n && i < j) ? mat[d_index(i, j, n, packed)] : 0.0f;
            }
        }
        const int64_t idx = (side ? J : I) * kFT + c;
#pragma unroll
        for (int r = 0; r < LR; r++)
            ln[r] = (gb[r] >= 0 && idx < n) ? (int32_t)g[gb[r] + idx] : -1 - side;
    };
    if (t0 < t_end) fetch(t0);
    __syncthreads();   // weights in LDS
    for (int64_t t = t0; t < t_end; t++) {
        double d2[16];
#pragma unroll
        for (int u = 0; u < 16; u++) d2[u] = (double)dn[u] * (double)dn[u];
#pragma unroll
        for (int r = 0; r < LR; r++) {
            const int q = wave / 2 + 2 * r;
            const int32_t v = ln[r];
            if (side) {
                scol[q][c] = v;
                swc[q][c] = (v >= 0 && v < k) ? (wl ? sw[v] : w[v]) : 0.0;
            } else {
                srow[q][c % 4][c / 4] = v;
            }
        }
        __syncthreads();
        if (t + 1 < t_end) fetch(t + 1);
#pragma unroll
        for (int q = 0; q < EQ; q++) {
            const int32_t lc = scol[q][c];
            const int4 *rl = reinterpret_cast<const int4 *>(&srow[q][wave][0]);
            uint32_t li[16];
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int4 r4 = rl[v];
                li[4 * v] = r4.x;
                li[4 * v + 1] = r4.y;
                li[4 * v + 2] = r4.z;
                li[4 * v + 3] = r4.w;
            }
            double sum = 0.0;
            masked_add16(sum, (uint32_t)lc, li, d2);
            acc[q] = __builtin_fma(sum, swc[q][c], acc[q]);
        }
        __syncthreads();   // this tile's labels are no longer read
    }
#pragma unroll
    for (int q = 0; q < EQ; q++) {
        double v = acc[q];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
        if (c == 0) sred[wave][q] = v;
    }
    __syncthreads();
    if (tid < EQ && q0 + tid < m)
        partial[(int64_t)blockIdx.x * m_pad + q0 + tid] =
            ((sred[0][tid] + sred[1][tid]) + sred[2][tid]) + sred[3][tid];
}

// out[q] = sum over runs, in a fixed order, of partial[run][q]: one
// work-group per grouping, strided partial sums then a tree in LDS.
__global__ __launch_bounds__(256) void k_reduce_few(const double *__restrict__ partial,
                                                    int64_t runs, int64_t m_pad,
                                                    double *__restrict__ out) {
    __shared__ double sh[256];
    const int64_t q = blockIdx.x;
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < runs; t += 256) s += partial[t * m_pad + q];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = sh[0];
}

} // namespace
} // namespace pstat

namespace pstat {

size_t few_partial_bytes(int64_t n, int64_t m) {
    const int64_t nt = ceil_div(n, kFT);
    const int64_t tiles = nt * (nt + 1) / 2;
    const int64_t runs = tiles < kFewChunks ? tiles : kFewChunks;
    const int64_t mm = m < kFewMaxM ? (m > 0 ? m : 1) : kFewMaxM;
    return (size_t)runs * (size_t)round_up(mm, 8) * sizeof(double);
}

namespace {
template <typename LT>
void sw_few_t(const float *mat, int64_t n, const LT *g, int64_t gstride, const int32_t *rows,
              int64_t m, int32_t k, const double *w, double *partial, double *out, hipStream_t s,
              int packed) {
    const int64_t nt = ceil_div(n, kFT);
    const int64_t tiles = nt * (nt + 1) / 2;
    const int64_t runs = tiles < kFewChunks ? tiles : kFewChunks;
    const int64_t tpc = ceil_div(tiles, runs);
    const int64_t used = ceil_div(tiles, tpc);
    for (int64_t b = 0; b < m; b += kFewMaxM) {
        const int64_t mm = m - b < kFewMaxM ? m - b : kFewMaxM;
        const int64_t m_pad = round_up(mm, 8);
        // whole groups of 16 groupings in one launch (one work-group row
        // each), the rest with the narrowest instance that holds it
        const int64_t full = mm > 16 ? mm / 16 : 0, rest = mm - 16 * full;
        if (full > 0)
            hipLaunchKernelGGL((k_sw_few<16, LT>), dim3((unsigned)used, (unsigned)full), dim3(256),
                               0, s, mat, n, nt, tiles, tpc, g, gstride, rows + b, 16 * full, k, w,
                               partial, m_pad, packed);
        const int32_t *rr = rows + b + 16 * full;
        double *pr = partial + 16 * full;
        if (rest == 0) {
        } else if (rest <= 4) {
            hipLaunchKernelGGL((k_sw_few<4, LT>), dim3((unsigned)used, 1), dim3(256), 0, s, mat, n,
                               nt, tiles, tpc, g, gstride, rr, rest, k, w, pr, m_pad, packed);
        } else if (rest <= 8) {
            hipLaunchKernelGGL((k_sw_few<8, LT>), dim3((unsigned)used, 1), dim3(256), 0, s, mat, n,
                               nt, tiles, tpc, g, gstride, rr, rest, k, w, pr, m_pad, packed);
        } else if (rest <= 12) {
            hipLaunchKernelGGL((k_sw_few<12, LT>), dim3((unsigned)used, 1), dim3(256), 0, s, mat,
                               n, nt, tiles, tpc, g, gstride, rr, rest, k, w, pr, m_pad, packed);
        } else {
            hipLaunchKernelGGL((k_sw_few<16, LT>), dim3((unsigned)used, 1), dim3(256), 0, s, mat,
                               n, nt, tiles, tpc, g, gstride, rr, rest, k, w, pr, m_pad, packed);
        }
        hipLaunchKernelGGL(k_reduce_few, dim3((unsigned)mm), dim3(256), 0, s, partial, used, m_pad,
                           out + b);
    }
}
} // namespace

void launch_reduce_partials(const double *partial, int64_t runs, int64_t stride, int64_t m,
                            double *out, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_reduce_few, dim3((unsigned)m), dim3(256), 0, s, partial, runs, stride, out);
}

void launch_sw_few(const float *mat, int64_t n, const int32_t *g, const int32_t *rows, int64_t m,
                   int32_t k, const double *w, double *partial, double *out, hipStream_t s,
                   int packed) {
    sw_few_t(mat, n, g, n, rows, m, k, w, partial, out, s, packed);
}

void launch_sw_few_u16(const float *mat, int64_t n, const uint16_t *g, int64_t stride,
                       const int32_t *rows, int64_t m, int32_t k, const double *w, double *partial,
                       double *out, hipStream_t s, int packed) {
    sw_few_t(mat, n, g, stride, rows, m, k, w, partial, out, s, packed);
}

} // namespace pstat
