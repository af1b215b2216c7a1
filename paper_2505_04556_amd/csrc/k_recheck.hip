// FP64 s_W of a few groupings (the tie recheck and the samples of the plain
// forms), in one pass over the strict upper triangle of D for all of them.

#include "internal.h"
#include "lane_mask.h"

namespace pstat {

namespace {

// With only a handful of groupings the lane-per-permutation form leaves most
// lanes idle and re-walks each tile per lane.  Here the lanes run over pairs
// instead: the strict upper triangle is cut into 64 x 64 tiles, each
// work-group takes a run of consecutive tiles, and each of its four waves
// takes one 16-row strip of every tile: a lane holds the d^2 of its column's
// 16 pairs in FP64 registers and, for each of EQ groupings, adds those whose
// two labels agree, times that label's weight (Algorithm 1's sum, split by
// column).  D is read once for all EQ groupings.  A pair counts through an
// add that runs under the lane mask of its label compare (two vector
// operations), and each lane keeps one running FP64 sum per grouping over the
// whole run; the cross-lane sums happen once per work-group.  The waves share
// nothing inside the loop: a wave keeps the row labels of its own strip in a
// slice of LDS that only it reads (restaged when the run moves to the next
// tile row), loads the column labels of its lanes itself, and steps from
// tile to tile by counting, so there is no barrier per tile and the waves of
// a CU drift freely between loads and arithmetic.  The D entries and column
// labels of the next tile are loaded while the current one is computed, and
// nothing waits on a global load in between: the weights come from LDS
// (WL), or, for more groups than LDS holds, are loaded for the current tile
// before the next tile's loads are issued.  Every sum has a fixed order
// (rows within a strip, tiles of the run, a butterfly over the wave, the four
// waves in order, then the runs in order), so results are reproducible.
constexpr int kFT = 64;               // tile edge
constexpr int kStrip = 16;            // rows per wave and tile
constexpr int64_t kFewChunks = 4096;  // work-groups (tile runs) per launch
constexpr int64_t kFewMaxM = 1024;    // groupings per launch
constexpr int kFewWLds = 1024;        // weights kept in LDS up to this many groups

template <int EQ, typename LT, bool WL>
__global__ __launch_bounds__(256) void k_sw_few(const float *__restrict__ mat, int64_t n,
                                                int64_t nt, int64_t tiles, int64_t tpc,
                                                const LT *__restrict__ g, int64_t gstride,
                                                const int32_t *__restrict__ rows, int64_t m,
                                                int32_t k, const double *__restrict__ w,
                                                double *__restrict__ partial, int64_t m_pad,
                                                int packed) {
    static_assert(EQ % 4 == 0, "a wave stages 16 row labels of 4 groupings per load");
    // row labels of each wave's strip as [wave][grouping][row]: 16 per
    // grouping, four 16-byte reads
    __shared__ __align__(16) uint32_t srow[4][EQ][kStrip];
    __shared__ double sred[4][EQ];
    __shared__ double sw[WL ? kFewWLds : 1];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64), c = tid % 64;
    const int64_t q0 = (int64_t)blockIdx.y * EQ;
    if constexpr (WL)
        for (int e = tid; e < k; e += 256) sw[e] = w[e];
    // Label rows of the EQ groupings (groupings past m repeat the first: their
    // sums are computed and dropped).  Label reads clamp the index into the
    // matrix: an entry past the edge has d = 0, so its label never counts.
    int64_t gq[EQ];
#pragma unroll
    for (int q = 0; q < EQ; q++) gq[q] = (int64_t)rows[q0 + q < m ? q0 + q : q0] * gstride;
    double acc[EQ];
#pragma unroll
    for (int q = 0; q < EQ; q++) acc[q] = 0.0;
    const int64_t t0 = (int64_t)blockIdx.x * tpc;
    const int64_t t_end = t0 + tpc < tiles ? t0 + tpc : tiles;
    __syncthreads();   // weights in LDS

    // Every load below is unconditional (masked values are fixed up when
    // they are used): a load under a branch makes the compiler wait for all
    // loads in flight, the next tile's included.  Tiles alternate between
    // two register buffers (the loop is unrolled by two), so no register is
    // copied between a load and its use.
    struct Buf {
        float dn[kStrip];   // D entries of the tile
        uint32_t ln[EQ];    // column labels of the tile
        uint32_t mk;        // edge tile: the lane's valid rows (bit u)
        bool edge;          // the tile has entries off the strict triangle
        int64_t I;          // tile row
        double wg[WL ? 1 : EQ];   // global weights of the column labels
    };
    auto fetch = [&](Buf &b, int64_t I, int64_t J) {
        const int64_t j = J * kFT + c;
        const int64_t i0 = I * kFT + kStrip * wave;
        b.I = I;
        b.edge = !(I < J && (J + 1) * kFT <= n);
        if (!b.edge) {
            // every pair of the strip is in the strict triangle and inside
            // the matrix: addresses as a wave-uniform base (the strip's first
            // row at column J * 64) plus 32-bit offsets.  Row i0 + u starts
            // u * n elements after row i0 in the square layout, and
            // u (n - i0 - 2) - u (u - 1) / 2 after it in the packed one (row
            // i holds n - i - 1 entries); both stay below 16 n, far inside
            // 32 bits.
            const char *base =
                reinterpret_cast<const char *>(mat + d_index(i0, J * kFT, n, packed));
            const uint32_t lane_b = 4u * (uint32_t)c;
            const uint32_t rstep = packed ? (uint32_t)(n - i0 - 2) : (uint32_t)n;
#pragma unroll
            for (int u = 0; u < kStrip; u++) {
                const uint32_t off =
                    (uint32_t)u * rstep - (packed ? (uint32_t)(u * (u - 1) / 2) : 0u);
                b.dn[u] = *reinterpret_cast<const float *>(base + (4u * off + lane_b));
            }
        } else {
            // the diagonal tile or the last tile column: entries off the
            // strict triangle or outside the matrix read element 0 instead
            // and are zeroed when used
            b.mk = 0;
#pragma unroll
            for (int u = 0; u < kStrip; u++) {
                const int64_t i = i0 + u;
                const bool in = j < n && i < j;
                b.mk |= (uint32_t)in << u;
                b.dn[u] = mat[in ? d_index(i, j, n, packed) : 0];
            }
        }
        const int64_t jc = j < n ? j : n - 1;
#pragma unroll
        for (int q = 0; q < EQ; q++) b.ln[q] = (uint32_t)g[gq[q] + jc];
    };
    // weight of label v (0 for anything not below k)
    auto weight = [&](uint32_t v, double wv) { return v < (uint32_t)k ? wv : 0.0; };
    // With the weights in global memory, a tile's weights are loaded before
    // the next tile's loads are issued: waiting for them must not also wait
    // for those.
    auto prep = [&](Buf &b) {
        if constexpr (!WL) {
#pragma unroll
            for (int q = 0; q < EQ; q++) {
                const uint32_t v = b.ln[q];
                b.wg[q] = weight(v, w[v < (uint32_t)k ? v : 0u]);
            }
        }
    };
    // the 16 x EQ row labels of this wave's strip of tile row I, four
    // groupings per load round (lane c: grouping 4r + c / 16, row c % 16)
    int64_t Ir = -1;
    auto stage_rows = [&](int64_t I) {
        int64_t i = I * kFT + kStrip * wave + c % kStrip;
        if (i > n - 1) i = n - 1;
#pragma unroll
        for (int r = 0; r < EQ / 4; r++) {
            // the lane's grouping differs across the wave: its row index is
            // loaded per lane (a table of the uniform gq would be indexed
            // per lane, i.e. kept in scratch memory)
            const int64_t q = q0 + 4 * r + c / kStrip;
            const int64_t base = (int64_t)rows[q < m ? q : q0] * gstride;
            srow[wave][4 * r + c / kStrip][c % kStrip] = (uint32_t)g[base + i];
        }
        // only this wave reads the slice: order its writes before the reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    auto compute = [&](Buf &b) {
        if (b.I != Ir) {
            stage_rows(b.I);
            Ir = b.I;
        }
        if (b.edge) {
#pragma unroll
            for (int u = 0; u < kStrip; u++)
                if (!((b.mk >> u) & 1u)) b.dn[u] = 0.0f;
        }
        double d2[kStrip];
#pragma unroll
        for (int u = 0; u < kStrip; u++) d2[u] = (double)b.dn[u] * (double)b.dn[u];
        static_assert(EQ % 2 == 0, "groupings in pairs");
#pragma unroll
        for (int q = 0; q < EQ; q += 2) {
            uint32_t li[2][kStrip];
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const uint4 *rl = reinterpret_cast<const uint4 *>(&srow[wave][q + h][0]);
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const uint4 r4 = rl[v];
                    li[h][4 * v] = r4.x;
                    li[h][4 * v + 1] = r4.y;
                    li[h][4 * v + 2] = r4.z;
                    li[h][4 * v + 3] = r4.w;
                }
            }
            double wc[2];
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const uint32_t v = b.ln[q + h];
                if constexpr (WL)
                    wc[h] = weight(v, sw[v < (uint32_t)k ? v : 0u]);
                else
                    wc[h] = b.wg[q + h];
            }
            // the 16 terms of each grouping in order, eight per call
            double s0 = 0.0, s1 = 0.0;
            masked_add8_pair(s0, b.ln[q], li[0], s1, b.ln[q + 1], li[1], d2);
            masked_add8_pair(s0, b.ln[q], li[0] + 8, s1, b.ln[q + 1], li[1] + 8, d2 + 8);
            acc[q] = __builtin_fma(s0, wc[0], acc[q]);
            acc[q + 1] = __builtin_fma(s1, wc[1], acc[q + 1]);
        }
    };
    // the run's tiles in order: along the tile row, then the next row
    int64_t I = 0, J = 0;
    auto advance = [&]() {
        if (++J == nt) {
            ++I;
            J = I;
        }
    };
    Buf A, B;
    if (t0 < t_end) {
        tri_decode(t0, nt, I, J);
        fetch(A, I, J);
    }
    for (int64_t t = t0; t < t_end; t += 2) {
        const bool more = t + 1 < t_end;
        prep(A);
        if (more) {
            advance();
            fetch(B, I, J);
        }
        compute(A);
        if (!more) break;
        prep(B);
        if (t + 2 < t_end) {
            advance();
            fetch(A, I, J);
        }
        compute(B);
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
// One instance of k_sw_few: weights in LDS when the groups fit there.
template <int EQ, typename LT>
void launch_few_eq(int32_t k, dim3 grid, hipStream_t s, const float *mat, int64_t n, int64_t nt,
                   int64_t tiles, int64_t tpc, const LT *g, int64_t gstride, const int32_t *rows,
                   int64_t m, const double *w, double *partial, int64_t m_pad, int packed) {
    if (k <= kFewWLds)
        hipLaunchKernelGGL((k_sw_few<EQ, LT, true>), grid, dim3(256), 0, s, mat, n, nt, tiles, tpc,
                           g, gstride, rows, m, k, w, partial, m_pad, packed);
    else
        hipLaunchKernelGGL((k_sw_few<EQ, LT, false>), grid, dim3(256), 0, s, mat, n, nt, tiles,
                           tpc, g, gstride, rows, m, k, w, partial, m_pad, packed);
}

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
            launch_few_eq<16, LT>(k, dim3((unsigned)used, (unsigned)full), s, mat, n, nt, tiles,
                                  tpc, g, gstride, rows + b, 16 * full, w, partial, m_pad, packed);
        const int32_t *rr = rows + b + 16 * full;
        double *pr = partial + 16 * full;
        const dim3 grid((unsigned)used, 1);
        if (rest == 0) {
        } else if (rest <= 4) {
            launch_few_eq<4, LT>(k, grid, s, mat, n, nt, tiles, tpc, g, gstride, rr, rest, w, pr,
                                 m_pad, packed);
        } else if (rest <= 8) {
            launch_few_eq<8, LT>(k, grid, s, mat, n, nt, tiles, tpc, g, gstride, rr, rest, w, pr,
                                 m_pad, packed);
        } else if (rest <= 12) {
            launch_few_eq<12, LT>(k, grid, s, mat, n, nt, tiles, tpc, g, gstride, rr, rest, w, pr,
                                  m_pad, packed);
        } else {
            launch_few_eq<16, LT>(k, grid, s, mat, n, nt, tiles, tpc, g, gstride, rr, rest, w, pr,
                                  m_pad, packed);
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
