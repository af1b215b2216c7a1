// FP64 reductions of per-block partials, and the statistic's last steps:
// F, the permutation p-value and the tie band of the p-value recheck.
#include <math.h>

#include "../../include/pstat.h"
#include "internal.h"

namespace pstat {

namespace {

inline unsigned blocks_for(int64_t count, int block) {
    int64_t g = ceil_div(count, block);
    if (g < 1) g = 1;
    if (g > 65535) g = 65535;
    return (unsigned)g;
}

// out[p] = sum over chunks, ascending, of partial[chunk][p].
__global__ void k_reduce_plain(const double *__restrict__ partial, int64_t chunks, int64_t P_pad,
                               int64_t P, const uint8_t *__restrict__ bad_perm,
                               double *__restrict__ out) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
         p += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
#pragma unroll 8
        for (int64_t c = 0; c < chunks; c++) s += partial[c * P_pad + p];
        out[p] = (bad_perm && bad_perm[p]) ? NAN : s;
    }
}

// tmp[slice][p][g] = sum over the items of slice `blockIdx.y` (items
// slice * per .. (slice + 1) * per - 1) of z[item][p][g] (FP32 -> FP64) in a
// fixed order: thread (e, r) of a 64 x 4 block adds the slice's items r, r + 4,
// ... ascending; the four sums are then added in order.  With one slice this
// is the whole sum; with several (few columns, many items: large n, few
// permutations) the slices are added by k_reduce_slices.
__global__ __launch_bounds__(256) void k_reduce_items(const float *__restrict__ z, int64_t items,
                                                      int64_t per, int64_t P, int32_t k,
                                                      double *__restrict__ tmp) {
    __shared__ double part[4][64];
    const int64_t total = P * k;
    const int el = threadIdx.x % 64, r = threadIdx.x / 64;
    const int64_t e = (int64_t)blockIdx.x * 64 + el;
    const int64_t i0 = (int64_t)blockIdx.y * per;
    const int64_t i1 = i0 + per < items ? i0 + per : items;
    double s = 0.0;
    if (e < total) {
#pragma unroll 4
        for (int64_t it = i0 + r; it < i1; it += 4) s += (double)z[it * total + e];
    }
    part[r][el] = s;
    __syncthreads();
    if (r == 0 && e < total)
        tmp[(int64_t)blockIdx.y * total + e] =
            ((part[0][el] + part[1][el]) + part[2][el]) + part[3][el];
}

// tmp[p][g] = sum over slices ascending of tmp[1 + slice][p][g] (the slices
// sit after the first P * k entries).
__global__ void k_reduce_slices(double *__restrict__ tmp, int64_t total, int64_t slices) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
#pragma unroll 8
        for (int64_t q = 0; q < slices; q++) s += tmp[(1 + q) * total + e];
        tmp[e] = s;
    }
}

// out[p] = sum over g ascending of w[g] * tmp[p][g]; with f16max set, times
// 2^-e, undoing the FP16 form's power-of-two scaling of the squares.
__global__ void k_weight_groups(const double *__restrict__ tmp, int64_t P, int32_t k,
                                const double *__restrict__ w,
                                const uint8_t *__restrict__ bad_perm, double *__restrict__ out,
                                const uint32_t *__restrict__ f16max) {
    const double unscale = f16max ? ldexp(1.0, -f16_scale_exp(*f16max)) : 1.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
         p += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int32_t g = 0; g < k; g++) s += w[g] * tmp[p * k + g];
        out[p] = (bad_perm && bad_perm[p]) ? NAN : s * unscale;
    }
}

// Complement form: column c of grouping p stands for group c (c < L) or
// c + 1; tmp[p][2c] sums the rows of that group, tmp[p][2c + 1] the rows not
// in L.  out[p] = sum_c w[g(c)] tmp[p][2c]
//               + w[L] ((S - vnot[p]) + sum_c tmp[p][2c + 1]),
// c ascending, then times 2^-e for the FP16 form.
__global__ void k_weight_cx(const double *__restrict__ tmp, int64_t P, int32_t k,
                            const double *__restrict__ w, const uint8_t *__restrict__ bad_perm,
                            double *__restrict__ out, const uint32_t *__restrict__ f16max,
                            const int32_t *__restrict__ Lp, const double *__restrict__ S,
                            const double *__restrict__ vnot) {
    const double unscale = f16max ? ldexp(1.0, -f16_scale_exp(*f16max)) : 1.0;
    const int32_t L = *Lp, kc = k - 1;
    const double sum_u = *S;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P;
         p += (int64_t)gridDim.x * blockDim.x) {
        const double *t = tmp + p * 2 * kc;
        double diag = 0.0, rest = 0.0;
        for (int32_t c = 0; c < kc; c++) {
            diag += w[c < L ? c : c + 1] * t[2 * c];
            rest += t[2 * c + 1];
        }
        const double s = diag + w[L] * ((sum_u - vnot[p]) + rest);
        out[p] = (bad_perm && bad_perm[p]) ? NAN : s * unscale;
    }
}

// *L = lowest index of the largest count (one thread).
__global__ void k_largest_group(const uint32_t *__restrict__ counts, int32_t k,
                                int32_t *__restrict__ L) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int32_t b = 0;
    uint32_t m = counts[0];
    for (int32_t g = 1; g < k; g++)
        if (counts[g] > m) {
            m = counts[g];
            b = g;
        }
    *L = b;
}

// Row sums r_i and row + column sums v_i of the stored U from the pre-pass's
// per-unit sums (unit (I, kb) is number I (kb_total - I + 1) + kb - 2I; row
// i lies in panel i / 128, column i in K block i / 64), in a fixed order:
// slice y of kComplementSlices takes every kComplementSlices-th unit of the
// row's panel and of the column's K block into part[y][0][i] and
// part[y][1][i]; the slices are then added in order.
constexpr int kComplementSlices = 8;
__global__ void k_complement_slices(const double *__restrict__ rcs, int64_t n_pad,
                                    int64_t kb_total, double *__restrict__ part) {
    const int64_t y = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t I = i / 128, kj = i / 64;
        double a = 0.0, b = 0.0;
#pragma unroll 8
        for (int64_t kb = 2 * I + y; kb < kb_total; kb += kComplementSlices)
            a += rcs[(I * (kb_total - I + 1) + kb - 2 * I) * 192 + i % 128];
#pragma unroll 8
        for (int64_t J = y; 2 * J <= kj; J += kComplementSlices)
            b += rcs[(J * (kb_total - J + 1) + kj - 2 * J) * 192 + 128 + i % 64];
        part[(y * 2) * n_pad + i] = a;
        part[(y * 2 + 1) * n_pad + i] = b;
    }
}

__global__ void k_complement_sums(const double *__restrict__ part, int64_t n_pad,
                                  double *__restrict__ v, double *__restrict__ r) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad;
         i += (int64_t)gridDim.x * blockDim.x) {
        double a = 0.0, b = 0.0;
        for (int y = 0; y < kComplementSlices; y++) {
            a += part[(y * 2) * n_pad + i];
            b += part[(y * 2 + 1) * n_pad + i];
        }
        r[i] = a;
        v[i] = a + b;
    }
}

// Fixed-order sum of `count` doubles by one work-group: thread t adds
// t, t + 256, ... ascending, then a butterfly per wave and the four waves in
// order.
__device__ inline double block_sum_fixed(double a, double *red4) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
    if (threadIdx.x % 64 == 0) red4[threadIdx.x / 64] = a;
    __syncthreads();
    const double t = ((red4[0] + red4[1]) + red4[2]) + red4[3];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(256) void k_sum_fixed(const double *__restrict__ x, int64_t count,
                                                   double *__restrict__ out) {
    __shared__ double red[4];
    double a = 0.0;
#pragma unroll 8
    for (int64_t i = threadIdx.x; i < count; i += 256) a += x[i];
    const double t = block_sum_fixed(a, red);
    if (threadIdx.x == 0) *out = t;
}

// vnot[p] = sum over i with lab[p][i] != *L of v[i]: ROWS groupings per
// work-group (each v entry is read once for all of them), eight labels (16
// bytes) per thread and step, fixed order.  Rows are read to their padded
// length (a multiple of 128): the pad entries' v is zero.  A grouping's sum
// does not depend on ROWS: the launch takes 2 rows per work-group for a few
// thousand groupings (enough work-groups to fill the device: 0.22 -> 0.07 ms
// for 1,000 groupings at n = 100,000) and 8 above.
template <int ROWS>
__global__ __launch_bounds__(256) void k_vnot(const uint16_t *__restrict__ lab, int64_t stride,
                                              int64_t n_pad, int64_t P,
                                              const int32_t *__restrict__ Lp,
                                              const double *__restrict__ v,
                                              double *__restrict__ vnot) {
    __shared__ double red[4][ROWS];
    const uint32_t L = (uint32_t)*Lp;
    for (int64_t p0 = (int64_t)blockIdx.x * ROWS; p0 < P;
         p0 += (int64_t)gridDim.x * ROWS) {
        double a[ROWS];
#pragma unroll
        for (int q = 0; q < ROWS; q++) a[q] = 0.0;
        for (int64_t c = threadIdx.x; c < n_pad / 8; c += 256) {
            const double2 *vv = reinterpret_cast<const double2 *>(v + c * 8);
            const double2 v0 = vv[0], v1 = vv[1], v2 = vv[2], v3 = vv[3];
            const double x[8] = {v0.x, v0.y, v1.x, v1.y, v2.x, v2.y, v3.x, v3.y};
#pragma unroll
            for (int q = 0; q < ROWS; q++) {
                if (p0 + q >= P) break;
                const uint4 l = reinterpret_cast<const uint4 *>(lab + (p0 + q) * stride)[c];
                const uint32_t lw[4] = {l.x, l.y, l.z, l.w};
#pragma unroll
                for (int e = 0; e < 8; e++)
                    a[q] += (((lw[e / 2] >> (16 * (e % 2))) & 0xFFFFu) != L) ? x[e] : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < ROWS; q++) {
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) a[q] += __shfl_xor(a[q], o);
            if (threadIdx.x % 64 == 0) red[threadIdx.x / 64][q] = a[q];
        }
        __syncthreads();
        if (threadIdx.x < ROWS && p0 + threadIdx.x < P)
            vnot[p0 + threadIdx.x] = ((red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                      red[2][threadIdx.x]) + red[3][threadIdx.x];
        __syncthreads();
    }
}

__device__ inline double pseudo_F(double sW, double sT, int64_t n, int32_t k) {
    if (k < 2 || n <= k) return NAN;
    return ((sT - sW) / (double)(k - 1)) / (sW / (double)(n - k));
}

__global__ void k_F(const double *__restrict__ sW, int64_t count, const double *__restrict__ sT,
                    int64_t n, int32_t k, double *__restrict__ F) {
    const double t = *sT;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        F[i] = pseudo_F(sW[i], t, n, k);
}

// One block: count s_W_perm[q] <= s_W_obs + PSTAT_TIE_RTOL |s_W_obs| (NaN
// compares false).
__global__ __launch_bounds__(1024) void k_pvalue(const double *__restrict__ obs,
                                                 const double *__restrict__ perm, int64_t P,
                                                 double *__restrict__ p) {
    const double edge = *obs + PSTAT_TIE_RTOL * fabs(*obs);
    unsigned long long c = 0;
    for (int64_t q = threadIdx.x; q < P; q += 1024) c += (perm[q] <= edge) ? 1ull : 0ull;
    __shared__ unsigned long long red[1024];
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *p = P > 0 ? (double)(1 + red[0]) / (double)(1 + P) : NAN;
}

// rows q in [q0, R) of sW_all whose value lies within *band (relative to
// |sW_all[0]|) of the p-value's decision interval [.., sW_all[0] (1 + tie
// tolerance)] edges are appended to list: from sW_all[0] (1 - band) to
// sW_all[0] (1 + tie tolerance + band).
__global__ void k_flag_ties(const double *__restrict__ sW_all, int64_t q0, int64_t R,
                            const double *__restrict__ band, int32_t *__restrict__ list,
                            int32_t *__restrict__ count) {
    const double o = sW_all[0];
    const double lo = o - *band * fabs(o);
    const double hi = o + (*band + PSTAT_TIE_RTOL) * fabs(o);
    for (int64_t q = q0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < R;
         q += (int64_t)gridDim.x * blockDim.x) {
        const double v = sW_all[q];
        if (v >= lo && v <= hi) {
            const int32_t at = atomicAdd(count, 1);
            list[at] = (int32_t)q;
        }
    }
}

// *band = margin * max_j |fast[j] - exact[j]| / |exact[0]| over the S samples
// (exact = FP64 recomputation), at least 1e-13.
__global__ void k_tie_band(const double *__restrict__ fast, const double *__restrict__ exact,
                           int64_t S, double margin, double *__restrict__ band) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double e = 0.0;
    for (int64_t j = 0; j < S; j++) {
        const double d = fabs(fast[j] - exact[j]);
        e = (d > e || d != d) ? d : e;  // NaN propagates
    }
    const double b = margin * e / fabs(exact[0]);
    *band = (b > 1e-13 || b != b) ? b : 1e-13;
}

__global__ void k_iota(int32_t *__restrict__ list, int64_t m) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        list[i] = (int32_t)i;
}

__global__ void k_scatter(const double *__restrict__ vals, const int32_t *__restrict__ list,
                          int64_t m, double *__restrict__ sW_all) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        sW_all[list[i]] = vals[i];
}

// result = [F_obs, p, s_W_obs, s_T]; F takes k as the number of non-empty
// groups of counts[0 .. k) when counts is given (one wave counts them).
__global__ void k_pack_result(const double *__restrict__ sW_all, const double *__restrict__ sT,
                              int64_t n, int32_t k, const uint32_t *__restrict__ counts,
                              const double *__restrict__ p, double *__restrict__ result) {
    int32_t kk = k;
    if (counts) {
        int32_t c = 0;
        for (int32_t g = threadIdx.x; g < k; g += 64) c += counts[g] ? 1 : 0;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o);
        kk = c;
    }
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        result[0] = pseudo_F(sW_all[0], *sT, n, kk);
        result[1] = *p;
        result[2] = sW_all[0];
        result[3] = *sT;
    }
}

} // namespace

void launch_reduce_plain(const double *partial, int64_t chunks, int64_t P_pad, int64_t P,
                         const uint8_t *bad_perm, double *out, hipStream_t s) {
    if (P <= 0) return;
    hipLaunchKernelGGL(k_reduce_plain, dim3(blocks_for(P, 256)), dim3(256), 0, s, partial, chunks,
                       P_pad, P, bad_perm, out);
}

// Item slices of the MFMA reduction: enough column blocks x slices to fill
// the chip (about 2,048 work-groups), at least 16 items per slice, at most 64
// slices; a function of the shape only, so every caller sums in the same order.
int64_t reduce_slices(int64_t items, int64_t P, int32_t k) {
    const int64_t cols = ceil_div(P * k, 64);
    int64_t sl = ceil_div(2048, cols > 0 ? cols : 1);
    if (sl > items / 16) sl = items / 16;
    if (sl > 64) sl = 64;
    return sl > 1 ? sl : 1;
}

size_t reduce_tmp_doubles(int64_t items, int64_t P, int32_t k) {
    const int64_t sl = reduce_slices(items, P, k);
    return (size_t)(P > 0 ? P : 1) * k * (sl > 1 ? 1 + sl : 1);
}

void launch_reduce_mfma(const float *z, int64_t items, int64_t P, int32_t k, const double *w,
                        const uint8_t *bad_perm, double *tmp, double *out, hipStream_t s,
                        const uint32_t *f16max, const Complement *cx) {
    if (P <= 0) return;
    const int32_t cols = cx ? 2 * (k - 1) : k;   // z entries per grouping
    const int64_t total = P * cols;
    const int64_t sl = reduce_slices(items, P, cols);
    if (sl == 1) {
        hipLaunchKernelGGL(k_reduce_items, dim3((unsigned)ceil_div(total, 64), 1), dim3(256), 0, s,
                           z, items, items, P, cols, tmp);
    } else {
        hipLaunchKernelGGL(k_reduce_items, dim3((unsigned)ceil_div(total, 64), (unsigned)sl),
                           dim3(256), 0, s, z, items, ceil_div(items, sl), P, cols, tmp + total);
        hipLaunchKernelGGL(k_reduce_slices, dim3(blocks_for(total, 256)), dim3(256), 0, s, tmp,
                           total, sl);
    }
    if (cx)
        hipLaunchKernelGGL(k_weight_cx, dim3(blocks_for(P, 256)), dim3(256), 0, s, tmp, P, k, w,
                           bad_perm, out, f16max, (const int32_t *)cx->L, (const double *)cx->S,
                           (const double *)cx->vnot);
    else
        hipLaunchKernelGGL(k_weight_groups, dim3(blocks_for(P, 256)), dim3(256), 0, s, tmp, P, k,
                           w, bad_perm, out, f16max);
}

int64_t complement_part_doubles(int64_t n) {
    const int64_t panels = ceil_div(n, 128);
    return panels * (panels + 1) * 192;
}

int64_t complement_slice_doubles(int64_t n) {
    return 2 * kComplementSlices * ceil_div(n, 128) * 128;
}

void launch_largest_group(const uint32_t *counts, int32_t k, int32_t *L, hipStream_t s) {
    hipLaunchKernelGGL(k_largest_group, dim3(1), dim3(64), 0, s, counts, k, L);
}

void launch_complement_sums(const Complement &cx, int64_t n, hipStream_t s) {
    const int64_t panels = ceil_div(n, 128);
    const int64_t n_pad = panels * 128;
    hipLaunchKernelGGL(k_complement_slices, dim3(blocks_for(n_pad, 64), kComplementSlices),
                       dim3(64), 0, s, (const double *)cx.rcs, n_pad, 2 * panels, cx.slices);
    hipLaunchKernelGGL(k_complement_sums, dim3(blocks_for(n_pad, 256)), dim3(256), 0, s,
                       (const double *)cx.slices, n_pad, cx.v, cx.r);
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, s, (const double *)cx.r, n_pad, cx.S);
}

void launch_vnot(const Complement &cx, const uint16_t *lab, int64_t stride, int64_t n, int64_t P,
                 hipStream_t s) {
    if (P <= 0) return;
    const int rows = P <= 4096 ? 2 : 8;
    const int64_t groups = ceil_div(P, rows);
    const unsigned g = (unsigned)(groups < 65535 ? groups : 65535);
    if (rows == 2)
        hipLaunchKernelGGL(k_vnot<2>, dim3(g), dim3(256), 0, s, lab, stride, round_up(n, 128), P,
                           (const int32_t *)cx.L, (const double *)cx.v, cx.vnot);
    else
        hipLaunchKernelGGL(k_vnot<8>, dim3(g), dim3(256), 0, s, lab, stride, round_up(n, 128), P,
                           (const int32_t *)cx.L, (const double *)cx.v, cx.vnot);
}

void launch_F(const double *sW, int64_t count, const double *sT, int64_t n, int32_t k,
              double *F, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_F, dim3(blocks_for(count, 256)), dim3(256), 0, s, sW, count, sT, n, k, F);
}

void launch_pvalue(const double *sW_obs, const double *sW_perm, int64_t P, double *p,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_pvalue, dim3(1), dim3(1024), 0, s, sW_obs, sW_perm, P, p);
}

void launch_flag_ties(const double *sW_all, int64_t q0, int64_t R, const double *band,
                      int32_t *list, int32_t *count, hipStream_t s) {
    if (R <= q0) return;
    hipLaunchKernelGGL(k_flag_ties, dim3(blocks_for(R - q0, 256)), dim3(256), 0, s, sW_all, q0, R,
                       band, list, count);
}

void launch_tie_band(const double *fast, const double *exact, int64_t S, double margin,
                     double *band, hipStream_t s) {
    hipLaunchKernelGGL(k_tie_band, dim3(1), dim3(64), 0, s, fast, exact, S, margin, band);
}

void launch_iota(int32_t *list, int64_t m, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_iota, dim3(blocks_for(m, 256)), dim3(256), 0, s, list, m);
}

void launch_scatter(const double *vals, const int32_t *list, int64_t m, double *sW_all,
                    hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(m, 256)), dim3(256), 0, s, vals, list, m, sW_all);
}

void launch_pack_result(const double *sW_all, const double *sT, int64_t n, int32_t k,
                        const uint32_t *counts, const double *p, double *result, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_result, dim3(1), dim3(64), 0, s, sW_all, sT, n, k, counts, p,
                       result);
}

} // namespace pstat
