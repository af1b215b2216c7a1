// Staging kernels: label validation and narrowing to u16, the per-group
// weights 1/n_g, and the FP64 total sum of squares s_T.
#include "internal.h"

namespace pstat {

namespace {

__device__ inline int32_t wave_max(int32_t v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    return v;
}

// Checks one label; returns the u16 to store (the pad value for a bad one).
__device__ inline uint16_t check_label(int32_t v, int32_t limit, int64_t p, uint8_t *bad_perm,
                                       int32_t *err_flag) {
    if (v < 0 || v >= limit) {
        bad_perm[p] = 1;
        atomicOr(err_flag, 1);
        return kPadLabel;
    }
    return (uint16_t)v;
}

// 64 x 64 transpose through LDS: block (64, 4), tile rows = permutations,
// tile columns = objects.
__global__ __launch_bounds__(256) void k_stage_labels_om(
    const int32_t *__restrict__ g, const int32_t *__restrict__ rows, int64_t n, int64_t P,
    int64_t n_pad, int64_t P_pad, int32_t limit, uint16_t *__restrict__ out,
    uint8_t *__restrict__ bad_perm, int32_t *__restrict__ err_flag) {
    __shared__ uint16_t tile[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;  // objects
    const int64_t p0 = (int64_t)blockIdx.y * 64;  // permutations
    const int tx = threadIdx.x, ty = threadIdx.y;
    for (int r = ty; r < 64; r += 4) {
        const int64_t p = p0 + r, i = i0 + tx;
        uint16_t v = kPadLabel;
        if (p < P && i < n) {
            const int64_t src = rows ? (int64_t)rows[p] : p;
            v = check_label(g[src * n + i], limit, p, bad_perm, err_flag);
        }
        tile[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t i = i0 + r, p = p0 + tx;
        if (i < n_pad && p < P_pad) out[i * P_pad + p] = tile[tx][r];
    }
}

__global__ __launch_bounds__(256) void k_stage_labels_pm(
    const int32_t *__restrict__ g, int64_t n, int64_t P, int64_t n_pad, int64_t P_pad,
    int32_t limit, uint16_t *__restrict__ out, uint8_t *__restrict__ bad_perm,
    int32_t *__restrict__ err_flag) {
    for (int64_t p = blockIdx.y; p < P_pad; p += gridDim.y) {
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_pad;
             i += (int64_t)gridDim.x * 256) {
            uint16_t v = kPadLabel;
            if (p < P && i < n) v = check_label(g[p * n + i], limit, p, bad_perm, err_flag);
            out[p * n_pad + i] = v;
        }
    }
}

// Same, four labels per thread (16-byte loads, 8-byte stores) when n % 4 == 0
// and g is 16-byte aligned.
__global__ __launch_bounds__(256) void k_stage_labels_pm4(
    const int32_t *__restrict__ g, int64_t n, int64_t P, int64_t n_pad, int64_t P_pad,
    int32_t limit, uint16_t *__restrict__ out, uint8_t *__restrict__ bad_perm,
    int32_t *__restrict__ err_flag) {
    const int64_t q_pad = n_pad / 4;
    for (int64_t p = blockIdx.y; p < P_pad; p += gridDim.y) {
        for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < q_pad;
             q += (int64_t)gridDim.x * 256) {
            const int64_t i = 4 * q;
            uint16_t v[4] = {kPadLabel, kPadLabel, kPadLabel, kPadLabel};
            if (p < P && i < n) {
                const int4 x = *reinterpret_cast<const int4 *>(g + p * n + i);
                v[0] = check_label(x.x, limit, p, bad_perm, err_flag);
                v[1] = check_label(x.y, limit, p, bad_perm, err_flag);
                v[2] = check_label(x.z, limit, p, bad_perm, err_flag);
                v[3] = check_label(x.w, limit, p, bad_perm, err_flag);
            }
            *reinterpret_cast<uint2 *>(out + p * n_pad + i) =
                make_uint2((uint32_t)v[0] | ((uint32_t)v[1] << 16),
                           (uint32_t)v[2] | ((uint32_t)v[3] << 16));
        }
    }
}

// Flat range check and maximum of int32 labels.
__global__ __launch_bounds__(256) void k_scan_labels(const int32_t *__restrict__ g, int64_t count,
                                                     int32_t limit, int32_t *__restrict__ err_flag,
                                                     int32_t *__restrict__ max_label) {
    int32_t local_max = -1;
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * 256) {
        const int32_t v = g[i];
        if (v < 0 || v >= limit) bad = true;
        else local_max = max(local_max, v);
    }
    if (bad) atomicOr(err_flag, 1);
    local_max = wave_max(local_max);
    __shared__ int32_t wmax[4];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = local_max;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int32_t m = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
        if (m >= 0) atomicMax(max_label, m);
    }
}

__global__ void k_fill_u8(uint8_t *p, int64_t count, uint8_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_u32(uint32_t *p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Group sizes: per-block histogram in LDS (k <= kHist), then one global
// atomic per non-empty bin; larger k counts with global atomics directly.
constexpr int kHist = 4096;
__global__ __launch_bounds__(256) void k_count_groups(const int32_t *__restrict__ grouping,
                                                      int64_t n, int32_t k,
                                                      uint32_t *__restrict__ counts) {
    __shared__ uint32_t hist[kHist];
    const bool local = k <= kHist;
    if (local)
        for (int g = threadIdx.x; g < k; g += blockDim.x) hist[g] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = grouping[i];
        if (v >= 0 && v < k) {
            if (local) atomicAdd(&hist[v], 1u);
            else atomicAdd(&counts[v], 1u);
        }
    }
    __syncthreads();
    if (local)
        for (int g = threadIdx.x; g < k; g += blockDim.x)
            if (hist[g]) atomicAdd(&counts[g], hist[g]);
}

__global__ void k_invert_counts(const uint32_t *__restrict__ counts, int32_t k,
                                double *__restrict__ inv) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < k) inv[g] = counts[g] ? 1.0 / (double)counts[g] : 0.0;
}

constexpr int kSTBlocks = 2048;

// Block b sums rows b, b + G, b + 2G, ...; each row's strict-upper part is
// strided over the 256 threads; fixed-shape tree reduction in LDS.
__global__ __launch_bounds__(256) void k_sT_partial(const float *__restrict__ mat, int64_t n,
                                                    double *__restrict__ partials, int packed) {
    double acc = 0.0;
    for (int64_t i = blockIdx.x; i < n - 1; i += gridDim.x) {
        const int64_t rb = d_row_base(i, n, packed);
        for (int64_t j = i + 1 + threadIdx.x; j < n; j += 256) {
            const double d = (double)mat[rb + j];
            acc += d * d;
        }
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// s_T = (sum of the partials) / n: thread t adds partials t, t + 256, ...
// ascending, then a fixed-shape tree over the 256 threads.
__global__ __launch_bounds__(256) void k_sT_final(const double *__restrict__ partials,
                                                  int64_t count, int64_t n,
                                                  double *__restrict__ sT) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < count; b += 256) s += partials[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *sT = red[0] / (double)n;
}

inline unsigned grid_for(int64_t count, int block, int64_t cap = 65535) {
    int64_t g = ceil_div(count, block);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

} // namespace

void launch_stage_labels_om(const int32_t *g, const int32_t *rows, int64_t n, int64_t P,
                            int64_t n_pad, int64_t P_pad, int32_t limit, uint16_t *out,
                            uint8_t *bad_perm, int32_t *err_flag, hipStream_t s) {
    dim3 grid((unsigned)ceil_div(n_pad, 64), (unsigned)ceil_div(P_pad, 64));
    hipLaunchKernelGGL(k_stage_labels_om, grid, dim3(64, 4), 0, s, g, rows, n, P, n_pad, P_pad,
                       limit, out, bad_perm, err_flag);
}

void launch_scan_labels(const int32_t *g, int64_t count, int32_t limit, int32_t *err_flag,
                        int32_t *max_label, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_scan_labels, dim3(grid_for(count, 256, 4096)), dim3(256), 0, s, g, count,
                       limit, err_flag, max_label);
}

void launch_stage_labels_pm(const int32_t *g, int64_t n, int64_t P, int64_t n_pad,
                            int64_t P_pad, int32_t limit, uint16_t *out, uint8_t *bad_perm,
                            int32_t *err_flag, hipStream_t s) {
    if (n % 4 == 0 && n_pad % 4 == 0 && (uintptr_t)g % 16 == 0 && (uintptr_t)out % 8 == 0) {
        dim3 grid(grid_for(n_pad / 4, 256, 64), (unsigned)(P_pad < 65535 ? P_pad : 65535));
        hipLaunchKernelGGL(k_stage_labels_pm4, grid, dim3(256), 0, s, g, n, P, n_pad, P_pad, limit,
                           out, bad_perm, err_flag);
        return;
    }
    dim3 grid(grid_for(n_pad, 256, 64), (unsigned)(P_pad < 65535 ? P_pad : 65535));
    hipLaunchKernelGGL(k_stage_labels_pm, grid, dim3(256), 0, s, g, n, P, n_pad, P_pad, limit,
                       out, bad_perm, err_flag);
}

void launch_fill_u8(uint8_t *p, int64_t count, uint8_t v, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(count, 256, 4096)), dim3(256), 0, s, p, count, v);
}

void launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(count, 256, 4096)), dim3(256), 0, s, p, count, v);
}

void launch_group_weights(const int32_t *grouping, int64_t n, int32_t k, uint32_t *counts,
                          double *inv, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(k, 256, 4096)), dim3(256), 0, s, counts,
                       (int64_t)k);
    hipLaunchKernelGGL(k_count_groups, dim3(grid_for(n, 256, 256)), dim3(256), 0, s, grouping,
                       n, k, counts);
    hipLaunchKernelGGL(k_invert_counts, dim3(grid_for(k, 256)), dim3(256), 0, s, counts, k, inv);
}

int64_t sT_partials_count(int64_t n) { return n - 1 < kSTBlocks ? (n > 1 ? n - 1 : 1) : kSTBlocks; }

void launch_sT(const float *mat, int64_t n, double *partials, double *sT, hipStream_t s,
               int packed) {
    const int64_t blocks = sT_partials_count(n);
    hipLaunchKernelGGL(k_sT_partial, dim3((unsigned)blocks), dim3(256), 0, s, mat, n, partials,
                       packed);
    hipLaunchKernelGGL(k_sT_final, dim3(1), dim3(256), 0, s, partials, blocks, n, sT);
}

void launch_sT_final(const double *partials, int64_t count, int64_t n, double *sT, hipStream_t s) {
    hipLaunchKernelGGL(k_sT_final, dim3(1), dim3(256), 0, s, partials, count, n, sT);
}

} // namespace pstat
