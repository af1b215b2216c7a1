// Device-side producers of the synthetic distance matrices (input generation
// only; none of the PERMANOVA statistic is computed here).  They give the same
// values as the numpy generators in synth/__init__.py:
//   uniform: d_ij = (2 * (h >> 41) + 1) * 2^-24 with h = mix64(key ^ mix64(seed)),
//            key = min(i,j) * n + max(i,j); zero diagonal.
//   euclid:  d_ij = RN_fp32(||x_i - x_j|| / dmax) from FP64 points, squared
//            differences summed in dimension order, correctly rounded sqrt and
//            division; dmax = the largest off-diagonal distance.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_uniform(float *__restrict__ out, int64_t n, int64_t row0, int64_t rows,
                          uint64_t seed_mix) {
    const int64_t r = blockIdx.y;
    for (int64_t rr = r; rr < rows; rr += gridDim.y) {
        const int64_t i = row0 + rr;
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
             j += (int64_t)gridDim.x * blockDim.x) {
            float v = 0.0f;
            if (i != j) {
                const uint64_t lo = (uint64_t)(i < j ? i : j), hi = (uint64_t)(i < j ? j : i);
                const uint64_t h = mix64((lo * (uint64_t)n + hi) ^ seed_mix);
                const uint64_t m = ((h >> 41) << 1) | 1ull;
                v = (float)((double)m * 0x1p-24);
            }
            out[(uint64_t)rr * (uint64_t)n + j] = v;
        }
    }
}

// The same values, strict upper triangle only, packed row after row (row i
// holds columns i + 1 .. n - 1 from element i (2n - i - 1) / 2 on).
__global__ void k_uniform_packed(float *__restrict__ out, int64_t n, uint64_t seed_mix) {
    for (int64_t i = blockIdx.y; i < n - 1; i += gridDim.y) {
        const int64_t base = i * (2 * n - i - 1) / 2 - i - 1;
        for (int64_t j = i + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
             j += (int64_t)gridDim.x * blockDim.x) {
            const uint64_t h = mix64(((uint64_t)i * (uint64_t)n + (uint64_t)j) ^ seed_mix);
            const uint64_t m = ((h >> 41) << 1) | 1ull;
            out[base + j] = (float)((double)m * 0x1p-24);
        }
    }
}

__device__ inline double pair_dist(const double *__restrict__ x, int64_t i, int64_t j, int dims) {
    double acc = 0.0;
    for (int d = 0; d < dims; d++) {
        const double t = x[i * dims + d] - x[j * dims + d];
        acc = __dadd_rn(acc, __dmul_rn(t, t));
    }
    return __dsqrt_rn(acc);
}

// Largest off-diagonal distance, as the bits of a non-negative double (order
// of the bits equals order of the values).
__global__ void k_euclid_max(const double *__restrict__ x, int64_t n, int dims,
                             unsigned long long *__restrict__ dmax_bits) {
    double m = 0.0;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y)
        for (int64_t j = i + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
             j += (int64_t)gridDim.x * blockDim.x)
            m = fmax(m, pair_dist(x, i, j, dims));
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(dmax_bits, (unsigned long long)__double_as_longlong(m));
}

__global__ void k_euclid(const double *__restrict__ x, int64_t n, int dims,
                         const unsigned long long *__restrict__ dmax_bits, float *__restrict__ out) {
    const double dmax = __longlong_as_double((long long)*dmax_bits);
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y)
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
             j += (int64_t)gridDim.x * blockDim.x) {
            float v = 0.0f;
            if (i != j) {
                const int64_t a = i < j ? i : j, b = i < j ? j : i;
                v = (float)__ddiv_rn(pair_dist(x, a, b, dims), dmax);
            }
            out[(uint64_t)i * (uint64_t)n + j] = v;
        }
}

}  // namespace

extern "C" {

// rows [row0, row0 + rows) of the uniform matrix into out (rows x n floats).
int synth_uniform(float *out, int64_t n, int64_t row0, int64_t rows, uint64_t seed_mix,
                  void *stream) {
    dim3 grid((unsigned)((n + 255) / 256 < 64 ? (n + 255) / 256 : 64),
              (unsigned)(rows < 4096 ? rows : 4096));
    hipLaunchKernelGGL(k_uniform, grid, dim3(256), 0, (hipStream_t)stream, out, n, row0, rows,
                       seed_mix);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// the uniform matrix's strict upper triangle, packed: n (n - 1) / 2 floats
int synth_uniform_packed(float *out, int64_t n, uint64_t seed_mix, void *stream) {
    dim3 grid((unsigned)((n + 255) / 256 < 64 ? (n + 255) / 256 : 64),
              (unsigned)(n < 8192 ? n : 8192));
    hipLaunchKernelGGL(k_uniform_packed, grid, dim3(256), 0, (hipStream_t)stream, out, n,
                       seed_mix);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// full n x n Euclidean matrix from n x dims FP64 points (device); scratch: 8 bytes.
int synth_euclid(float *out, const double *x, int64_t n, int dims, unsigned long long *scratch,
                 void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (hipMemsetAsync(scratch, 0, 8, s) != hipSuccess) return -1;
    dim3 grid((unsigned)((n + 255) / 256 < 64 ? (n + 255) / 256 : 64),
              (unsigned)(n < 4096 ? n : 4096));
    hipLaunchKernelGGL(k_euclid_max, grid, dim3(256), 0, s, x, n, dims, scratch);
    hipLaunchKernelGGL(k_euclid, grid, dim3(256), 0, s, x, n, dims, scratch, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // extern "C"
