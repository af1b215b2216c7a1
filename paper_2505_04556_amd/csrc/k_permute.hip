// Permutation generator: for permutation p, Durstenfeld's Fisher-Yates shuffle
// of the base labels (i from n-1 down to 1, swap a[i] with a uniform a[j],
// 0 <= j <= i), the random relabeling of the permutation test (section 1).
//
// Random numbers: one SplitMix64 stream per permutation (Steele, Lea & Flood,
// OOPSLA 2014: state += 0x9E3779B97F4A7C15, output = the state through the
// 30/27/31 xor-shift-multiply finaliser), started at mix(seed ^ mix(p + 1)).
// Each bounded draw in [0, s) takes the upper 32 bits x of an output and uses
// Lemire's multiply-shift with rejection (ACM TOMACS 2019): m = x * s,
// accept when the low 32 bits of m are >= (2^32 - s) mod s, return m >> 32.
//
// Each lane shuffles one permutation.  When n labels of the narrowest type
// that holds them fit in LDS, a work-group of one wave keeps up to 64 arrays
// in LDS (random swaps then cost LDS latency, not HBM latency) and writes the
// finished rows out coalesced; otherwise lanes shuffle in place in the output.
#include "internal.h"

namespace pstat {

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Stream {
    uint64_t state;
    __device__ inline uint32_t next_hi() {
        state += kGamma;
        return (uint32_t)(mix64(state) >> 32);
    }
    __device__ inline uint32_t below(uint32_t s) {
        uint64_t m = (uint64_t)next_hi() * (uint64_t)s;
        uint32_t lo = (uint32_t)m;
        if (lo < s) {
            const uint32_t thresh = (uint32_t)(0u - s) % s;
            while (lo < thresh) {
                m = (uint64_t)next_hi() * (uint64_t)s;
                lo = (uint32_t)m;
            }
        }
        return (uint32_t)(m >> 32);
    }
};

__device__ inline uint64_t stream_start(uint64_t seed, uint64_t p) {
    return mix64(seed ^ mix64(p + 1));
}

// The draw for the next step does not depend on the array, so it is taken
// while the current step's two reads are in flight.
template <typename E>
__device__ inline void shuffle(E *a, int64_t n, uint64_t seed, int64_t p) {
    if (n < 2) return;
    Stream st{stream_start(seed, (uint64_t)p)};
    uint32_t j = st.below((uint32_t)n);
    for (int64_t i = n - 1; i >= 1; --i) {
        const E ai = a[i];
        const E aj = a[j];
        const uint32_t jn = i > 1 ? st.below((uint32_t)i) : 0u;
        a[i] = aj;
        a[j] = ai;
        j = jn;
    }
}

template <typename E>
__global__ __launch_bounds__(64) void k_permute_lds(const int32_t *__restrict__ base, int64_t n,
                                                    int64_t P, uint64_t seed, int ppw,
                                                    int vec, int32_t *__restrict__ out) {
    extern __shared__ __align__(16) unsigned char smem[];
    E *arr = reinterpret_cast<E *>(smem);
    const int64_t p0 = (int64_t)blockIdx.x * ppw;
    const int tid = threadIdx.x;
    int live = ppw;
    if (p0 + live > P) live = (int)(P - p0);
    // Copy in: each base label is loaded once (four per lane per load when
    // base and every output row are 16-byte aligned: `vec`) and written into
    // every permutation's slot.
    const int64_t n4 = vec ? n / 4 : 0;
    const int4 *base4 = reinterpret_cast<const int4 *>(base);
    for (int64_t v = tid; v < n4; v += 64) {
        const int4 b = base4[v];
        for (int q = 0; q < live; q++) {
            E *d = arr + (int64_t)q * n + 4 * v;
            d[0] = (E)b.x;
            d[1] = (E)b.y;
            d[2] = (E)b.z;
            d[3] = (E)b.w;
        }
    }
    for (int64_t i = 4 * n4 + tid; i < n; i += 64) {
        const E b = (E)base[i];
        for (int q = 0; q < live; q++) arr[(int64_t)q * n + i] = b;
    }
    __syncthreads();
    if (tid < live) shuffle<E>(arr + (int64_t)tid * n, n, seed, p0 + tid);
    __syncthreads();
    // Copy out, 16-byte stores under the same condition.
    for (int q = 0; q < live; q++) {
        const E *src = arr + (int64_t)q * n;
        int32_t *dst = out + (p0 + q) * n;
        int4 *dst4 = reinterpret_cast<int4 *>(dst);
        for (int64_t v = tid; v < n4; v += 64)
            dst4[v] = make_int4(src[4 * v], src[4 * v + 1], src[4 * v + 2], src[4 * v + 3]);
        for (int64_t i = 4 * n4 + tid; i < n; i += 64) dst[i] = (int32_t)src[i];
    }
}

__global__ __launch_bounds__(64) void k_permute_global(const int32_t *__restrict__ base, int64_t n,
                                                       int64_t P, uint64_t seed,
                                                       int32_t *__restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (p >= P) return;
    int32_t *a = out + p * n;
    for (int64_t i = 0; i < n; i++) a[i] = base[i];
    shuffle<int32_t>(a, n, seed, p);
}

template <typename E>
int launch_lds(const int32_t *base, int64_t n, int64_t P, uint64_t seed, int32_t *out,
               size_t lds_limit, hipStream_t s) {
    const size_t row = (size_t)n * sizeof(E);
    int64_t ppw = (int64_t)(lds_limit / row);
    if (ppw < 1) return 1;  // does not fit
    if (ppw > 64) ppw = 64;
    if (ppw > P) ppw = P;
    const size_t bytes = (size_t)ppw * row;
    (void)hipFuncSetAttribute((const void *)k_permute_lds<E>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    const int64_t blocks = ceil_div(P, ppw);
    const int vec = (n % 4 == 0) && ((uintptr_t)base % 16 == 0) && ((uintptr_t)out % 16 == 0);
    hipLaunchKernelGGL(k_permute_lds<E>, dim3((unsigned)blocks), dim3(64), bytes, s, base, n, P,
                       seed, (int)ppw, vec, out);
    return 0;
}

} // namespace

int launch_permute(const int32_t *base, int64_t n, int64_t P, uint64_t seed, int32_t max_label,
                   int32_t *out, size_t lds_limit, hipStream_t s) {
    if (P <= 0 || n <= 0) return 0;
    if (max_label < 256 && launch_lds<uint8_t>(base, n, P, seed, out, lds_limit, s) == 0) return 0;
    if (max_label < 65536 && launch_lds<uint16_t>(base, n, P, seed, out, lds_limit, s) == 0)
        return 0;
    hipLaunchKernelGGL(k_permute_global, dim3((unsigned)ceil_div(P, 64)), dim3(64), 0, s, base, n,
                       P, seed, out);
    return 0;
}

} // namespace pstat
