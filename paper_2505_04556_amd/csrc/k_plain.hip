// Plain (VALU) form of s_W: one permutation per lane.
//
// The strict upper triangle of D is cut into T x T tiles (I <= J; the diagonal
// tiles are masked to col > row, which is Algorithm 2's column start of
// section 2).  A work-group owns LANES permutations (one per lane) and a
// contiguous run of tiles.  For each tile it stages d^2 into LDS once; every
// lane then walks the whole tile against its own permutation's labels, which
// sit in registers for the tile's columns.  The LDS reads use one address per
// wave (broadcast), so a staged tile is reused by all LANES permutations and D
// streams from HBM once per LANES permutations instead of once per
// permutation.  Per row segment the matching d^2 are summed in Acc (FP32 or
// FP64; each add runs under a lane mask set by its label compare) and
// then multiplied once by that row's group weight in FP64 --
// Algorithm 2's hoisting of inv_group_sizes -- into a per-lane FP64 total.
// Lanes never share a sum, so no cross-lane reduction is needed; each
// work-group writes one FP64 partial per permutation and a fixed-order FP64
// reduction combines them.
#include "internal.h"
#include "lane_mask.h"

namespace pstat {

namespace {

constexpr int kWeightCache = 1024;  // weights held in LDS (k up to this many)
constexpr int64_t kMaxChunks = 2048;  // partial rows per permutation (bounds the reduction)


template <typename Acc>
struct VecOf;
template <>
struct VecOf<float> { using type = float4; };
template <>
struct VecOf<double> { using type = double2; };

template <typename Acc>
__device__ inline Acc square(float d);
template <>
__device__ inline float square<float>(float d) { return d * d; }
template <>
__device__ inline double square<double>(float d) { return (double)d * (double)d; }

// One work unit: tile chunk `chunk` of the triangle for the LANES permutations
// of group `pg`; writes partial[chunk * P_pad + pg * LANES + lane].  PK: D in
// the packed layout (a separate instantiation, so the square one keeps its
// plain row-major addressing).
template <int T, int LANES, typename Acc, bool PK>
__device__ inline void plain_unit(const float *__restrict__ mat, int64_t n, int64_t nt,
                                  int64_t n_tiles, int64_t tiles_per_chunk,
                                  const uint16_t *__restrict__ lab, int64_t P_pad,
                                  const double *__restrict__ w, int32_t k,
                                  double *__restrict__ partial, int64_t chunk, int64_t pg,
                                  Acc (&sD)[T][T], double (&sWt)[kWeightCache]) {
    const int tid = threadIdx.x;
    const int64_t perm = pg * LANES + tid;
    const int kc = k < kWeightCache ? k : kWeightCache;
    const bool wlds = k <= kWeightCache;   // uniform: every weight in LDS
    for (int g = tid; g < kc; g += LANES) sWt[g] = w[g];

    const int64_t t0 = chunk * tiles_per_chunk;
    int64_t t1 = t0 + tiles_per_chunk;
    if (t1 > n_tiles) t1 = n_tiles;
    double tot = 0.0;
    if (t0 < t1) {
        int64_t I, J;
        tri_decode(t0, nt, I, J);
        constexpr int kPer = T * T / LANES;  // staged elements per thread
        static_assert(kPer >= 1 && (T * T) % LANES == 0, "tile/lane shape");
        float pre[kPer];
        auto fetch = [&](int64_t I_, int64_t J_) {
            const int64_t i0 = I_ * T, j0 = J_ * T;
            // packed: the row base of this thread's first row, then stepped
            // by LANES / T rows (d_row_base(i + 1) = d_row_base(i) + n - i - 2)
            constexpr int S = LANES / T;
            int64_t rb = PK ? d_row_base(i0 + tid / T, n, 1) : 0;
#pragma unroll
            for (int q = 0; q < kPer; q++) {
                const int e = tid + q * LANES;
                const int r = e / T, c = e % T;
                const int64_t i = i0 + r, j = j0 + c;
                float v = 0.0f;
                if (i < n && j < n && (I_ < J_ || c > r))
                    v = PK ? mat[rb + j] : mat[(uint64_t)i * (uint64_t)n + j];
                pre[q] = v;
                if (PK) rb += S * (n - i - 2) - S * (S - 1) / 2;
            }
        };
        fetch(I, J);
        for (int64_t t = t0; t < t1; ++t) {
            const int64_t i0 = I * T, j0 = J * T;
            __syncthreads();  // previous tile fully consumed (and weights written)
#pragma unroll
            for (int q = 0; q < kPer; q++) {
                const int e = tid + q * LANES;
                sD[e / T][e % T] = square<Acc>(pre[q]);
            }
            // this lane's labels of the tile's columns and rows
            uint32_t Lc[T], Li[T];
#pragma unroll
            for (int c = 0; c < T; c++) Lc[c] = lab[(j0 + c) * P_pad + perm];
#pragma unroll
            for (int r = 0; r < T; r++) Li[r] = lab[(i0 + r) * P_pad + perm];
#pragma unroll
            for (int c = 0; c < T; c++) asm volatile("" : "+v"(Lc[c]));
            __syncthreads();
            // Next tile's global loads overlap this tile's arithmetic.
            int64_t In = I, Jn = J + 1;
            if (Jn == nt) { In = I + 1; Jn = In; }
            if (t + 1 < t1) fetch(In, Jn);
#pragma unroll 2
            for (int r = 0; r < T; r++) {
                uint32_t li = Li[r];
                // The row's d^2 come in as 16-byte broadcast reads, all of
                // them, before any select (left alone, the compiler predicates
                // each LDS read on its label test); the empty asm statements
                // pin that, and make the label compares plain 32-bit ones.
                constexpr int V = 16 / sizeof(Acc);
                using Vec = typename VecOf<Acc>::type;
                const Vec *row = reinterpret_cast<const Vec *>(
                    __builtin_assume_aligned(&sD[r][0], 16));
                Acc d[T];
#pragma unroll
                for (int c4 = 0; c4 < T / V; c4++) {
                    const Vec v = row[c4];
                    __builtin_memcpy(&d[c4 * V], &v, sizeof(Vec));
                }
#pragma unroll
                for (int c = 0; c < T; c++) asm volatile("" : "+v"(d[c]));
                asm volatile("" : "+v"(li));
                Acc acc = Acc(0);
                // The matching d^2 are added under an execution mask
                // (compares into lane masks, then per column the mask becomes
                // EXEC and one add runs): two vector operations and one scalar
                // move per pair-permutation instead of compare, select, add.
                static_assert(T % 16 == 0, "masked adds take 16 columns at a time");
#pragma unroll
                for (int c = 0; c < T; c += 16) masked_add16(acc, li, &Lc[c], &d[c]);
                // weights from LDS (k <= kWeightCache), else from global memory;
                // padding rows (label kPadLabel >= k) weigh 0
                double wv = 0.0;
                if (wlds) {
                    // an LDS pointer, so the load stays an LDS read
                    const __attribute__((address_space(3))) double *sw =
                        (const __attribute__((address_space(3))) double *)sWt;
                    if (li < (uint32_t)k) wv = sw[li];
                } else {
                    if (li < (uint32_t)k) wv = w[li];
                }
                tot += (double)acc * wv;
            }
            I = In;
            J = Jn;
        }
    }
    partial[chunk * P_pad + perm] = tot;
}

// Blocks are dealt to the 8 XCDs round-robin; map them so that consecutive
// logical blocks (the permutation groups of one tile chunk) share an XCD and
// therefore its L2.
__device__ inline int64_t xcd_logical(int64_t bid, int64_t gpad) {
    return (bid & 7) * (gpad >> 3) + (bid >> 3);
}

template <int T, int LANES, typename Acc, bool PK>
__global__ __launch_bounds__(LANES) void k_plain(
    const float *__restrict__ mat, int64_t n, int64_t nt, int64_t n_tiles,
    int64_t tiles_per_chunk, int64_t pgroups, int64_t grid_real,
    const uint16_t *__restrict__ lab, int64_t P_pad, const double *__restrict__ w, int32_t k,
    double *__restrict__ partial) {
    const int64_t logical = xcd_logical(blockIdx.x, gridDim.x);
    if (logical >= grid_real) return;
    __shared__ __align__(16) Acc sD[T][T];
    __shared__ double sWt[kWeightCache];
    plain_unit<T, LANES, Acc, PK>(mat, n, nt, n_tiles, tiles_per_chunk, lab, P_pad, w, k, partial,
                              logical / pgroups, logical % pgroups, sD, sWt);
}

// Work-list form: block b runs unit units[b] = (job, chunk, pgroup) of the
// job table, so one launch can mix units of many independent problems.
__global__ __launch_bounds__(kServeLanes) void k_plain_worklist(
    const JobDesc *__restrict__ jobs, const UnitDesc *__restrict__ units,
    const int32_t *__restrict__ count) {
    const int64_t logical = xcd_logical(blockIdx.x, gridDim.x);
    if (logical >= *count) return;
    const UnitDesc u = units[logical];
    const JobDesc j = jobs[u.job];
    __shared__ __align__(16) float sD[kServeTile][kServeTile];
    __shared__ double sWt[kWeightCache];
    if (j.packed)
        plain_unit<kServeTile, kServeLanes, float, true>(j.mat, j.n, j.nt, j.n_tiles,
                                                         j.tiles_per_chunk, j.lab, j.P_pad, j.w,
                                                         j.k, j.partial, u.chunk, u.pgroup, sD,
                                                         sWt);
    else
        plain_unit<kServeTile, kServeLanes, float, false>(j.mat, j.n, j.nt, j.n_tiles,
                                                          j.tiles_per_chunk, j.lab, j.P_pad, j.w,
                                                          j.k, j.partial, u.chunk, u.pgroup, sD,
                                                          sWt);
}

template <int T, int LANES, typename Acc>
void launch_one(const PlainPlan &pl, const float *mat, int packed, int64_t n,
                const uint16_t *lab, const double *w, int32_t k, double *partial, hipStream_t s) {
    const int64_t grid_real = pl.chunks * pl.pgroups;
    const int64_t gpad = round_up(grid_real, 8);  // xcd_logical needs a multiple of 8
    if (packed)
        hipLaunchKernelGGL((k_plain<T, LANES, Acc, true>), dim3((unsigned)gpad), dim3(LANES), 0,
                           s, mat, n, pl.n_t, pl.n_tiles, pl.tiles_per_chunk, pl.pgroups,
                           grid_real, lab, pl.P_pad, w, k, partial);
    else
        hipLaunchKernelGGL((k_plain<T, LANES, Acc, false>), dim3((unsigned)gpad), dim3(LANES), 0,
                           s, mat, n, pl.n_t, pl.n_tiles, pl.tiles_per_chunk, pl.pgroups,
                           grid_real, lab, pl.P_pad, w, k, partial);
}

} // namespace

PlainPlan plain_plan(int64_t n, int64_t P, int tile, int lanes, int n_cu) {
    PlainPlan pl{};
    pl.tile = tile;
    pl.lanes = lanes;
    pl.n_t = ceil_div(n, tile);
    pl.n_pad = pl.n_t * tile;
    pl.n_tiles = tri_count(pl.n_t);
    pl.P_pad = round_up(P > 0 ? P : 1, lanes);
    pl.pgroups = pl.P_pad / lanes;
    // Enough work-groups to fill every CU several times over.
    const int64_t target = (int64_t)(n_cu > 0 ? n_cu : 256) * 32;
    int64_t chunks = ceil_div(target, pl.pgroups);
    if (chunks > kMaxChunks) chunks = kMaxChunks;
    if (chunks > pl.n_tiles) chunks = pl.n_tiles;
    if (chunks < 1) chunks = 1;
    pl.tiles_per_chunk = ceil_div(pl.n_tiles, chunks);
    pl.chunks = ceil_div(pl.n_tiles, pl.tiles_per_chunk);
    return pl;
}

int launch_plain(const PlainPlan &pl, bool f64, const float *mat, int64_t n,
                 const uint16_t *lab_om, const double *w, int32_t k, double *partial,
                 hipStream_t s, int packed) {
#define PSTAT_PLAIN_CASE(T_, L_)                                                                 \
    if (pl.tile == T_ && pl.lanes == L_) {                                                       \
        if (f64) launch_one<T_, L_, double>(pl, mat, packed, n, lab_om, w, k, partial, s);       \
        else launch_one<T_, L_, float>(pl, mat, packed, n, lab_om, w, k, partial, s);            \
        return 0;                                                                                \
    }
    PSTAT_PLAIN_CASE(32, 64)
    PSTAT_PLAIN_CASE(32, 128)
    PSTAT_PLAIN_CASE(32, 256)
    PSTAT_PLAIN_CASE(64, 64)
    PSTAT_PLAIN_CASE(64, 128)
    PSTAT_PLAIN_CASE(64, 256)
#undef PSTAT_PLAIN_CASE
    return -1;
}

void launch_plain_worklist(const JobDesc *jobs, const UnitDesc *units, const int32_t *count,
                           int64_t max_units, hipStream_t s) {
    const int64_t gpad = round_up(max_units > 0 ? max_units : 1, 8);
    hipLaunchKernelGGL(k_plain_worklist, dim3((unsigned)gpad), dim3(kServeLanes), 0, s, jobs, units,
                       count);
}

} // namespace pstat
