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
// Batched form (used whenever a few arrays fit in LDS).  Draw d of a stream is
// hi32(mix(start + (d + 1) * gamma)), so any draw can be computed on its own.
// A wave holds 64 / B arrays in LDS and advances each by B steps per batch:
// lane t of a permutation's group computes draw d + t, the step it would
// serve if no draw of the batch is rejected (top index i - t, bound i - t + 1)
// and its swap partner j_t.  A swap whose two positions no other swap of the
// batch touches commutes with all of them, so those swaps run at once (one
// LDS round trip); the others then run one at a time in step order, which
// leaves the array exactly as the sequential order does.  A rejected draw
// shifts every later step of its batch onto another draw, so such a batch is
// replayed by the group's first lane in order, rejections included.  Each
// batch consumes B draws per permutation either way, so the result is
// bit-identical to the one-lane-per-permutation form.  Labels below 4 are
// stored two bits to an entry (sixteen per LDS word) and labels below 16 four
// bits (eight per word), both swapped with atomic xor, else one byte or one
// u16; the output is int32 rows, or u16 rows padded to a stride (the MFMA
// forms' staged layout).
//
// Fallbacks: one lane per permutation with the arrays in LDS, or in place in
// the output when not even one array fits.
#include <atomic>

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

// Value of lane (t + r) mod 16 of this lane's 16-lane row (DPP row rotation,
// no LDS round trip).
__device__ inline uint32_t rotate_row(uint32_t v, int r) {
    // row_ror:R moves lane l's value to lane l + R (mod 16): read the other
    // direction, 16 - r
    switch (r) {
#define PSTAT_ROR(R_) case R_: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x120 + (16 - R_) % 16, 0xF, 0xF, true);
    PSTAT_ROR(1) PSTAT_ROR(2) PSTAT_ROR(3) PSTAT_ROR(4) PSTAT_ROR(5) PSTAT_ROR(6) PSTAT_ROR(7)
    PSTAT_ROR(8) PSTAT_ROR(9) PSTAT_ROR(10) PSTAT_ROR(11) PSTAT_ROR(12) PSTAT_ROR(13) PSTAT_ROR(14)
    PSTAT_ROR(15)
#undef PSTAT_ROR
    }
    return v;
}

// OR over the 64 lanes of the wave, the same value in every lane: prefix ORs
// within each row of 16 lanes (shifts by 1, 2, 4, 8), row 0's and row 2's
// totals carried into the next row, lane 31's into rows 2 and 3, and lane
// 63's result read out.
__device__ inline uint32_t or_wave(uint32_t v) {
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);
    v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// The ballot bits of this lane's group of B lanes.
template <int B>
__device__ inline uint64_t group_mask(int gbase) {
    if constexpr (B == 64) return ~0ull;
    else return ((1ull << B) - 1) << gbase;
}

// Label storage of the batched shuffle.  WideStore keeps one label per
// 8- or 16-bit entry; each lane with nothing to swap swaps a private dummy
// slot, so a batch's writes never race.  PackedStore packs labels below 16
// eight to a 32-bit word (n = 10,000 takes 5,000 bytes, so twice as many
// arrays share a CU's LDS), or labels below 4 sixteen to a word, and writes
// by xor: a swap of values u and v adds
// u ^ v into both positions with an LDS atomic xor, so swaps of different
// positions in one word commute, and a lane with nothing to swap adds zero.
template <typename E>
struct WideStore {
    static constexpr size_t row_bytes(int64_t n) { return (size_t)n * sizeof(E); }
    static constexpr size_t spare_bytes() { return 256 * sizeof(E); }
    E *a;        // this lane's array
    E *dummy;    // this thread's private slot
    __device__ WideStore(unsigned char *smem, int64_t n, int slot, int ppg, int tid)
        : a(reinterpret_cast<E *>(smem) + (int64_t)slot * n),
          dummy(reinterpret_cast<E *>(smem) + (int64_t)ppg * n + tid) {}
    __device__ void swap(int32_t i, int32_t j) const {
        const E ai = a[i], aj = a[j];
        a[i] = aj;
        a[j] = ai;
    }
    // the batch's parallel swap; `between` runs after the reads are issued
    template <typename F>
    __device__ void swap_all(bool now, int32_t i, int32_t j, F &&between) const {
        E *pa = now ? a + i : dummy;
        E *pb = now ? a + j : dummy;
        const E va = *pa, vb = *pb;
        between();
        *pa = vb;
        *pb = va;
    }
    // Copy in: each base label is loaded once (four per load when `vec`) and
    // written into every live array.
    __device__ static void fill(unsigned char *smem, const int32_t *base, int64_t n, int live,
                                int vec, int tid, int nthr) {
        E *arr = reinterpret_cast<E *>(smem);
        const int64_t n4 = vec ? n / 4 : 0;
        const int4 *base4 = reinterpret_cast<const int4 *>(base);
        for (int64_t v = tid; v < n4; v += nthr) {
            const int4 b = base4[v];
            for (int q = 0; q < live; q++) {
                E *d = arr + (int64_t)q * n + 4 * v;
                d[0] = (E)b.x;
                d[1] = (E)b.y;
                d[2] = (E)b.z;
                d[3] = (E)b.w;
            }
        }
        for (int64_t i = 4 * n4 + tid; i < n; i += nthr) {
            const E b = (E)base[i];
            for (int q = 0; q < live; q++) arr[(int64_t)q * n + i] = b;
        }
    }
    // Copy out into rows of `stride` entries: int32 rows (16-byte stores when
    // `vec`), or u16 rows padded with kPadLabel up to the stride.
    template <typename O>
    __device__ static void drain(const unsigned char *smem, O *out, int64_t stride, int64_t p0,
                                 int64_t n, int live, int vec, int tid, int nthr) {
        const E *arr = reinterpret_cast<const E *>(smem);
        const int64_t n4 = (vec && sizeof(O) == 4) ? n / 4 : 0;
        for (int q = 0; q < live; q++) {
            const E *src = arr + (int64_t)q * n;
            O *dst = out + (p0 + q) * stride;
            int4 *dst4 = reinterpret_cast<int4 *>(dst);
            for (int64_t v = tid; v < n4; v += nthr)
                dst4[v] = make_int4(src[4 * v], src[4 * v + 1], src[4 * v + 2], src[4 * v + 3]);
            for (int64_t i = 4 * n4 + tid; i < n; i += nthr) dst[i] = (O)src[i];
            for (int64_t i = n + tid; i < stride; i += nthr) dst[i] = (O)kPadLabel;
        }
    }
};

template <int BITS>
struct PackedStore {
    static constexpr int PER = 32 / BITS;               // labels per word
    static constexpr uint32_t MASK = (1u << BITS) - 1;
    static constexpr size_t row_bytes(int64_t n) { return (size_t)((n + PER - 1) / PER) * 4; }
    static constexpr size_t spare_bytes() { return 0; }
    uint32_t *w;   // this lane's array, PER labels per word
    __device__ PackedStore(unsigned char *smem, int64_t n, int slot, int, int)
        : w(reinterpret_cast<uint32_t *>(smem) + (int64_t)slot * ((n + PER - 1) / PER)) {}
    __device__ uint32_t get(uint32_t i) const {
        return (w[i / PER] >> (BITS * (i % PER))) & MASK;
    }
    __device__ void flip(uint32_t i, uint32_t d) const {
        atomicXor(&w[i / PER], d << (BITS * (i % PER)));
    }
    __device__ void swap(int32_t i, int32_t j) const {
        const uint32_t d = get((uint32_t)i) ^ get((uint32_t)j);
        flip((uint32_t)i, d);
        flip((uint32_t)j, d);
    }
    template <typename F>
    __device__ void swap_all(bool now, int32_t i, int32_t j, F &&between) const {
        const uint32_t ia = now ? (uint32_t)i : 0u, ib = now ? (uint32_t)j : 0u;
        const uint32_t wa = w[ia / PER], wb = w[ib / PER];
        between();
        const uint32_t sa = BITS * (ia % PER), sb = BITS * (ib % PER);
        const uint32_t d = ((wa >> sa) ^ (wb >> sb)) & MASK;   // 0 for a lane with nothing to swap
        atomicXor(&w[ia / PER], d << sa);
        atomicXor(&w[ib / PER], d << sb);
    }
    __device__ static void fill(unsigned char *smem, const int32_t *base, int64_t n, int live,
                                int vec, int tid, int nthr) {
        uint32_t *arr = reinterpret_cast<uint32_t *>(smem);
        const int64_t nw = (n + PER - 1) / PER;
        for (int64_t v = tid; v < nw; v += nthr) {
            uint32_t word = 0;
            if (vec && PER * v + PER <= n) {
#pragma unroll
                for (int r = 0; r < PER / 4; r++) {
                    const int4 b = reinterpret_cast<const int4 *>(base)[(PER / 4) * v + r];
                    word |= ((uint32_t)b.x << (BITS * (4 * r))) |
                            ((uint32_t)b.y << (BITS * (4 * r + 1))) |
                            ((uint32_t)b.z << (BITS * (4 * r + 2))) |
                            ((uint32_t)b.w << (BITS * (4 * r + 3)));
                }
            } else {
                for (int e = 0; e < PER; e++)
                    if (PER * v + e < n) word |= (uint32_t)base[PER * v + e] << (BITS * e);
            }
            for (int q = 0; q < live; q++) arr[(int64_t)q * nw + v] = word;
        }
    }
    // Copy out into rows of `stride` entries: int32 rows (PER / 4 16-byte
    // stores per word when `vec`), or u16 rows (PER / 8 16-byte stores per
    // word when `vec`) padded with kPadLabel up to the stride.
    template <typename O>
    __device__ static void drain(const unsigned char *smem, O *out, int64_t stride, int64_t p0,
                                 int64_t n, int live, int vec, int tid, int nthr) {
        const uint32_t *arr = reinterpret_cast<const uint32_t *>(smem);
        const int64_t nw = (n + PER - 1) / PER;
        for (int q = 0; q < live; q++) {
            const uint32_t *src = arr + (int64_t)q * nw;
            O *dst = out + (p0 + q) * stride;
            for (int64_t v = tid; v < nw; v += nthr) {
                const uint32_t word = src[v];
                const int64_t i0 = PER * v;
                auto lab = [&](int e) { return (word >> (BITS * e)) & MASK; };
                if (vec && i0 + PER <= n) {
                    if constexpr (sizeof(O) == 4) {
#pragma unroll
                        for (int r = 0; r < PER / 4; r++)
                            *reinterpret_cast<int4 *>(dst + i0 + 4 * r) =
                                make_int4(lab(4 * r), lab(4 * r + 1), lab(4 * r + 2),
                                          lab(4 * r + 3));
                    } else {
#pragma unroll
                        for (int r = 0; r < PER / 8; r++)
                            *reinterpret_cast<uint4 *>(dst + i0 + 8 * r) =
                                make_uint4(lab(8 * r) | lab(8 * r + 1) << 16,
                                           lab(8 * r + 2) | lab(8 * r + 3) << 16,
                                           lab(8 * r + 4) | lab(8 * r + 5) << 16,
                                           lab(8 * r + 6) | lab(8 * r + 7) << 16);
                    }
                } else {
                    for (int e = 0; e < PER; e++)
                        if (i0 + e < n) dst[i0 + e] = (O)lab(e);
                }
            }
            for (int64_t i = n + tid; i < stride; i += nthr) dst[i] = (O)kPadLabel;
        }
    }
};
// labels below 16, eight to a word; labels below 4, sixteen to a word (n =
// 100,000 takes 25,000 bytes: six arrays share a CU's LDS instead of three)
using NibbleStore = PackedStore<4>;
using CrumbStore = PackedStore<2>;

// Batched shuffle: B lanes per permutation, 64 / B permutations per wave,
// blockDim.x / 64 waves per work-group, arrays in dynamic LDS as S stores them;
// permutation p goes to row p of `out` (O = int32 rows of n labels, or u16
// rows of `ostride` entries padded with kPadLabel).
// This launch covers permutations pfirst .. P - 1.
template <typename S, int B, typename O>
__global__ __launch_bounds__(256) void k_permute_batch(const int32_t *__restrict__ base, int64_t n,
                                                       int64_t pfirst, int64_t P, uint64_t seed,
                                                       int apw, int vec, O *__restrict__ out,
                                                       int64_t ostride, int ovec) {
    static_assert(B == 16 || B == 64, "lanes per permutation");
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int ppg = (nthr / 64) * apw;                // permutations per work-group (apw per wave)
    const int64_t p0 = pfirst + (int64_t)blockIdx.x * ppg;
    int live = ppg;
    if (p0 + live > P) live = (int)(P - p0);
    S::fill(smem, base, n, live, vec, tid, nthr);
    __syncthreads();

    const int wave = tid / 64, lane = tid % 64;
    const int ps = lane / B, t = lane % B;          // permutation slot in the wave, lane in group
    const int slot = wave * apw + ps;
    const bool mine = ps < apw && slot < live;
    const int gbase = (lane / B) * B;               // first lane of the group
    const S a(smem, n, mine ? slot : 0, ppg, tid);
    const uint64_t start = stream_start(seed, (uint64_t)(p0 + slot));
    // current i of the permutation; 32-bit index arithmetic (an array that
    // fits in LDS has far fewer than 2^31 entries)
    int32_t top = mine ? (int32_t)(n - 1) : 0;
    // this lane's counter, start + (d + t + 1) * gamma, advanced by B draws per batch
    uint64_t ctr = start + ((uint64_t)t + 1) * kGamma;
    uint32_t x = (uint32_t)(mix64(ctr) >> 32);
    for (;;) {
        // the wave runs until all of its permutations are done
        if (__ballot(top >= 1) == 0) break;
        const int32_t it = top - t;                  // this lane's step if nothing is rejected
        const bool valid = it >= 1;
        const uint32_t sb = (uint32_t)(it + 1);
        const uint64_t m = (uint64_t)x * (uint64_t)sb;
        const uint32_t lo = (uint32_t)m;
        const int32_t j = (int32_t)(m >> 32);
        bool ok = true;
        if (valid && lo < sb) ok = lo >= (uint32_t)(0u - sb) % sb;
        const uint64_t gmask = group_mask<B>(gbase);
        // A rejected draw shifts every later step of the batch onto another
        // draw: such a group replays the batch in order (rare).
        const bool grej = (__ballot(valid && !ok) & gmask) != 0;
        // Conflicts: a swap whose partner is another step's top index, two
        // swaps with the same partner, or a step whose top is some other
        // step's partner.  Swaps without conflict commute with every other
        // swap of the batch; the conflicting ones keep their order.
        const bool real = valid && j != it;
        int32_t lowtop = top - B + 1;
        if (lowtop < 1) lowtop = 1;
        // a partner on a later step's top index (top - s for some s > t)
        bool conflict = real && j >= lowtop && j < it;
        // Two equal partners (`shared`).
        bool shared;
        if constexpr (B == 16) {
            // every other lane's partner key (idle lanes and self-swaps carry
            // ~t, which no partner or other key equals) is compared with this
            // lane's; a zero of key ^ other marks it, and the minimum over
            // the group is kept with one three-operand min per two lanes
            // rotated in
            const uint32_t key = real ? (uint32_t)j : ~(uint32_t)t;
            uint32_t mn = 0xFFFFFFFFu;
            uint32_t prev = 0xFFFFFFFFu;
#pragma unroll
            for (int r = 1; r < B; r++) {
                const uint32_t ko = rotate_row(key, r);
                if (r % 2 == 1) {
                    prev = ko ^ key;
                } else {
                    mn = min(min(mn, prev), ko ^ key);
                    prev = 0xFFFFFFFFu;
                }
            }
            shared = min(mn, prev) == 0;
        } else {
            // B == 64: the lanes with real swaps whose partners agree with
            // this lane's in the low kMatchBits bits, as the AND over those
            // bits of the ballot of lanes with the bit set (or its
            // complement); a lane is marked when any lane but itself is
            // left.  Partners that differ only above those bits are marked
            // too: their swaps just keep step order with the other marked
            // ones, which gives the same result.
            constexpr int kMatchBits = 16;
            const uint64_t any = __ballot(real);
            uint32_t m_lo = (uint32_t)any, m_hi = (uint32_t)(any >> 32);
            uint64_t on[kMatchBits];
#pragma unroll
            for (int b = 0; b < kMatchBits; b++) on[b] = __ballot((((uint32_t)j >> b) & 1u) != 0);
#pragma unroll
            for (int b = 0; b < kMatchBits; b++) {
                // all ones where bit b of j is set
                const uint32_t e = (uint32_t)(((int32_t)((uint32_t)j << (31 - b))) >> 31);
                m_lo &= (uint32_t)on[b] ^ ~e;
                m_hi &= (uint32_t)(on[b] >> 32) ^ ~e;
            }
            if (lane < 32) m_lo &= ~(1u << lane);
            else m_hi &= ~(1u << (lane - 32));
            shared = real && (m_lo | m_hi) != 0;
        }
        // A step whose top index is another step's partner: the partners on
        // top indices set bit s (top - j) of a group-wide mask.
        uint32_t hit;
        if constexpr (B == 16) {
            // OR over the 16 lanes of the row: rotations by 8, 4, 2, 1
            uint32_t hm = conflict ? 1u << (uint32_t)(top - j) : 0u;
            hm |= rotate_row(hm, 8);
            hm |= rotate_row(hm, 4);
            hm |= rotate_row(hm, 2);
            hm |= rotate_row(hm, 1);
            hit = (hm >> t) & 1u;
        } else {
            // B == 64: a 64-bit mask, OR-reduced over the wave
            uint32_t lo = 0, hi = 0;
            if (conflict) {
                const uint32_t s = (uint32_t)(top - j);
                lo = s < 32 ? 1u << s : 0u;
                hi = s < 32 ? 0u : 1u << (s - 32);
            }
            lo = or_wave(lo);
            hi = or_wave(hi);
            hit = ((t < 32 ? lo >> t : hi >> (t - 32))) & 1u;
        }
        conflict = (conflict || shared || hit != 0) && valid;

        // swaps without conflict, all at once; the next batch's draw is
        // computed while their reads are in flight (a scheduling barrier
        // keeps it after the reads, the empty asm before the writes)
        uint32_t xn;
        a.swap_all(valid && !conflict && mine && !grej, it, j, [&]() {
            __builtin_amdgcn_sched_barrier(0);
            ctr += (uint64_t)B * kGamma;
            xn = (uint32_t)(mix64(ctr) >> 32);
            asm volatile("" : "+v"(xn));
        });

        if (__ballot(grej) != 0) {
            // gather the group's draws into its first lane, all lanes active
            uint32_t xs[B];
#pragma unroll
            for (int r = 0; r < B; r++) xs[r] = __shfl(x, gbase + r);
            if (grej && t == 0 && mine) {
                int32_t i = top;
#pragma unroll
                for (int r = 0; r < B; r++) {
                    if (i >= 1) {
                        const uint32_t sr = (uint32_t)(i + 1);
                        const uint64_t mr = (uint64_t)xs[r] * (uint64_t)sr;
                        const uint32_t lr = (uint32_t)mr;
                        // a rejected draw is consumed and the step keeps its bound
                        if (!(lr < sr && lr < (uint32_t)(0u - sr) % sr)) {
                            a.swap(i, (int32_t)(mr >> 32));
                            --i;
                        }
                    }
                }
                top = i;
            }
            top = __shfl(top, gbase);
        }
        // then the conflicting swaps of each group, lowest step first
        uint64_t cm = __ballot(conflict && mine && !grej);
        while (cm != 0) {
            const uint64_t g = cm & gmask;
            const bool turn = g != 0 && lane == __builtin_ctzll(g);
            if (turn) a.swap(it, j);
            cm &= ~__ballot(turn);
        }
        if (!grej) top = top - B < 0 ? 0 : top - B;
        x = xn;
    }
    __syncthreads();
    S::drain(smem, out, ostride, p0, n, live, ovec, tid, nthr);
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

// Raises a kernel's dynamic-LDS limit to `limit` (the device's maximum) the
// first time it is launched on a device, instead of before every launch.
template <typename K>
void allow_lds(K *kernel, size_t limit) {
    constexpr int kDevices = 64;
    static std::atomic<size_t> set[kDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevices) {
        (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)limit);
        return;
    }
    if (set[dev].load(std::memory_order_relaxed) == limit) return;
    (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)limit);
    set[dev].store(limit, std::memory_order_relaxed);
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
    allow_lds(k_permute_lds<E>, lds_limit);
    const int64_t blocks = ceil_div(P, ppw);
    const int vec = (n % 4 == 0) && ((uintptr_t)base % 16 == 0) && ((uintptr_t)out % 16 == 0);
    hipLaunchKernelGGL(k_permute_lds<E>, dim3((unsigned)blocks), dim3(64), bytes, s, base, n, P,
                       seed, (int)ppw, vec, out);
    return 0;
}

// One launch of the batched form over permutations pfirst .. plast - 1.
template <typename S, int B, typename O>
void launch_part(const int32_t *base, int64_t n, int64_t pfirst, int64_t plast, uint64_t seed,
                 O *out, int64_t ostride, int pw, int64_t waves, size_t lds_limit, hipStream_t s) {
    const int64_t ppg = waves * pw;
    const size_t bytes = (size_t)ppg * S::row_bytes(n) + S::spare_bytes();
    const int64_t blocks = ceil_div(plast - pfirst, ppg);
    // 16-byte loads of the base labels; 16-byte stores of whole rows' words
    const int vec = (n % 4 == 0) && ((uintptr_t)base % 16 == 0);
    const int ovec = (uintptr_t)out % 16 == 0 &&
                     (sizeof(O) == 4 ? n % 4 == 0 : ostride % 8 == 0);
    allow_lds(k_permute_batch<S, B, O>, lds_limit);
    hipLaunchKernelGGL((k_permute_batch<S, B, O>), dim3((unsigned)blocks),
                       dim3((unsigned)(64 * waves)), bytes, s, base, n, pfirst, plast, seed, pw,
                       vec, out, ostride, ovec);
}

// Batched form: up to four waves per work-group (one per SIMD), up to 16
// arrays; B = 16 lanes per permutation and 1, 2 or 4 arrays per wave when at
// least four arrays fit, else B = 64 and one array per wave.  Work-groups
// small enough share a CU.
template <typename S, typename O>
int launch_batch(const int32_t *base, int64_t n, int64_t P, uint64_t seed, O *out,
                 int64_t ostride, size_t lds_limit, int n_cu, hipStream_t s) {
    const size_t row = S::row_bytes(n);
    const size_t spare = S::spare_bytes();       // the per-thread dummy slots
    if (lds_limit <= spare) return 1;
    int64_t fit = (int64_t)((lds_limit - spare) / row);
    if (fit < 1) return 1;
    if (fit > 16) fit = 16;
    if (fit > P) fit = P;
    const int64_t cus = n_cu > 0 ? n_cu : 256;
    // Arrays a CU holds with one per wave (64 lanes each): work-groups of w
    // waves, as many as its LDS takes.  When that runs every permutation at
    // once, each gets a whole wave (the shortest chain of batches); with
    // more permutations than that, 16 lanes each and several per wave.
    const int64_t per_cu = fit;
    int64_t w64 = per_cu < 4 ? per_cu : 4;
    for (int64_t w = w64; w >= 1; --w)
        if ((per_cu / w) * w > (per_cu / w64) * w64) w64 = w;
    if (!(fit >= 4 && P > cus * per_cu)) {
        launch_part<S, 64, O>(base, n, 0, P, seed, out, ostride, 1, w64, lds_limit, s);
        return 0;
    }
    int pw = (int)ceil_div(fit, 4);
    if (pw == 3) pw = 2;                         // 1, 2 or 4 arrays per wave
    int64_t waves = fit / pw;
    if (waves > 4) waves = 4;
    // The permutations the device runs at once with 16 lanes each; a last
    // partial round small enough to run with a whole wave per permutation
    // does so in a launch of its own, a quarter of the batches long.
    const int64_t ppg = waves * pw;
    int64_t groups = (int64_t)(lds_limit / ((size_t)ppg * row + spare));
    if (groups < 1) groups = 1;
    const int64_t round = cus * groups * ppg;
    const int64_t rest = P % round;
    const int64_t split = P > round && rest > 0 && rest <= cus * per_cu ? P - rest : P;
    launch_part<S, 16, O>(base, n, 0, split, seed, out, ostride, pw, waves, lds_limit, s);
    if (split < P)
        launch_part<S, 64, O>(base, n, split, P, seed, out, ostride, 1, w64, lds_limit, s);
    return 0;
}

} // namespace

int launch_permute(const int32_t *base, int64_t n, int64_t P, uint64_t seed, int32_t max_label,
                   int32_t *out, size_t lds_limit, int n_cu, hipStream_t s) {
    if (P <= 0 || n <= 0) return 0;
    if (max_label < 4 && launch_batch<CrumbStore>(base, n, P, seed, out, n, lds_limit, n_cu, s) == 0)
        return 0;
    if (max_label < 16 && launch_batch<NibbleStore>(base, n, P, seed, out, n, lds_limit, n_cu, s) == 0)
        return 0;
    if (max_label < 256 &&
        launch_batch<WideStore<uint8_t>>(base, n, P, seed, out, n, lds_limit, n_cu, s) == 0)
        return 0;
    if (max_label < 65536 &&
        launch_batch<WideStore<uint16_t>>(base, n, P, seed, out, n, lds_limit, n_cu, s) == 0)
        return 0;
    if (max_label < 256 && launch_lds<uint8_t>(base, n, P, seed, out, lds_limit, s) == 0) return 0;
    if (max_label < 65536 && launch_lds<uint16_t>(base, n, P, seed, out, lds_limit, s) == 0)
        return 0;
    hipLaunchKernelGGL(k_permute_global, dim3((unsigned)ceil_div(P, 64)), dim3(64), 0, s, base, n,
                       P, seed, out);
    return 0;
}

int launch_permute_u16(const int32_t *base, int64_t n, int64_t P, uint64_t seed, int32_t max_label,
                       uint16_t *out, int64_t stride, size_t lds_limit, int n_cu, hipStream_t s) {
    if (P <= 0 || n <= 0) return 0;
    if (stride < n || max_label >= 65535) return 1;
    if (max_label < 4 &&
        launch_batch<CrumbStore>(base, n, P, seed, out, stride, lds_limit, n_cu, s) == 0)
        return 0;
    if (max_label < 16 &&
        launch_batch<NibbleStore>(base, n, P, seed, out, stride, lds_limit, n_cu, s) == 0)
        return 0;
    if (max_label < 256 &&
        launch_batch<WideStore<uint8_t>>(base, n, P, seed, out, stride, lds_limit, n_cu, s) == 0)
        return 0;
    if (launch_batch<WideStore<uint16_t>>(base, n, P, seed, out, stride, lds_limit, n_cu, s) == 0)
        return 0;
    return 1;
}

} // namespace pstat
