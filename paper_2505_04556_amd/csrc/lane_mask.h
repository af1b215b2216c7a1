// Masked adds: acc += d[c] for each c < N with y[c] == x, in order of c.
//
// The N compares write N lane masks (SGPR pairs); then, for each c in turn,
// the mask becomes EXEC and one add runs, so only the lanes whose labels match
// add.  EXEC is saved first and restored before the statement ends.  Two
// vector operations (compare, add) and one scalar move per term, where a
// select-based form needs three vector operations (compare, select, add) in
// FP32 and four in FP64; the sums are the same, term by term, in the same
// order.  Every lane that enters must be active in EXEC on entry (the caller's
// code is not divergent here).
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace pstat {

__device__ inline void masked_add16(float &acc, uint32_t x, const uint32_t *y, const float *d) {
    uint64_t m[16], sv;
    asm volatile(
        "v_cmp_eq_u32_e64 %[m0], %[x], %[y0]\n"
        "v_cmp_eq_u32_e64 %[m1], %[x], %[y1]\n"
        "v_cmp_eq_u32_e64 %[m2], %[x], %[y2]\n"
        "v_cmp_eq_u32_e64 %[m3], %[x], %[y3]\n"
        "v_cmp_eq_u32_e64 %[m4], %[x], %[y4]\n"
        "v_cmp_eq_u32_e64 %[m5], %[x], %[y5]\n"
        "v_cmp_eq_u32_e64 %[m6], %[x], %[y6]\n"
        "v_cmp_eq_u32_e64 %[m7], %[x], %[y7]\n"
        "v_cmp_eq_u32_e64 %[m8], %[x], %[y8]\n"
        "v_cmp_eq_u32_e64 %[m9], %[x], %[y9]\n"
        "v_cmp_eq_u32_e64 %[m10], %[x], %[y10]\n"
        "v_cmp_eq_u32_e64 %[m11], %[x], %[y11]\n"
        "v_cmp_eq_u32_e64 %[m12], %[x], %[y12]\n"
        "v_cmp_eq_u32_e64 %[m13], %[x], %[y13]\n"
        "v_cmp_eq_u32_e64 %[m14], %[x], %[y14]\n"
        "v_cmp_eq_u32_e64 %[m15], %[x], %[y15]\n"
        "s_mov_b64 %[sv], exec\n"
        "s_mov_b64 exec, %[m0]\n"
        "v_add_f32 %[acc], %[acc], %[d0]\n"
        "s_mov_b64 exec, %[m1]\n"
        "v_add_f32 %[acc], %[acc], %[d1]\n"
        "s_mov_b64 exec, %[m2]\n"
        "v_add_f32 %[acc], %[acc], %[d2]\n"
        "s_mov_b64 exec, %[m3]\n"
        "v_add_f32 %[acc], %[acc], %[d3]\n"
        "s_mov_b64 exec, %[m4]\n"
        "v_add_f32 %[acc], %[acc], %[d4]\n"
        "s_mov_b64 exec, %[m5]\n"
        "v_add_f32 %[acc], %[acc], %[d5]\n"
        "s_mov_b64 exec, %[m6]\n"
        "v_add_f32 %[acc], %[acc], %[d6]\n"
        "s_mov_b64 exec, %[m7]\n"
        "v_add_f32 %[acc], %[acc], %[d7]\n"
        "s_mov_b64 exec, %[m8]\n"
        "v_add_f32 %[acc], %[acc], %[d8]\n"
        "s_mov_b64 exec, %[m9]\n"
        "v_add_f32 %[acc], %[acc], %[d9]\n"
        "s_mov_b64 exec, %[m10]\n"
        "v_add_f32 %[acc], %[acc], %[d10]\n"
        "s_mov_b64 exec, %[m11]\n"
        "v_add_f32 %[acc], %[acc], %[d11]\n"
        "s_mov_b64 exec, %[m12]\n"
        "v_add_f32 %[acc], %[acc], %[d12]\n"
        "s_mov_b64 exec, %[m13]\n"
        "v_add_f32 %[acc], %[acc], %[d13]\n"
        "s_mov_b64 exec, %[m14]\n"
        "v_add_f32 %[acc], %[acc], %[d14]\n"
        "s_mov_b64 exec, %[m15]\n"
        "v_add_f32 %[acc], %[acc], %[d15]\n"
        "s_mov_b64 exec, %[sv]\n"
        : [acc] "+v"(acc), [m0] "=&s"(m[0]), [m1] "=&s"(m[1]), [m2] "=&s"(m[2]), [m3] "=&s"(m[3]), [m4] "=&s"(m[4]), [m5] "=&s"(m[5]), [m6] "=&s"(m[6]), [m7] "=&s"(m[7]), [m8] "=&s"(m[8]), [m9] "=&s"(m[9]), [m10] "=&s"(m[10]), [m11] "=&s"(m[11]), [m12] "=&s"(m[12]), [m13] "=&s"(m[13]), [m14] "=&s"(m[14]), [m15] "=&s"(m[15]), [sv] "=&s"(sv)
        : [x] "v"(x), [y0] "v"(y[0]), [y1] "v"(y[1]), [y2] "v"(y[2]), [y3] "v"(y[3]), [y4] "v"(y[4]), [y5] "v"(y[5]), [y6] "v"(y[6]), [y7] "v"(y[7]), [y8] "v"(y[8]), [y9] "v"(y[9]), [y10] "v"(y[10]), [y11] "v"(y[11]), [y12] "v"(y[12]), [y13] "v"(y[13]), [y14] "v"(y[14]), [y15] "v"(y[15]), [d0] "v"(d[0]), [d1] "v"(d[1]), [d2] "v"(d[2]), [d3] "v"(d[3]), [d4] "v"(d[4]), [d5] "v"(d[5]), [d6] "v"(d[6]), [d7] "v"(d[7]), [d8] "v"(d[8]), [d9] "v"(d[9]), [d10] "v"(d[10]), [d11] "v"(d[11]), [d12] "v"(d[12]), [d13] "v"(d[13]), [d14] "v"(d[14]), [d15] "v"(d[15]));
}

__device__ inline void masked_add16(double &acc, uint32_t x, const uint32_t *y, const double *d) {
    uint64_t m[16], sv;
    asm volatile(
        "v_cmp_eq_u32_e64 %[m0], %[x], %[y0]\n"
        "v_cmp_eq_u32_e64 %[m1], %[x], %[y1]\n"
        "v_cmp_eq_u32_e64 %[m2], %[x], %[y2]\n"
        "v_cmp_eq_u32_e64 %[m3], %[x], %[y3]\n"
        "v_cmp_eq_u32_e64 %[m4], %[x], %[y4]\n"
        "v_cmp_eq_u32_e64 %[m5], %[x], %[y5]\n"
        "v_cmp_eq_u32_e64 %[m6], %[x], %[y6]\n"
        "v_cmp_eq_u32_e64 %[m7], %[x], %[y7]\n"
        "v_cmp_eq_u32_e64 %[m8], %[x], %[y8]\n"
        "v_cmp_eq_u32_e64 %[m9], %[x], %[y9]\n"
        "v_cmp_eq_u32_e64 %[m10], %[x], %[y10]\n"
        "v_cmp_eq_u32_e64 %[m11], %[x], %[y11]\n"
        "v_cmp_eq_u32_e64 %[m12], %[x], %[y12]\n"
        "v_cmp_eq_u32_e64 %[m13], %[x], %[y13]\n"
        "v_cmp_eq_u32_e64 %[m14], %[x], %[y14]\n"
        "v_cmp_eq_u32_e64 %[m15], %[x], %[y15]\n"
        "s_mov_b64 %[sv], exec\n"
        "s_mov_b64 exec, %[m0]\n"
        "v_add_f64 %[acc], %[acc], %[d0]\n"
        "s_mov_b64 exec, %[m1]\n"
        "v_add_f64 %[acc], %[acc], %[d1]\n"
        "s_mov_b64 exec, %[m2]\n"
        "v_add_f64 %[acc], %[acc], %[d2]\n"
        "s_mov_b64 exec, %[m3]\n"
        "v_add_f64 %[acc], %[acc], %[d3]\n"
        "s_mov_b64 exec, %[m4]\n"
        "v_add_f64 %[acc], %[acc], %[d4]\n"
        "s_mov_b64 exec, %[m5]\n"
        "v_add_f64 %[acc], %[acc], %[d5]\n"
        "s_mov_b64 exec, %[m6]\n"
        "v_add_f64 %[acc], %[acc], %[d6]\n"
        "s_mov_b64 exec, %[m7]\n"
        "v_add_f64 %[acc], %[acc], %[d7]\n"
        "s_mov_b64 exec, %[m8]\n"
        "v_add_f64 %[acc], %[acc], %[d8]\n"
        "s_mov_b64 exec, %[m9]\n"
        "v_add_f64 %[acc], %[acc], %[d9]\n"
        "s_mov_b64 exec, %[m10]\n"
        "v_add_f64 %[acc], %[acc], %[d10]\n"
        "s_mov_b64 exec, %[m11]\n"
        "v_add_f64 %[acc], %[acc], %[d11]\n"
        "s_mov_b64 exec, %[m12]\n"
        "v_add_f64 %[acc], %[acc], %[d12]\n"
        "s_mov_b64 exec, %[m13]\n"
        "v_add_f64 %[acc], %[acc], %[d13]\n"
        "s_mov_b64 exec, %[m14]\n"
        "v_add_f64 %[acc], %[acc], %[d14]\n"
        "s_mov_b64 exec, %[m15]\n"
        "v_add_f64 %[acc], %[acc], %[d15]\n"
        "s_mov_b64 exec, %[sv]\n"
        : [acc] "+v"(acc), [m0] "=&s"(m[0]), [m1] "=&s"(m[1]), [m2] "=&s"(m[2]), [m3] "=&s"(m[3]), [m4] "=&s"(m[4]), [m5] "=&s"(m[5]), [m6] "=&s"(m[6]), [m7] "=&s"(m[7]), [m8] "=&s"(m[8]), [m9] "=&s"(m[9]), [m10] "=&s"(m[10]), [m11] "=&s"(m[11]), [m12] "=&s"(m[12]), [m13] "=&s"(m[13]), [m14] "=&s"(m[14]), [m15] "=&s"(m[15]), [sv] "=&s"(sv)
        : [x] "v"(x), [y0] "v"(y[0]), [y1] "v"(y[1]), [y2] "v"(y[2]), [y3] "v"(y[3]), [y4] "v"(y[4]), [y5] "v"(y[5]), [y6] "v"(y[6]), [y7] "v"(y[7]), [y8] "v"(y[8]), [y9] "v"(y[9]), [y10] "v"(y[10]), [y11] "v"(y[11]), [y12] "v"(y[12]), [y13] "v"(y[13]), [y14] "v"(y[14]), [y15] "v"(y[15]), [d0] "v"(d[0]), [d1] "v"(d[1]), [d2] "v"(d[2]), [d3] "v"(d[3]), [d4] "v"(d[4]), [d5] "v"(d[5]), [d6] "v"(d[6]), [d7] "v"(d[7]), [d8] "v"(d[8]), [d9] "v"(d[9]), [d10] "v"(d[10]), [d11] "v"(d[11]), [d12] "v"(d[12]), [d13] "v"(d[13]), [d14] "v"(d[14]), [d15] "v"(d[15]));
}

// Two sums at once over the same eight terms d: a0 over the c with
// y0[c] == x0, a1 over those with y1[c] == x1, each in order of c; the adds
// of the two alternate, so neither waits on its own previous add.
__device__ inline void masked_add8_pair(double &a0, uint32_t x0, const uint32_t *y0, double &a1,
                                      uint32_t x1, const uint32_t *y1, const double *d) {
    uint64_t m[8], n[8], sv;
    asm volatile(
        "v_cmp_eq_u32_e64 %[m0], %[x0], %[y00]\n"
        "v_cmp_eq_u32_e64 %[n0], %[x1], %[y10]\n"
        "v_cmp_eq_u32_e64 %[m1], %[x0], %[y01]\n"
        "v_cmp_eq_u32_e64 %[n1], %[x1], %[y11]\n"
        "v_cmp_eq_u32_e64 %[m2], %[x0], %[y02]\n"
        "v_cmp_eq_u32_e64 %[n2], %[x1], %[y12]\n"
        "v_cmp_eq_u32_e64 %[m3], %[x0], %[y03]\n"
        "v_cmp_eq_u32_e64 %[n3], %[x1], %[y13]\n"
        "v_cmp_eq_u32_e64 %[m4], %[x0], %[y04]\n"
        "v_cmp_eq_u32_e64 %[n4], %[x1], %[y14]\n"
        "v_cmp_eq_u32_e64 %[m5], %[x0], %[y05]\n"
        "v_cmp_eq_u32_e64 %[n5], %[x1], %[y15]\n"
        "v_cmp_eq_u32_e64 %[m6], %[x0], %[y06]\n"
        "v_cmp_eq_u32_e64 %[n6], %[x1], %[y16]\n"
        "v_cmp_eq_u32_e64 %[m7], %[x0], %[y07]\n"
        "v_cmp_eq_u32_e64 %[n7], %[x1], %[y17]\n"
        "s_mov_b64 %[sv], exec\n"
        "s_mov_b64 exec, %[m0]\n"
        "v_add_f64 %[a0], %[a0], %[d0]\n"
        "s_mov_b64 exec, %[n0]\n"
        "v_add_f64 %[a1], %[a1], %[d0]\n"
        "s_mov_b64 exec, %[m1]\n"
        "v_add_f64 %[a0], %[a0], %[d1]\n"
        "s_mov_b64 exec, %[n1]\n"
        "v_add_f64 %[a1], %[a1], %[d1]\n"
        "s_mov_b64 exec, %[m2]\n"
        "v_add_f64 %[a0], %[a0], %[d2]\n"
        "s_mov_b64 exec, %[n2]\n"
        "v_add_f64 %[a1], %[a1], %[d2]\n"
        "s_mov_b64 exec, %[m3]\n"
        "v_add_f64 %[a0], %[a0], %[d3]\n"
        "s_mov_b64 exec, %[n3]\n"
        "v_add_f64 %[a1], %[a1], %[d3]\n"
        "s_mov_b64 exec, %[m4]\n"
        "v_add_f64 %[a0], %[a0], %[d4]\n"
        "s_mov_b64 exec, %[n4]\n"
        "v_add_f64 %[a1], %[a1], %[d4]\n"
        "s_mov_b64 exec, %[m5]\n"
        "v_add_f64 %[a0], %[a0], %[d5]\n"
        "s_mov_b64 exec, %[n5]\n"
        "v_add_f64 %[a1], %[a1], %[d5]\n"
        "s_mov_b64 exec, %[m6]\n"
        "v_add_f64 %[a0], %[a0], %[d6]\n"
        "s_mov_b64 exec, %[n6]\n"
        "v_add_f64 %[a1], %[a1], %[d6]\n"
        "s_mov_b64 exec, %[m7]\n"
        "v_add_f64 %[a0], %[a0], %[d7]\n"
        "s_mov_b64 exec, %[n7]\n"
        "v_add_f64 %[a1], %[a1], %[d7]\n"
        "s_mov_b64 exec, %[sv]\n"
        : [a0] "+v"(a0), [a1] "+v"(a1), [m0] "=&s"(m[0]), [m1] "=&s"(m[1]), [m2] "=&s"(m[2]), [m3] "=&s"(m[3]), [m4] "=&s"(m[4]), [m5] "=&s"(m[5]), [m6] "=&s"(m[6]), [m7] "=&s"(m[7]), [n0] "=&s"(n[0]), [n1] "=&s"(n[1]), [n2] "=&s"(n[2]), [n3] "=&s"(n[3]), [n4] "=&s"(n[4]), [n5] "=&s"(n[5]), [n6] "=&s"(n[6]), [n7] "=&s"(n[7]), [sv] "=&s"(sv)
        : [x0] "v"(x0), [x1] "v"(x1), [y00] "v"(y0[0]), [y01] "v"(y0[1]), [y02] "v"(y0[2]), [y03] "v"(y0[3]), [y04] "v"(y0[4]), [y05] "v"(y0[5]), [y06] "v"(y0[6]), [y07] "v"(y0[7]), [y10] "v"(y1[0]), [y11] "v"(y1[1]), [y12] "v"(y1[2]), [y13] "v"(y1[3]), [y14] "v"(y1[4]), [y15] "v"(y1[5]), [y16] "v"(y1[6]), [y17] "v"(y1[7]), [d0] "v"(d[0]), [d1] "v"(d[1]), [d2] "v"(d[2]), [d3] "v"(d[3]), [d4] "v"(d[4]), [d5] "v"(d[5]), [d6] "v"(d[6]), [d7] "v"(d[7]));
}

} // namespace pstat
