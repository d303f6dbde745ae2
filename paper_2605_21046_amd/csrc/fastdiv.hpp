// Quotient by an invariant divisor with one high multiply (Granlund and Montgomery, "Division by
// invariant integers using multiplication", PLDI 1994): for 1 <= d < 2^32, with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, floor(n / d) = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0),
// t = floor(m n / 2^32), for every 32-bit n.  Built on the host, used by kernels (and by host tests).
#pragma once

#include <hip/hip_runtime.h>

namespace sg {

struct FastDiv {
    unsigned d, m;
    int s1, s2;
};

inline FastDiv make_fastdiv(unsigned d) {
    int l = 0;
    while ((1ull << l) < d) ++l;
    const unsigned long long m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
    return {d, (unsigned)m, l < 1 ? l : 1, l > 1 ? l - 1 : 0};
}

__host__ __device__ inline unsigned fast_quot(const FastDiv& f, unsigned n) {
    const unsigned t = (unsigned)(((unsigned long long)f.m * n) >> 32);
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

}  // namespace sg
