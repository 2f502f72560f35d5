/*
 * Operation count of the FP64 oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * hydro_oracle.c is compiled here as C++ with its floating-point type replaced by CountedReal, a
 * type of the same size and layout as a double whose arithmetic counts itself.  The library has
 * the oracle's C entry points (the ctypes binding loads it in place of liboracle.so) plus
 * or_opcount / or_opcount_reset, so that running the oracle's step on a workload yields the
 * floating-point operations the plain algorithm executes per cell and step: the algorithmic work
 * of one zone-cycle, with nothing recomputed and nothing fused.
 *
 * Counted: add/sub, mul, div, sqrt (one flop each), comparisons, min/max/abs, and the
 * transcendental calls of the set-up and the learned limiter (sin, cos, exp, tanh, log, pow).
 * Negation and conversions are not counted.  Work that the oracle marks as a repetition (each
 * face flux is evaluated by both neighbouring cells) is counted apart.
 */
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <math.h>
#include <stdlib.h>
#include <string.h>

namespace {
struct OpCounts {
    unsigned long long add, mul, div, sqrt, cmp, minmax_abs, transc;
};
OpCounts g_counts[2];  // [0] the algorithm's work, [1] work the oracle repeats (marked by it)
OpCounts* g_cur = &g_counts[0];
}  // namespace
#define g_ops (*g_cur)
#define OR_REPEATED_WORK(on) (g_cur = &g_counts[(on) ? 1 : 0])

struct CountedReal {
    double v;
    CountedReal() = default;
    constexpr CountedReal(double x) : v(x) {}
    constexpr CountedReal(int x) : v(x) {}
    constexpr CountedReal(long x) : v((double)x) {}
    constexpr CountedReal(long long x) : v((double)x) {}
    constexpr CountedReal(unsigned x) : v(x) {}
    constexpr CountedReal(unsigned long x) : v((double)x) {}
    explicit operator int() const { return (int)v; }
    explicit operator long() const { return (long)v; }
    explicit operator long long() const { return (long long)v; }
    explicit operator unsigned long() const { return (unsigned long)v; }
    explicit operator double() const { return v; }
    CountedReal operator-() const { return CountedReal(-v); }
    CountedReal operator+() const { return *this; }
    CountedReal& operator+=(CountedReal b)
    {
        g_ops.add++;
        v += b.v;
        return *this;
    }
    CountedReal& operator-=(CountedReal b)
    {
        g_ops.add++;
        v -= b.v;
        return *this;
    }
    CountedReal& operator*=(CountedReal b)
    {
        g_ops.mul++;
        v *= b.v;
        return *this;
    }
    CountedReal& operator/=(CountedReal b)
    {
        g_ops.div++;
        v /= b.v;
        return *this;
    }
};
static_assert(sizeof(CountedReal) == sizeof(double), "layout of a double");

inline CountedReal operator+(CountedReal a, CountedReal b) { g_ops.add++; return CountedReal(a.v + b.v); }
inline CountedReal operator-(CountedReal a, CountedReal b) { g_ops.add++; return CountedReal(a.v - b.v); }
inline CountedReal operator*(CountedReal a, CountedReal b) { g_ops.mul++; return CountedReal(a.v * b.v); }
inline CountedReal operator/(CountedReal a, CountedReal b) { g_ops.div++; return CountedReal(a.v / b.v); }
inline bool operator<(CountedReal a, CountedReal b) { g_ops.cmp++; return a.v < b.v; }
inline bool operator>(CountedReal a, CountedReal b) { g_ops.cmp++; return a.v > b.v; }
inline bool operator<=(CountedReal a, CountedReal b) { g_ops.cmp++; return a.v <= b.v; }
inline bool operator>=(CountedReal a, CountedReal b) { g_ops.cmp++; return a.v >= b.v; }
inline bool operator==(CountedReal a, CountedReal b) { g_ops.cmp++; return a.v == b.v; }
inline bool operator!=(CountedReal a, CountedReal b) { g_ops.cmp++; return a.v != b.v; }
inline bool operator!(CountedReal a) { g_ops.cmp++; return !a.v; }

inline CountedReal sqrt(CountedReal a) { g_ops.sqrt++; return CountedReal(std::sqrt(a.v)); }
inline CountedReal fabs(CountedReal a) { g_ops.minmax_abs++; return CountedReal(std::fabs(a.v)); }
inline CountedReal fmin(CountedReal a, CountedReal b) { g_ops.minmax_abs++; return CountedReal(std::fmin(a.v, b.v)); }
inline CountedReal fmax(CountedReal a, CountedReal b) { g_ops.minmax_abs++; return CountedReal(std::fmax(a.v, b.v)); }
inline CountedReal sin(CountedReal a) { g_ops.transc++; return CountedReal(std::sin(a.v)); }
inline CountedReal cos(CountedReal a) { g_ops.transc++; return CountedReal(std::cos(a.v)); }
inline CountedReal exp(CountedReal a) { g_ops.transc++; return CountedReal(std::exp(a.v)); }
inline CountedReal tanh(CountedReal a) { g_ops.transc++; return CountedReal(std::tanh(a.v)); }
inline CountedReal log(CountedReal a) { g_ops.transc++; return CountedReal(std::log(a.v)); }
inline CountedReal pow(CountedReal a, CountedReal b) { g_ops.transc++; return CountedReal(std::pow(a.v, b.v)); }
inline int isfinite(CountedReal a) { return std::isfinite(a.v); }
inline int isnan(CountedReal a) { return std::isnan(a.v); }

#define double CountedReal
#include "hydro_oracle.c"
#undef double

extern "C" {
/* out[14] = add/sub, mul, div, sqrt, comparisons, min/max/abs, transcendental calls since the
 * last reset: out[0..6] the algorithm's work, out[7..13] the work the oracle repeats */
void or_opcount(unsigned long long* out)
{
    for (int b = 0; b < 2; b++) {
        const OpCounts& c = g_counts[b];
        unsigned long long* o = out + 7 * b;
        o[0] = c.add;
        o[1] = c.mul;
        o[2] = c.div;
        o[3] = c.sqrt;
        o[4] = c.cmp;
        o[5] = c.minmax_abs;
        o[6] = c.transc;
    }
}
void or_opcount_reset(void)
{
    std::memset(g_counts, 0, sizeof g_counts);
    g_cur = &g_counts[0];
}
}
