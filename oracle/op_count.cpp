/*
 * op_count.cpp -- operation counter of the FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY (like the oracle itself).  It compiles
 * rtgd_oracle.c unchanged, as C++, with every `double` of the oracle standing
 * for `Counted`: a number type that holds one double, performs exactly the
 * oracle's own arithmetic and counts each operation as it happens.  The
 * counting build therefore returns bit-identical results and counts the
 * operations of the method as the oracle writes it out.
 *
 * Counting rule: +, -, *, / and each libm call (sqrt, exp, sin, cos, atan2,
 * floor, ceil) count 1; a fused multiply-add would count 2 (the oracle has
 * none: it is built without contraction); negation, comparisons, copies and
 * integer arithmetic count 0.  Counters are process-wide and not thread
 * safe: the counting build has no OpenMP.
 *
 * Layout: Counted is a standard-layout struct of one double, so arrays of
 * doubles passed through the oracle's C interface are read in place, and a
 * Counted passed or returned by value travels like a double.
 */
#include <cmath>
#include <cstdlib>
#include <cstring>

namespace {

struct Tally {
    unsigned long long add, mul, div, lib;
} g_tally;

}  // namespace

struct Counted {
    double v;
    Counted() = default;
    Counted(double x) : v(x) {}
    Counted(int x) : v(double(x)) {}
    Counted(long x) : v(double(x)) {}
    Counted(long long x) : v(double(x)) {}
    explicit operator int() const { return int(v); }
    explicit operator long() const { return long(v); }
    explicit operator long long() const { return (long long)(v); }
    Counted &operator+=(Counted o) { ++g_tally.add; v += o.v; return *this; }
    Counted &operator-=(Counted o) { ++g_tally.add; v -= o.v; return *this; }
    Counted &operator*=(Counted o) { ++g_tally.mul; v *= o.v; return *this; }
    Counted &operator/=(Counted o) { ++g_tally.div; v /= o.v; return *this; }
};
static_assert(sizeof(Counted) == sizeof(double), "Counted must be laid out as a double");

inline Counted operator+(Counted a, Counted b) { ++g_tally.add; return a.v + b.v; }
inline Counted operator-(Counted a, Counted b) { ++g_tally.add; return a.v - b.v; }
inline Counted operator*(Counted a, Counted b) { ++g_tally.mul; return a.v * b.v; }
inline Counted operator/(Counted a, Counted b) { ++g_tally.div; return a.v / b.v; }
inline Counted operator-(Counted a) { return -a.v; }
inline Counted operator+(Counted a) { return a; }
inline bool operator<(Counted a, Counted b) { return a.v < b.v; }
inline bool operator>(Counted a, Counted b) { return a.v > b.v; }
inline bool operator<=(Counted a, Counted b) { return a.v <= b.v; }
inline bool operator>=(Counted a, Counted b) { return a.v >= b.v; }
inline bool operator==(Counted a, Counted b) { return a.v == b.v; }
inline bool operator!=(Counted a, Counted b) { return a.v != b.v; }
inline bool isfinite(Counted a) { return std::isfinite(a.v); }
inline Counted sqrt(Counted a) { ++g_tally.lib; return std::sqrt(a.v); }
inline Counted exp(Counted a) { ++g_tally.lib; return std::exp(a.v); }
inline Counted sin(Counted a) { ++g_tally.lib; return std::sin(a.v); }
inline Counted cos(Counted a) { ++g_tally.lib; return std::cos(a.v); }
inline Counted floor(Counted a) { ++g_tally.lib; return std::floor(a.v); }
inline Counted ceil(Counted a) { ++g_tally.lib; return std::ceil(a.v); }
inline Counted atan2(Counted a, Counted b) { ++g_tally.lib; return std::atan2(a.v, b.v); }

#define double Counted
#include "rtgd_oracle.c"
#undef double

extern "C" {

void or_count_reset(void) { std::memset(&g_tally, 0, sizeof(g_tally)); }

/* out = {add/sub, mul, div, libm calls} since the last reset */
void or_count_get(unsigned long long out[4])
{
    out[0] = g_tally.add;
    out[1] = g_tally.mul;
    out[2] = g_tally.div;
    out[3] = g_tally.lib;
}

}  // extern "C"
