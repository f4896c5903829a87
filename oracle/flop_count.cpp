// flop_count.cpp -- TEST INFRASTRUCTURE ONLY: an instrumented build of the
// oracle that counts the floating-point operations the method performs.
//
// The oracle's own source (ppmlr_oracle.c, unchanged) is compiled as C++
// with every `double` replaced by `fd`, a value type that holds one double
// and counts each arithmetic operation applied to it: additions and
// subtractions, multiplications, divisions, square roots, comparisons, and
// min / max / |x| / sign selections.  The arithmetic itself is the plain FP64
// arithmetic of the oracle (the counts do not change any result), so the
// figures are the operation counts of the method as the oracle performs it,
// independent of how the GPU kernels are compiled.  Only oracle/flop_count.py
// (and through it the tests) loads the library this file builds.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

namespace fcount {
// single-threaded use only (the counting driver sets one OpenMP thread)
static long long n_add, n_mul, n_div, n_sqrt, n_cmp, n_sel;
}

struct fd {
    double v;
    fd() = default;
    fd(double x) : v(x) {}
    explicit operator double() const { return v; }
    explicit operator int() const { return (int)v; }
    explicit operator long() const { return (long)v; }
    explicit operator long long() const { return (long long)v; }
    explicit operator bool() const { return v != 0.0; }
    fd &operator+=(fd o) { ++fcount::n_add; v += o.v; return *this; }
    fd &operator-=(fd o) { ++fcount::n_add; v -= o.v; return *this; }
    fd &operator*=(fd o) { ++fcount::n_mul; v *= o.v; return *this; }
    fd &operator/=(fd o) { ++fcount::n_div; v /= o.v; return *this; }
};
static inline fd operator+(fd a, fd b) { ++fcount::n_add; return fd(a.v + b.v); }
static inline fd operator-(fd a, fd b) { ++fcount::n_add; return fd(a.v - b.v); }
static inline fd operator*(fd a, fd b) { ++fcount::n_mul; return fd(a.v * b.v); }
static inline fd operator/(fd a, fd b) { ++fcount::n_div; return fd(a.v / b.v); }
static inline fd operator-(fd a) { return fd(-a.v); }
static inline fd operator+(fd a) { return a; }
static inline bool operator<(fd a, fd b) { ++fcount::n_cmp; return a.v < b.v; }
static inline bool operator>(fd a, fd b) { ++fcount::n_cmp; return a.v > b.v; }
static inline bool operator<=(fd a, fd b) { ++fcount::n_cmp; return a.v <= b.v; }
static inline bool operator>=(fd a, fd b) { ++fcount::n_cmp; return a.v >= b.v; }
static inline bool operator==(fd a, fd b) { ++fcount::n_cmp; return a.v == b.v; }
static inline bool operator!=(fd a, fd b) { ++fcount::n_cmp; return a.v != b.v; }
static inline bool operator!(fd a) { return a.v == 0.0; }
static inline fd sqrt(fd a) { ++fcount::n_sqrt; return fd(::sqrt(a.v)); }
static inline fd fabs(fd a) { ++fcount::n_sel; return fd(::fabs(a.v)); }
static inline fd floor(fd a) { ++fcount::n_sel; return fd(::floor(a.v)); }
static inline bool isfinite(fd a) { return ::isfinite(a.v); }

static_assert(sizeof(fd) == sizeof(double), "fd has the layout of a double");

#define double fd
extern "C" {
#include "ppmlr_oracle.c"
}
#undef double

extern "C" {
void oracle_count_reset(void)
{
    fcount::n_add = fcount::n_mul = fcount::n_div = fcount::n_sqrt = fcount::n_cmp = fcount::n_sel = 0;
}
// out: additions/subtractions, multiplications, divisions, square roots,
// comparisons, selections (min / max / |x| / floor)
void oracle_count_get(long long out[6])
{
    out[0] = fcount::n_add;
    out[1] = fcount::n_mul;
    out[2] = fcount::n_div;
    out[3] = fcount::n_sqrt;
    out[4] = fcount::n_cmp;
    out[5] = fcount::n_sel;
}
}
