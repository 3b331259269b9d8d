// Independent reference for the oracle's 64-bit finaliser: pybind11 ships its own copy of
// Stafford's variant 13 of the MurmurHash3 finaliser (the SplitMix64 output function,
// Steele, Lea and Flood, OOPSLA 2014) as pybind11::detail::mix64.  This program only runs
// that function: one hexadecimal input per line on stdin, one hexadecimal output per line.
#include <pybind11/detail/internals.h>

#include <cinttypes>
#include <cstdio>

int main() {
    unsigned long long x;
    while (std::scanf("%llx", &x) == 1)
        std::printf("%016" PRIx64 "\n", pybind11::detail::mix64(static_cast<std::uint64_t>(x)));
    return 0;
}
