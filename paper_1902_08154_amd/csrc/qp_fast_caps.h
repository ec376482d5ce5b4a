// qp_fast_caps.h -- waves per SIMD that the register allocation of each
// dense-sweep instantiation aims for: the highest value at which the compiler
// needs no scratch (spill) memory for that kernel.  build.py checks every
// kernel of the library for scratch use after compiling and lowers an entry
// here (rewriting this file) when a change makes that kernel spill.
#pragma once

// [adjoint][fingerprint][n_int - 1][n_states - 1]
constexpr int qpf_caps[2][2][4][4] = {
    {{{4, 3, 3, 2}, {3, 3, 3, 2}, {3, 3, 3, 2}, {2, 2, 2, 2}},
     {{3, 3, 3, 2}, {3, 3, 3, 2}, {3, 3, 2, 2}, {2, 2, 2, 2}}},
    {{{3, 2, 2, 2}, {3, 2, 2, 2}, {3, 2, 2, 2}, {2, 2, 2, 2}},
     {{3, 2, 2, 2}, {3, 2, 2, 1}, {3, 2, 2, 1}, {2, 2, 2, 1}}},
};
