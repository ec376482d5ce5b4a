// qp_fast_caps.h -- waves per SIMD that the register allocation of each
// dense-sweep instantiation aims for: the highest value at which the compiler
// needs no scratch (spill) memory for that kernel.  These are the defaults:
// build.py copies them to _build/qp_fast_caps_gen.h, which the kernel
// includes instead when it exists, and lowers an entry there when a compiler
// makes that kernel spill.  This file is not rewritten.
#pragma once

// [adjoint][fingerprint][n_int - 1][n_states - 1]
constexpr int qpf_caps[2][2][4][4] = {
    {{{4, 3, 3, 2}, {3, 3, 3, 2}, {3, 3, 3, 2}, {2, 2, 2, 2}},
     {{3, 3, 3, 2}, {3, 3, 3, 2}, {3, 3, 2, 2}, {2, 2, 2, 2}}},
    {{{3, 2, 2, 2}, {3, 2, 2, 2}, {3, 2, 2, 2}, {2, 2, 2, 2}},
     {{3, 2, 2, 2}, {3, 2, 2, 1}, {3, 2, 2, 1}, {2, 2, 2, 1}}},
};
