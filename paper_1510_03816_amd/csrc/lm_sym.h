// lm_sym.h -- the decomposition shared by the symmetric pair kernels (lm_sym.hip: the
// right-hand side; lm_sym_vjp.hip: its vector-Jacobian product).
//
// The 64-point tiles are grouped into superblocks of kSymRows * W tiles; a workgroup of W
// wavefronts takes one pair (X, Y), X <= Y, of superblocks: off-diagonal pairs first, numbered
// Y(Y-1)/2 + X, then the S diagonal ones, which carry half the work.  In a diagonal pair a row
// tile meets the column tiles after it from both sides, itself from one side (all 64 x 64
// ordered pairs, the self pair included) and skips the ones before it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lm_internal.h"

namespace lm {

constexpr int kSymSteps = 64;     // column points per tile
constexpr int kSymUnroll = 8;     // steps per unrolled loop body

// Superblock pair (X, Y) of workgroup b out of S(S+1)/2.
__device__ __forceinline__ void sym_superblocks(int64_t b, int64_t S, int64_t& X, int64_t& Y)
{
    const int64_t noff = S * (S - 1) / 2;
    if (b < noff) {
        int64_t y = (int64_t)(0.5 * (1.0 + __builtin_sqrt(1.0 + 8.0 * (double)b)));
        while (y * (y - 1) / 2 > b) --y;
        while ((y + 1) * y / 2 <= b) ++y;
        Y = y;
        X = b - y * (y - 1) / 2;
    } else {
        X = Y = b - noff;
    }
}

enum SymMode : int { SYM_SKIP = 0, SYM_ONE = 1, SYM_BOTH = 2 };

// What row tile I does with column tile J (NT tiles in all) in a diagonal or off-diagonal pair.
__device__ __forceinline__ int sym_mode(bool diag, int64_t I, int64_t J, int64_t NT)
{
    if (I >= NT) return SYM_SKIP;
    if (!diag || I < J) return SYM_BOTH;
    return I == J ? SYM_ONE : SYM_SKIP;
}

}  // namespace lm
