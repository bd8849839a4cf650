// The 3x3x3-block part of the local bubble-splitting test (bubble model, end of
// Sec. 2.2: a bubble is a connected region of gas, D3Q19 neighbours connected).
// Pure functions of bit sets, compiled for the device (the splitting test) and for
// the host (the exactness check against a global labelling).
#pragma once

#include "fsl_device.hpp"

namespace fsl {

// block cells as a 27-bit set, bit (dx + 1) + 3 (dy + 1) + 9 (dz + 1); the centre is 13
// cells of the block one D3Q19 step away from a cell of m
__host__ __device__ __forceinline__ unsigned blk_step(unsigned m) {
    unsigned out = 0u;
    for (int b = 0; b < 27; ++b) {
        if (!((m >> b) & 1u)) continue;
        const int a0 = b % 3, a1 = (b / 3) % 3, a2 = b / 9;
        for (int q = 1; q < Q; ++q) {
            const int e0 = a0 + cx(q), e1 = a1 + cy(q), e2 = a2 + cz(q);
            if (e0 < 0 || e0 > 2 || e1 < 0 || e1 > 2 || e2 < 0 || e2 > 2) continue;
            out |= 1u << (e0 + 3 * e1 + 9 * e2);
        }
    }
    return out;
}

// The centre cell left the gas; gas: the block's cells that are still gas of its
// root bubble, rem: those that also left it in this step.  True when the root's gas
// stays connected for certain: (1) the gas neighbours of the centre are connected
// within the block, and (2) each neighbour that also left touches that connected
// set.  A gas path through a run of removed cells can then be rerouted through the
// block gas of each cell of the run.
__host__ __device__ __forceinline__ bool split_block_ok(unsigned gas, unsigned rem) {
    const unsigned n18 = blk_step(1u << 13);
    const unsigned s = gas & n18;
    if (!s) return true;
    unsigned comp = s & (~s + 1u);
    for (int it = 0; it < 27; ++it) {
        const unsigned grown = comp | (blk_step(comp) & gas);
        if (grown == comp) break;
        comp = grown;
    }
    if (s & ~comp) return false;
    for (unsigned rm = rem & n18; rm; rm &= rm - 1u)
        if (!(blk_step(rm & (~rm + 1u)) & comp)) return false;
    return true;
}

}  // namespace fsl
