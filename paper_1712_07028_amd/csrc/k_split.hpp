// Bubble splitting (bubble model, end of Sec. 2.2): a bubble is a connected region of
// gas, so a bubble whose gas falls apart becomes several bubbles.
//
// Two gas cells are connected when they are D3Q19 neighbours (the neighbourhood of
// the merge rule) and belong to the same root bubble.  Where the gas of a root falls
// into several parts, the part holding the lowest cell index keeps the bubble and
// the others, in order of their lowest cell index, take the lowest ids that are not
// alive (merges relabel the cells to their roots, so merged ids are free); an
// interface cell goes with the part of its gas neighbours (the lowest when they
// differ) and stays with the bubble without any; the gas mass is shared in
// proportion to the parts' volumes (gas cells plus 1 - phi of their interface
// cells), so that every part starts at the density of its bubble.
//
// The gas of a bubble can only come apart in a step where gas cells leave the gas
// phase (new interface cells, cells covered by a particle), where cells enter it
// (emptied cells, cells uncovered as gas) or where bubbles merge.  A cell that left
// is tested on its 3x3x3 block, a cell that entered must touch older gas of its
// bubble, and a merge always asks for labelling; only then does a union-find
// labelling of all gas cells run.  The tests are exact given that every root's gas
// was connected before the step, which the labelling establishes at initialisation
// and whenever tables or particles are set.
#pragma once

#include "k_particles.hpp"
#include "split_block.hpp"

namespace fsl {

constexpr int SPLIT_MAXC = 1024;  // gas components one labelling may list

struct SplitBuf {
    int *lab;     // per gas cell: union-find link, then the part's lowest cell index;
                  // at that cell, -(slot + 2) once the parts are numbered
    int *comp;    // lowest cell index of each part, in discovery order
    int *cid;     // per slot (parts by lowest cell index): new bubble id, -1 = keeps its id
    int *parent;  // per slot: root bubble
    double *vol;  // per slot: volume of a part that takes a new id
};

// ---- local test on the 3x3x3 block ------------------------------------------------
__device__ __forceinline__ int blk_cell(const Geom &G, int x, int y, int z, int dx, int dy, int dz) {
    int a = x + dx, b = y + dy, d = z + dz;
    if (a < 0 || a >= G.nx) { if (!G.per[0]) return -1; a = wrapc(a, G.nx); }
    if (b < 0 || b >= G.ny) { if (!G.per[1]) return -1; b = wrapc(b, G.ny); }
    if (d < 0 || d >= G.nz) { if (!G.per[2]) return -1; d = wrapc(d, G.nz); }
    return a + G.nx * (b + G.ny * d);
}

// Cell c left the gas phase: its block's gas and removed cells of its root, tested by
// split_block_ok.
__device__ bool split_local_ok(const Geom &G, const Dev &D, int c) {
    int x, y, z;
    cell_xyz(G, c, x, y, z);
    const int r = bubble_root(D, D.bub[c]);
    unsigned gas = 0u, rem = 0u;
    for (int b = 0; b < 27; ++b) {
        if (b == 13) continue;
        const int n = blk_cell(G, x, y, z, b % 3 - 1, (b / 3) % 3 - 1, b / 9 - 1);
        if (n < 0) continue;
        if (D.flags[n] == GAS) {
            if (bubble_root(D, D.bub[n]) == r) gas |= 1u << b;
        } else if ((D.cv[n] & CV_GRM) && bubble_root(D, D.bub[n]) == r) {
            rem |= 1u << b;
        }
    }
    return split_block_ok(gas, rem);
}

// Cell c entered the gas phase: it joins the older gas of its root (gas before the
// step and still gas) through a D3Q19 neighbour.
__device__ bool split_added_ok(const Geom &G, const Dev &D, int c) {
    int x, y, z;
    cell_xyz(G, c, x, y, z);
    const int r = bubble_root(D, D.bub[c]);
    for (int q = 1; q < Q; ++q) {
        const int n = nbr_idx(G, x, y, z, q, 1);
        if (n >= 0 && D.flags[n] == GAS && !(D.cv[n] & CV_GAD) && bubble_root(D, D.bub[n]) == r) return true;
    }
    return false;
}

// the step's cells that left the gas (new interface cells from gas, covered gas
// cells: CV_GRM) and that entered it (emptied cells, cells uncovered as gas: CV_GAD),
// taken from the step's lists in that order
__device__ __forceinline__ int split_cell(const Dev &D, int i, int nG, int nC, int nE) {
    if (i < nG) return D.lNG[i];
    i -= nG;
    if (i < nC) return D.lCov[2 * i];
    i -= nC;
    if (i < nE) return D.lE[i];
    return D.lUnc[2 * (i - nE)];
}

// a failed test or a merge in this step asks for labelling
__global__ void k_split_test(Geom G, Dev D) {
    const int nG = list_len(D, C_NNG), nC = event_len(D, C_NCOVER);
    const int nE = list_len(D, C_NE), nU = event_len(D, C_NUNCOVER);
    // a periodic axis shorter than the block folds it onto itself: always label
    const bool fold = (G.per[0] && G.nx < 3) || (G.per[1] && G.ny < 3) || (G.per[2] && G.nz < 3);
    if (blockIdx.x == 0 && threadIdx.x == 0 && D.counters[C_NMERGE] > 0) atomicOr(D.counters + C_SPLIT, 1);
    GRID_STRIDE(i, nG + nC + nE + nU) {
        const int c = split_cell(D, i, nG, nC, nE);
        const uint8_t m = D.cv[c];
        bool ok = true;
        if (m & CV_GRM) ok = !fold && split_local_ok(G, D, c);
        else if (m & CV_GAD) ok = split_added_ok(G, D, c);
        if (!ok) atomicOr(D.counters + C_SPLIT, 1);
    }
}


// labelling of the current state regardless of the test (initial state, new tables
// or particles)
__global__ void k_split_force(Dev D) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        D.counters[C_SPLIT] = 1;
        D.counters[C_NCOMP] = 0;
    }
}

// ---- labelling: union-find over the gas cells -------------------------------------
// Links only ever point to a lower cell index, so every part ends at its lowest cell.
__device__ __forceinline__ int lab_get(const int *lab, int x) {
    return __hip_atomic_load(lab + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int lab_find(const int *lab, int x) {
    for (;;) {
        const int p = lab_get(lab, x);
        if (p == x) return x;
        x = p;
    }
}

// join the parts of a and b: the higher root is linked below the lower one; a root
// relinked by another thread meanwhile is followed and joined in turn (the larger of
// the two indices falls every round, so this ends)
__device__ void lab_unite(int *lab, int a, int b) {
    for (;;) {
        a = lab_find(lab, a);
        b = lab_find(lab, b);
        if (a == b) return;
        if (a < b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicMin(lab + a, b);
        if (old == a) return;
        a = old;
    }
}

#define CELL_STRIDE(c, n)                                                                      \
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < (n);              \
         c += (long long)gridDim.x * blockDim.x)

// clears the marks the test read (cv is zero outside the conversion phase), then
// starts the labelling: every gas cell its own part
__global__ void k_ccl_init(Geom G, Dev D, SplitBuf B) {
    const int nG = list_len(D, C_NNG), nC = event_len(D, C_NCOVER);
    const int nE = list_len(D, C_NE), nU = event_len(D, C_NUNCOVER);
    GRID_STRIDE(i, nG + nC + nE + nU) D.cv[split_cell(D, i, nG, nC, nE)] = 0;
    if (D.counters[C_SPLIT] == 0) return;
    CELL_STRIDE(c, G.N) if (D.flags[c] == GAS) B.lab[c] = (int)c;
}

__global__ void k_ccl_union(Geom G, Dev D, SplitBuf B) {
    if (D.counters[C_SPLIT] == 0) return;
    CELL_STRIDE(c, G.N) {
        if (D.flags[c] != GAS) continue;
        int x, y, z;
        cell_xyz(G, (int)c, x, y, z);
        const int r = bubble_root(D, D.bub[c]);
        for (int q = 1; q < Q; ++q) {
            if (opp(q) < q) continue;  // one direction of each pair
            const int n = nbr_idx(G, x, y, z, q, 1);
            if (n < 0 || D.flags[n] != GAS || bubble_root(D, D.bub[n]) != r) continue;
            lab_unite(B.lab, (int)c, n);
        }
    }
}

// every gas cell links straight to its part's lowest cell (a concurrent find only
// ever sees a link to an ancestor); the parts' lowest cells are listed
__global__ void k_ccl_flatten(Geom G, Dev D, SplitBuf B) {
    if (D.counters[C_SPLIT] == 0) return;
    CELL_STRIDE(c, G.N) {
        if (D.flags[c] != GAS) continue;
        const int root = lab_find(B.lab, (int)c);
        if (root != (int)c) {
            __hip_atomic_store(B.lab + c, root, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        const int s = atomicAdd(D.counters + C_NCOMP, 1);
        if (s < SPLIT_MAXC) B.comp[s] = (int)c;
        else atomicOr(D.err, ERR_CAP);
    }
}

// parts in order of their lowest cell index: the first part of each root keeps it,
// the others take the lowest ids that are not alive
__global__ __launch_bounds__(1024) void k_split_plan(Dev D, SplitBuf B, int open) {
    if (D.counters[C_SPLIT] == 0) return;
    __shared__ int sorted[SPLIT_MAXC];
    __shared__ unsigned char seen[64], taken[64];
    if (D.counters[C_NCOMP] > SPLIT_MAXC) {  // not every part listed: no split, error set
        if (threadIdx.x == 0) D.counters[C_SPLIT] = 1;
        return;
    }
    const int n = D.counters[C_NCOMP];
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const int v = B.comp[k];
        int rank = 0;
        for (int j = 0; j < n; ++j) rank += B.comp[j] < v;
        sorted[rank] = v;
    }
    for (int i = threadIdx.x; i < 64; i += blockDim.x) seen[i] = taken[i] = 0;
    __syncthreads();
    if (threadIdx.x) return;
    int used = D.counters[C_BUSED], any = 0;
    for (int k = 0; k < n; ++k) {
        const int c = sorted[k];
        const int r = bubble_root(D, D.bub[c]);
        int id = -1;
        if (r == 0 && open) {
            // every part of an open atmosphere stays at the outlet
        } else if (!seen[r]) {
            seen[r] = 1;
        } else {
            // the lowest id that is not alive: never used, or merged away (merges
            // relabel the cells to their roots)
            int b = 1;
            while (b < D.maxB && (D.balive[b] || taken[b])) ++b;
            if (b < D.maxB) {
                id = b;
                taken[b] = 1;
                used = max(used, b + 1);
                any = 1;
            } else {
                atomicOr(D.err, ERR_CAP);
            }
        }
        B.cid[k] = id;
        B.parent[k] = r;
        B.vol[k] = 0.0;
        B.lab[c] = -(k + 2);
    }
    D.counters[C_BUSED] = used;
    D.counters[C_SPLIT] = any ? 2 : 1;
}

__device__ __forceinline__ int lab_slot(const int *lab, int c) {
    const int l = lab[c];
    return l < 0 ? -l - 2 : -lab[l] - 2;
}

// interface cells first: they find their part through the ids of their gas
// neighbours, which the next kernel changes
__global__ void k_split_ifc(Geom G, Dev D, SplitBuf B, const double *phi) {
    if (D.counters[C_SPLIT] != 2) return;
    CELL_STRIDE(c, G.N) {
        if (D.flags[c] != IFC) continue;
        int x, y, z;
        cell_xyz(G, (int)c, x, y, z);
        const int r = bubble_root(D, D.bub[c]);
        int best = -1;
        for (int q = 1; q < Q; ++q) {
            const int n = nbr_idx(G, x, y, z, q, 1);
            if (n < 0 || D.flags[n] != GAS || bubble_root(D, D.bub[n]) != r) continue;
            const int l = B.lab[n];
            const int rep = l < 0 ? n : l;
            if (best < 0 || rep < best) best = rep;
        }
        if (best < 0) continue;
        const int k = -B.lab[best] - 2;
        const int id = B.cid[k];
        if (id < 0) continue;
        D.bub[c] = (uint16_t)id;
        unsafeAtomicAdd(B.vol + k, 1.0 - phi[c]);
    }
}

// gas cells: 16 consecutive cells per thread, their count summed per part
__global__ void k_split_gas(Geom G, Dev D, SplitBuf B) {
    if (D.counters[C_SPLIT] != 2) return;
    const long long nchunk = (G.N + 15) / 16;
    int ks = -1;
    double acc = 0.0;
    for (long long ch = blockIdx.x * (long long)blockDim.x + threadIdx.x; ch < nchunk;
         ch += (long long)gridDim.x * blockDim.x) {
        for (long long c = ch * 16; c < ch * 16 + 16 && c < G.N; ++c) {
            if (D.flags[c] != GAS) continue;
            const int k = lab_slot(B.lab, (int)c);
            const int id = B.cid[k];
            if (id < 0) continue;
            D.bub[c] = (uint16_t)id;
            if (k != ks) {
                if (ks >= 0) unsafeAtomicAdd(B.vol + ks, acc);
                ks = k;
                acc = 0.0;
            }
            acc += 1.0;
        }
    }
    if (ks >= 0) unsafeAtomicAdd(B.vol + ks, acc);
}

// gas masses of the new bubbles: M_part = M_root V_part / V_root, the root keeps
// the rest (the root volumes are those of the state before the split); the block
// also clears the volume sums for the recount that follows
__global__ void k_split_mass(Dev D, SplitBuf B) {
    if (D.counters[C_SPLIT] != 2 || blockIdx.x) return;
    for (int i = threadIdx.x; i < D.nb * BACC_STRIDE; i += blockDim.x) D.bacc[i] = 0.0;
    if (threadIdx.x) return;
    __shared__ double Mr[64], taken[64];
    for (int r = 0; r < D.maxB; ++r) {
        Mr[r] = D.btab[r * B_STRIDE + B_M];
        taken[r] = 0.0;
    }
    const int n = min(D.counters[C_NCOMP], SPLIT_MAXC);
    for (int k = 0; k < n; ++k) {
        const int id = B.cid[k];
        if (id < 0) continue;
        const int r = B.parent[k];
        double *t = D.btab + id * B_STRIDE;
        t[B_M] = Mr[r] * B.vol[k] / D.btab[r * B_STRIDE + B_V];
        t[B_V0] = B.vol[k];
        D.broot[id] = id;
        D.balive[id] = 1;
        taken[r] += t[B_M];
    }
    for (int r = 0; r < D.maxB; ++r)
        if (taken[r] != 0.0) D.btab[r * B_STRIDE + B_M] = Mr[r] - taken[r];
}

}  // namespace fsl
