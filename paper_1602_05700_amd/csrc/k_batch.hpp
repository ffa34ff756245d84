// Batched substeps: many independent grids of uneven sizes advanced together.
//
// One launch covers every grid: a persistent grid of workgroups walks a work
// list of (grid, tile, z chunk) items sorted by decreasing cost, workgroup b
// taking items b, b + G, b + 2G, ... (a static longest-first assignment:
// deterministic, no counters to reset).  Per-grid geometry, coefficients and
// buffers come from a descriptor array in device memory.  The tile bodies are
// the single-grid ones, so a batched step is bit-identical to stepping each
// grid alone.  The host captures the nsub-substep sequence of launches in a
// hipGraph and replays it every hydrodynamical step.
#pragma once

#include "common.hpp"
#include "k_stencil.hpp"
#include "k_tblock.hpp"

namespace hgs {

template <typename S>
struct GridDesc {
    Layout L;
    StepCoef c;
    S* buf[4];      // padded state buffers of the grid
    const S* rho;   // this hydro step's density (compact)
};

struct WorkItem {
    int grid, tx, ty, k0, k1;
};

// tile shape of the batched fused launches: the default shape of each depth
template <typename S, int T>
struct BatchTile {
    static constexpr int R = TileSet<S, T>::at(0).R;
    static constexpr int W = TileSet<S, T>::at(0).W;
    static constexpr int PF = TileSet<S, T>::at(0).PF;
    static constexpr bool SB = TileSet<S, T>::at(0).SB;
    static constexpr bool UPF = TileSet<S, T>::at(0).UPF;
};

// T fused substeps on every grid: (buf[in0], buf[in1]) -> (buf[out0], buf[out1])
template <typename S, int T, int R, int W, int PF, bool SB, bool UPF>
__global__ __launch_bounds__(64 * W) void k_tblock_batch(const GridDesc<S>* __restrict__ grids,
                                                         const WorkItem* __restrict__ items, int nitems, int in0,
                                                         int in1, int out0, int out1) {
    constexpr int IX = 64 - 2 * T;
    constexpr int IY = W * R - 2 * T;
    __shared__ TBShared<S, T, W> sh;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const WorkItem wi = items[it];
        const GridDesc<S>& g = grids[wi.grid];
        const Layout L = g.L;
        const StepCoef c = g.c;
        const int xlo = wi.tx * IX - T, ylo = wi.ty * IY - T;
        const bool inner = xlo >= 0 && xlo + 64 <= L.nx && ylo >= 0 && ylo + W * R <= L.ny;
        if (inner) {
            TBTile<S, T, R, W, PF, SB, UPF, false> t(g.buf[in0], g.buf[in1], g.rho, g.buf[out0], g.buf[out1], L, c, sh, wi.tx,
                                        wi.ty, wi.k0, wi.k1);
            t.run();
        } else {
            TBTile<S, T, R, W, PF, SB, UPF, true> t(g.buf[in0], g.buf[in1], g.rho, g.buf[out0], g.buf[out1], L, c, sh, wi.tx,
                                       wi.ty, wi.k0, wi.k1);
            t.run();
        }
        __syncthreads();  // the next item reuses the LDS slots
    }
}

// The same fused substeps with one workgroup per work item: items are in grid
// order (z chunks, then tile rows, then tiles, as a single-grid launch walks
// them) and each XCD takes a contiguous range, so the items resident on an
// XCD at one time are neighbours of one grid at the same heights and share
// their halo lines in its L2; the hardware hands items to CUs as they free up.
template <typename S, int T, int R, int W, int PF, bool SB, bool UPF>
__global__ __launch_bounds__(64 * W) void k_tblock_batch_items(const GridDesc<S>* __restrict__ grids,
                                                               const WorkItem* __restrict__ items, int in0,
                                                               int in1, int out0, int out1) {
    constexpr int IX = 64 - 2 * T;
    constexpr int IY = W * R - 2 * T;
    __shared__ TBShared<S, T, W> sh;
    const WorkItem wi = items[xcd_remap(blockIdx.x, gridDim.x)];
    const GridDesc<S>& g = grids[wi.grid];
    const Layout L = g.L;
    const StepCoef c = g.c;
    const int xlo = wi.tx * IX - T, ylo = wi.ty * IY - T;
    const bool inner = xlo >= 0 && xlo + 64 <= L.nx && ylo >= 0 && ylo + W * R <= L.ny;
    if (inner) {
        TBTile<S, T, R, W, PF, SB, UPF, false> t(g.buf[in0], g.buf[in1], g.rho, g.buf[out0], g.buf[out1], L, c, sh,
                                                 wi.tx, wi.ty, wi.k0, wi.k1);
        t.run();
    } else {
        TBTile<S, T, R, W, PF, SB, UPF, true> t(g.buf[in0], g.buf[in1], g.rho, g.buf[out0], g.buf[out1], L, c, sh,
                                                wi.tx, wi.ty, wi.k0, wi.k1);
        t.run();
    }
}

// one streaming substep on every grid: buf[cur] is phi^n, buf[old] receives phi^{n+1}
template <typename S, int BY>
__global__ __launch_bounds__(64 * BY) void k_stream_batch(const GridDesc<S>* __restrict__ grids,
                                                          const WorkItem* __restrict__ items, int nitems, int cur,
                                                          int old) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const WorkItem wi = items[it];
        const GridDesc<S>& g = grids[wi.grid];
        const Layout L = g.L;
        const StepCoef c = g.c;
        stream_v_tile<S, BY>(g.buf[cur], g.buf[old], g.rho, L, c, wi.tx, wi.ty, wi.k0, wi.k1, 0.0);
    }
}

}  // namespace hgs
