// persistent.hpp -- one persistent launch that runs many chains (a batch of
// images with their own sizes and chain lengths) to completion.
//
// Work is cut into items (image, tile, block): block b of a tile advances its
// core from step b*k to step min((b+1)*k, n) with the same register-resident
// body as the per-launch kernel (chain_block.hpp).  Items sit in one global
// list ordered by block index, so the list is a valid topological order of
// the dependencies below.  Workgroups draw tickets from one counter; a
// ticket is a run of `chunk` consecutive list items (neighbouring tiles of
// one image), which the workgroup runs in list order.  Before loading an
// item it waits until the item's 3x3 neighbourhood of tiles has finished
// block b-1 (a per-tile counter, released after the tile's stores).  This is the GPU counterpart of the
// paper's per-filter row counters with acquire/release semantics (Section
// 3.5): here the counters are per tile and per block of k steps instead of
// per row and per step.
//
// Progress, with any number of resident workgroups: a workgroup draws a new
// ticket only after it has finished the items of its previous one, runs a
// ticket's items in list order, and an item waits only for items earlier
// in the list, all of which were drawn by workgroups that are running.  The
// earliest unfinished item is therefore always the one a running workgroup
// is working on, and nothing it waits for is unfinished.  Every wait is still bounded, by elapsed
// time (the constant 100 MHz clock): past the bound the item sets the error
// word and no later wait of the launch blocks, so the launch always drains.
//
// Buffers: block b reads state from marker (b = 0) or ws[(b-1)&1] and writes
// ws[b&1], except the last block which writes out.  A tile's block b may
// overwrite ws[b&1] only after its neighbours finished block b-1, which was
// the last reader of that buffer, so the same counters also order the
// write-after-read reuse of the two work buffers.  With two or more blocks
// the marker may be out itself (in place, or a run-to-stability image that
// continues from its previous result): the last block writes a tile's core
// only after its neighbours, the only other readers of it, passed block 0.
//
// DETECT (plans with run-to-stability images): each block ORs the per-step
// change bits of its core into the image's word for that block, so the host
// can tell after the launch whether, and at which step, the image stopped
// changing.  Images whose `active` flag is 0 are skipped whole.
#pragma once

#include "chain_block.hpp"

namespace geochain {

struct PlanImage {
    const void *marker;
    const void *mask;
    void *out;
    void *ws0;
    void *ws1;
    int64_t pitch;
    int32_t width, height;
    int32_t n_steps;
    int32_t k;          // steps per block (the last block may be shorter)
    int32_t core_x, core_y;
    int32_t tiles_x, tiles_y;
    int32_t blocks;
    int32_t flag_base;  // first per-tile counter of this image
    int32_t src0_ws1;   // block 0 reads ws1 (in-place single-block chains)
    int32_t active;     // 0: the image's items are skipped in this launch
    uint32_t *change;   // run-to-stability images: per block, the OR over
                        // tiles of the block's per-step change bits (else null)
};

struct PlanItem {
    int32_t image;
    int32_t tile;
    int32_t block;
    int32_t pad;
};

struct PersistentArgs {
    const PlanImage *images;
    const PlanItem *items;
    int32_t n_items;
    uint32_t *ticket;    // next item to draw (zero at launch)
    uint32_t *flags;     // per tile: number of blocks finished
    uint32_t *error;     // bit 0: a wait hit its time bound
    uint64_t wait_ticks; // bound of one wait, in ticks of the 100 MHz clock
    int32_t chunk;       // consecutive items per ticket
};

// Waits until every tile of the 3x3 neighbourhood of (tx, ty) has finished
// at least `need` blocks.  Called by one whole wave; lane j < 9 watches
// neighbour j.  Returns false if the wait outlasted a.wait_ticks.
__device__ __forceinline__ bool wait_neighbours(const PersistentArgs &a, const PlanImage &im, int tx, int ty,
                                                uint32_t need) {
    const int lane = threadIdx.x & 63;
    const int dy = lane / 3 - 1, dx = lane % 3 - 1;
    const int nx = tx + dx, ny = ty + dy;
    const bool mine = lane < 9 && nx >= 0 && nx < im.tiles_x && ny >= 0 && ny < im.tiles_y;
    const uint32_t *flag = a.flags + im.flag_base + (mine ? ny * im.tiles_x + nx : 0);
    if (a.wait_ticks == 0) return false;   // a bound of 0: every wait fails at once (tests of the error path)
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
        bool ok = true;
        if (mine) ok = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need;
        if (__builtin_amdgcn_ballot_w64(!ok) == 0) return true;
        if (__builtin_amdgcn_s_memrealtime() - t0 > a.wait_ticks) return false;
        __builtin_amdgcn_s_sleep(2);
    }
}

template <typename T, int OP, int MODE, int CW, int RPW, int NW, int G = 1, bool DETECT = false>
__global__ __launch_bounds__(64 * NW) void persistent_chain_kernel(PersistentArgs a) {
    using R = typename RegOf<T>::type;
    __shared__ __attribute__((aligned(16))) R xch[2][NW][2 * G][lanes_per_group<G>() * CW];
    // (no LDS staging here: the second workgroup per CU hides the loads)
    __shared__ __attribute__((aligned(16))) uint8_t stage[stage_bytes<T, CW, RPW, NW, G, false>()];

    const int tid = threadIdx.x;
    __shared__ int32_t drawn;
    // change bits of the current item, ORed by its waves (one device-scope
    // atomic per item instead of one per wave, as in chain_block_kernel)
    __shared__ uint32_t wg_bits;
    if (DETECT && tid == 0) wg_bits = 0;
    for (;;) {
        // ---- draw the next chunk of items (list order) ----
        // The first wave as a whole takes this branch (a uniform condition);
        // lane 0 draws and readfirstlane hands the ticket to the wave, so no
        // lane-divergent region contains a barrier or the loop's exit.
        if (tid < 64) {
            uint32_t t = 0;
            if (tid == 0) t = atomicAdd(a.ticket, 1u);
            t = __builtin_amdgcn_readfirstlane(t);
            if (tid == 0) drawn = (int32_t)min((uint64_t)t * (uint32_t)a.chunk, (uint64_t)a.n_items);
        }
        __syncthreads();
        const int first_it = drawn;
        if (first_it >= a.n_items) break;
        const int end_it = (int)min((int64_t)first_it + a.chunk, (int64_t)a.n_items);
        for (int it = first_it; it < end_it; ++it) {
            const PlanItem item = a.items[it];
            const PlanImage &im = a.images[item.image];
            // the same item for every wave: a uniform skip, barriers stay matched;
            // only items of the same image depend on a skipped item
            if (!im.active) {
                __syncthreads();  // every wave has read `drawn` before the next draw
                continue;
            }
            const int tx = item.tile % im.tiles_x;
            const int ty = item.tile / im.tiles_x;
            const int b = item.block;

            // ---- wait for the 3x3 neighbourhood to finish block b-1 ----
            // Once any wait has failed the results are void anyway: stop waiting
            // so the launch drains quickly.
            if (b > 0 && tid < 64 &&
                __hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                const bool ok = wait_neighbours(a, im, tx, ty, (uint32_t)b);
                if (!ok && tid == 0) atomicOr(a.error, 1u);
            }
            // Make the neighbours' stores visible to this workgroup's loads: the
            // waiting wave acquires at agent scope (this invalidates the CU's L1
            // and the stale lines of the XCD's L2, shared by every wave of the
            // workgroup) and the barrier orders the other waves after it.  One
            // acquire per workgroup instead of one per wave: each is an L2
            // invalidate.
            if (tid < 64) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __syncthreads();

            // ---- the block itself ----
            const int k_b = (b == im.blocks - 1) ? im.n_steps - b * im.k : im.k;
            BlockArgs ba{};
            ba.src = b == 0 ? (im.src0_ws1 ? (const void *)im.ws1 : im.marker)
                            : (const void *)((b - 1) & 1 ? im.ws1 : im.ws0);
            ba.mask = im.mask;
            ba.dst = b == im.blocks - 1 ? im.out : (b & 1 ? im.ws1 : im.ws0);
            ba.width = im.width;
            ba.height = im.height;
            ba.pitch = im.pitch;
            ba.k = k_b;
            ba.halo = im.k;
            ba.core_x = im.core_x;
            ba.core_y = im.core_y;
            ba.tiles_x = im.tiles_x;
            const int rx0 = tx * im.core_x - im.k;
            const int ry0 = ty * im.core_y - im.k;
            // The core goes out with agent-scope stores: they reach the level
            // that every XCD sees by themselves, so the agent-scope release below
            // has (almost) no dirty L2 lines to write back.  The release is still
            // what orders them before the counter.
            const uint32_t bits = chain_block_dispatch<T, OP, MODE, DETECT, CW, RPW, NW, G, true>(ba, rx0, ry0, xch, stage);
            if constexpr (DETECT) {
                if (bits != 0 && (tid & 63) == 0) atomicOr(&wg_bits, bits);
            }

            // ---- publish: stores first, then the tile's counter ----
            // (the barrier also keeps `drawn` until every wave has read it)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __syncthreads();
            if (tid < 64) {
                if (tid == 0) {
                    if constexpr (DETECT) {
                        // read after the barrier; cleared before wave 0 reaches
                        // the next item's barriers, which order it before that
                        // item's ORs
                        if (wg_bits != 0 && im.change != nullptr) atomicOr(im.change + b, wg_bits);
                        wg_bits = 0;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    __hip_atomic_store(a.flags + im.flag_base + item.tile, (uint32_t)(b + 1), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
}

}  // namespace geochain
