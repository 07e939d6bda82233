// lpa_internal.h -- private declarations shared by the runtime (lpa_runtime.hip)
// and the kernels (lpa_kernels.hip) of the label-propagation library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpa {

// Error bits raised by kernels into a device word.
enum : uint32_t {
    ERR_COL = 1u,     // a col value >= n
    ERR_WOVF = 2u,    // weighted degree + self weight >= 2^32
    ERR_ROWPTR = 4u,  // row_ptr not monotone / not ending at m
    ERR_LABEL = 8u,   // a label value >= n
};

// Degree bins (see lpa_options in lpa.h).
enum { BIN_ZERO = 0, BIN_THREAD = 1, BIN_GROUP = 2, BIN_WAVE = 3, BIN_HUB = 4, NBINS = 5 };

constexpr int kThreadMaxCap = 8;    // register-array size of the one-lane vote
constexpr int kGroupLanes = 16;
constexpr int kGroupSlots = 64;     // LDS slots per 16-lane group (degree <= 32)
constexpr int kWaveSlots = 512;     // LDS slots per wavefront (degree <= 256)
constexpr int kBlockThreads = 256;
constexpr int kChunkSlotsMax = 4096;  // LDS slots per hub block (chunk <= 2048)
constexpr uint32_t kNoHub = 0xFFFFFFFFu;

struct Graph {
    const uint64_t *rp;
    const uint32_t *col;
    const uint32_t *w;  // nullptr = unit weights
    uint32_t n;
    uint64_t m;
};

// Arguments common to every vote kernel of one round.
struct RoundArgs {
    Graph g;
    const uint32_t *L_old;
    uint32_t *L_new;
    uint32_t sw;                  // self weight
    uint32_t check;               // nonzero: verify weighted degrees fit 32 bits
    unsigned long long *changed;  // this round's changed counter
    uint32_t *err;                // error bits
};

// One block work item for high-degree rows: arcs [b0, b1) of vertex v.
// hub == kNoHub: the row fits one chunk and the block finishes the vote;
// otherwise hub indexes the multi-chunk state below.
struct HubItem {
    uint32_t v;
    uint32_t hub;
    uint64_t b0;
    uint64_t b1;
};

// State of the rows longer than one chunk (arrays of `count` entries).
struct HubState {
    const uint32_t *vertex;       // vertex id
    const uint64_t *slab_off;     // offset of the row's slab (u64 slots)
    const uint32_t *slab_mask;    // slab size - 1 (power of two >= 2 * degree)
    const uint64_t *touched_off;  // offset of the row's touched-slot list (capacity = degree)
    unsigned long long *slab;     // global hashtable slots, EMPTY between rounds
    uint32_t *touched;            // slot indices claimed this round
    uint32_t *tcount;             // claimed slots this round (reset by hub_final)
    unsigned long long *best;     // max (weight << 32 | ~label) (reset by hub_final)
    unsigned long long *own_sum;  // weight of neighbours holding the row's own label
    uint32_t *own_seen;           // some neighbour holds the row's own label
    unsigned long long *rowsum;   // weighted degree (checked in round 1)
};

// Phase-2 item: touched-list positions [t0, t1) of multi-chunk hub `hub`.
struct ReduceItem {
    uint32_t hub;
    uint32_t t0;
    uint32_t t1;
    uint32_t pad;
};

struct ModArgs {
    Graph g;
    const uint32_t *labels;
    unsigned long long *K;         // n, summed weighted degree per community
    unsigned long long *sums;      // [0] = 2m, [1] = Sigma_in
    uint32_t *err;
};

// ---- launchers (defined in lpa_kernels.hip) ------------------------------
hipError_t launch_fill_u32_iota(uint32_t *a, uint32_t *b, uint32_t n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, uint64_t count, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint64_t count, hipStream_t s);
hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, uint64_t count, hipStream_t s);
hipError_t launch_check_labels(const uint32_t *labels, uint32_t n, uint32_t *err, hipStream_t s);

hipError_t launch_bin_count(const Graph &g, uint32_t tmax, uint32_t gmax, uint32_t wmax, uint32_t *blk_counts,
                            unsigned long long *blk_arcs, uint32_t nblk, uint32_t *err, hipStream_t s);
hipError_t launch_bin_scan(uint32_t *blk_counts, const unsigned long long *blk_arcs, uint32_t nblk,
                           uint32_t *totals, unsigned long long *arc_totals, hipStream_t s);
hipError_t launch_bin_scatter(const Graph &g, uint32_t tmax, uint32_t gmax, uint32_t wmax,
                              const uint32_t *blk_offsets, uint32_t nblk, uint32_t *order, hipStream_t s);
hipError_t launch_gather_rows(const uint64_t *rp, const uint32_t *verts, uint32_t count, uint64_t *out3,
                              hipStream_t s);

hipError_t launch_vote_thread(const RoundArgs &a, const uint32_t *list, uint32_t cnt, int grid_cap,
                              hipStream_t s);
hipError_t launch_vote_group(const RoundArgs &a, const uint32_t *list, uint32_t cnt, int grid_cap,
                             hipStream_t s);
hipError_t launch_vote_wave(const RoundArgs &a, const uint32_t *list, uint32_t cnt, int grid_cap,
                            hipStream_t s);
hipError_t launch_vote_hub(const RoundArgs &a, const HubItem *items, uint32_t count, uint32_t chunk,
                           const HubState &hs, hipStream_t s);
hipError_t launch_hub_reduce(const HubState &hs, const ReduceItem *items, uint32_t count, hipStream_t s);
hipError_t launch_hub_final(const RoundArgs &a, const HubState &hs, uint32_t count, hipStream_t s);

hipError_t launch_mod_small(const ModArgs &a, const uint32_t *list, uint32_t cnt, hipStream_t s);
hipError_t launch_mod_wave(const ModArgs &a, const uint32_t *list, uint32_t cnt, hipStream_t s);
hipError_t launch_mod_hub(const ModArgs &a, const HubItem *items, uint32_t count, hipStream_t s);
hipError_t launch_mod_sumsq(const unsigned long long *K, uint32_t n, unsigned long long *partials,
                            uint32_t nparts, hipStream_t s);

}  // namespace lpa
