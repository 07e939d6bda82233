// lpa_copra.h -- COPRA (arXiv 2301.09125, Section 3.3): the arguments of one
// half-round and the launchers of lpa_copra.hip.
#pragma once

#include "lpa_internal.h"

namespace lpa {

// One COPRA half-round (lpa_copra.hip) on the caller's CSR.  The state of
// vertex v is one record of `stride` u32 words at v * stride: word 0 the
// count of kept labels, word 1 the best label, then (label, coefficient)
// pairs, so that a neighbour's whole state is one gather of one line.
// `in` is the state of the round before, `out` the state written.  half 0 =
// every vertex votes; 1 / 2 = only the vertices whose draw names that half,
// the others copy their record.
struct CopraArgs {
    Graph g;
    uint32_t V;       // max_labels, 1..64
    uint32_t stride;  // u32 words per record (2 + 2 V rounded up)
    const uint32_t *in;
    uint32_t *out;
    uint32_t t, half, tie;
    unsigned long long seed;
    unsigned long long *changed;  // kCountWords counter words: best labels changed
    uint32_t *ovf_rows;           // rows left to the device-memory table ...
    uint32_t *ovf_count;          // ... and their number
    uint32_t *err;                // ERR_TABLE if a table had no free slot
    uint32_t first;               // every vertex is still alone (round 1, first half)
    const uint8_t *distinct;      // per row: its neighbours are listed once
};

// Words per state record: 2 + 2 V rounded up to a power of two up to 32
// words (one 128-byte line holds the record), to a multiple of 32 beyond.
inline uint32_t copra_stride(uint32_t V) {
    const uint32_t w = 2 + 2 * V;
    if (w > 32) return (w + 31) / 32 * 32;
    uint32_t p = 1;
    while (p < w) p <<= 1;
    return p;
}

// A piece of a COPRA row voted through a device-memory table: arcs
// [b0, b1) of row rows[i].
struct CopraPiece {
    uint32_t i;
    uint32_t pad;
    uint64_t b0, b1;
};

// ---- launchers: lpa_copra.hip --------------------------------------------
// Check a caller's CSR (row_ptr, col < n, weighted degrees < 2^32) into
// err; distinct (u8[n] or NULL) receives whether each row's neighbours are
// strictly increasing; wsum: u64[n] scratch for the rows longer than
// kHeadArcs arcs.
hipError_t launch_csr_check(const Graph &g, uint32_t *err, uint8_t *distinct, unsigned long long *wsum,
                            hipStream_t s);
// Every vertex alone with belonging 1, in the records of `rec`.
hipError_t launch_copra_init(uint32_t n, uint32_t stride, uint32_t *rec, hipStream_t s);
// Records to the caller's arrays: best labels, and (when not NULL) the kept
// labels and coefficients (V slots per vertex) and their counts.
hipError_t launch_copra_output(const uint32_t *rec, uint32_t n, uint32_t V, uint32_t stride, uint32_t *best,
                               uint32_t *labs, uint32_t *coefs, uint32_t *cnt, hipStream_t s);
// Rows with arcs by class of deg * V into rows[0] (<= 32), rows[1] (<= 128),
// rows[2] (<= 512) and rows[3] (larger), count[0..4) (zeroed by the caller).
constexpr int kCopraClasses = 4;
hipError_t launch_copra_list(const Graph &g, uint32_t V, uint32_t *const *rows, uint32_t *count, hipStream_t s);
// Table sizes (next_pow2(2 * min(deg * V, n))) and piece counts (pieces of
// at most `per` arcs) of the listed rows.
hipError_t launch_copra_sizes(const Graph &g, uint32_t V, const uint32_t *rows, uint32_t count, uint32_t per,
                              unsigned long long *size, unsigned long long *npieces, hipStream_t s);
// One half-round over the kCopraClasses row lists (count: host copy of their sizes).
hipError_t launch_copra_round(const CopraArgs &a, const uint32_t *const *rows, const uint32_t *count,
                              hipStream_t s);
// Device-table slots one decision block scans.
constexpr uint32_t kCopraSliceSlots = 16384;
// The listed rows through device-memory tables (off: table offsets, count + 1
// entries; first: first piece of each row, pieces of at most `per` arcs;
// sfirst: first slice of each row's table, slices of kCopraSliceSlots;
// rowstate: (5 + 2 V) * count u64 words.  Tables, totals and rowstate
// zeroed (table keys empty) by the caller).
hipError_t launch_copra_global(const CopraArgs &a, const uint32_t *rows, uint32_t count,
                               const unsigned long long *first, uint32_t per, CopraPiece *pieces, uint64_t npieces,
                               const unsigned long long *off, uint32_t *slab_key, unsigned long long *slab_tal,
                               unsigned long long *total, const unsigned long long *sfirst, CopraPiece *slices,
                               uint64_t nslices, unsigned long long *rowstate, hipStream_t s);
}  // namespace lpa
