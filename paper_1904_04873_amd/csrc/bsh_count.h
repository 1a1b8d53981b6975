// Shared declarations of the stage-1 count kernels (bsh_count_tile.h, bsh_count_kernels.h,
// bsh_count.hip, bsh_count_batch.hip, bsh_count_table.hip) and the batched plan (bsh_batch.hip).
// Internal to libbsh.
#pragma once

#include "bsh_internal.h"

namespace bsh {

constexpr int kMaxLanes = 512;       // largest tile (binary templates per block)
constexpr int kDefaultLanes = 256;
constexpr int kDefaultChunk = 256;   // segments staged per LDS pass
constexpr int kFlush = 64;           // segments per FP32 partial sum
constexpr int kRowPad = 4;           // zero words staged after each row (a failed track reads them)
constexpr int kNF = BSH_MAX_F0;
constexpr int kEccMode = 3;          // kernel modes kEccMode.. are the ELL1 forms of modes 0..
// Kernel mode + kProvenMode: the same table variant for a launch whose every track the host has
// proven to stay inside the staged rows and to drift less than half a bin across the band
// (proven_window): the per-track range and model checks are left out.
constexpr int kProvenMode = 8;
constexpr int mode_base(int mode) { return mode % kProvenMode; }
constexpr bool mode_ecc(int mode) { return mode_base(mode) >= kEccMode; }
constexpr bool mode_table(int mode) { return mode_base(mode) % kEccMode == 2; }
constexpr bool mode_proven(int mode) { return mode >= kProvenMode; }

// Everything a tile needs about its work item (one segment set, one band grid, a run of
// sky pixels of that grid, and the item's output map).
struct ItemDesc {
    const double* t_mid;
    const double* v;
    const float* w;
    const uint32_t* bits;
    const double* sky;
    const double* a_p;
    const double* period;
    const int64_t* tasc_off;
    const double* t_asc;
    uint32_t* count_out;
    float* wsum_out;
    int32_t* status;
    int64_t n_seg;
    int64_t n_bin;
    int64_t k_lo;
    int64_t k0;
    int32_t w_per_sky;
    int32_t n_words;
    int32_t n_bins;
    int32_t n_f0;
    int32_t n_ap;
    int32_t n_per;
    int32_t sky_lo;     // first pixel of the item in the grid's sky table
    int32_t n_sky;      // pixels of the item
    double ec, es;      // (e cos w, e sin w) of the grid's ELL1 track; zeros for a circular grid
    // The bounds a proven launch relies on (0 when the window is not proven): |v/c| of every
    // segment and a_p W (1 + e) of every template, checked on the device as they are staged.
    double v_claim, apw_claim;
};

struct PlainLaunch {
    ItemDesc d;
    int32_t tiles_per_sky;
    int32_t tile_start[BSH_MAX_PER + 1];   // first tile of each period group
};

// One queue entry of the persistent kernel.
struct WorkUnit {
    int32_t item;
    int32_t sky;        // pixel inside the item
    int32_t ip;         // period index
    int32_t tile;       // tile inside the period group
};

// Table variant: 256-entry subset-sum tables of groups of eight segments (1 KB each), each entry
// the sum of the 16-entry subset sums of the group's two halves.
constexpr int kGroup = 4;
constexpr int kGroup8 = 2 * kGroup;
// Eight-segment groups per register partial sum of the table variant: each fold into the map is a
// read-modify-write of the lane's slots, and 128 groups (1024 segments) keep the FP32 error bound
// (kFlushGroups + 4 + n_seg / (8 kFlushGroups)) ulps below 1e-5 relative for up to ~35000 segments.
constexpr int kFlushGroups = 128;

// Per staged segment: D cos(W t), D sin(W t) and the Doppler factor D of the tile's pixel, and
// for the ELL1 track D cos(2 W t), D sin(2 W t) (zero-length arrays on a circular grid, which
// leave the layout as it is); for the table variant the subset-sum tables.  The bit-packed rows
// precede the structure in LDS, sized at launch for the widest row of the launch (row_bytes), so
// that a block of the table variant at 256-segment chunks fits three times into a CU's 160 KB.
template <int kChunk, bool kEcc>
struct TileSmemLut {
    float T8[(kChunk / kGroup8) * 256];
    double DC[kChunk];
    double DS[kChunk];
    double D[kChunk];
    double DC2[kEcc ? kChunk : 0];
    double DS2[kEcc ? kChunk : 0];
};

template <int kChunk, bool kEcc>
struct TileSmem {
    double DC[kChunk];
    double DS[kChunk];
    double D[kChunk];
    double DC2[kEcc ? kChunk : 0];
    double DS2[kEcc ? kChunk : 0];
    float W[kChunk];
};

// LDS bytes of the staged rows of one chunk: kRowPad zero words after each row's n_words.
inline size_t row_bytes(int chunk, int n_words) { return (size_t)chunk * (size_t)(n_words + kRowPad) * 4u; }

// Binary templates per tile: the table variant gives each template a pair of lanes.
inline int tile_templates(int mode, int lanes) { return mode_table(mode) ? lanes / 2 : lanes; }

int64_t plan_tiles(const bsh_grid* g, int lanes, int32_t* tile_start, int64_t* group_sizes);
void fill_desc(ItemDesc& d, const bsh_segments* seg, const bsh_grid* grid, int32_t sky_lo,
               int32_t n_sky, uint32_t* count_out, float* wsum_out, int32_t* status);
int zero_words(void* p, int64_t n_words, hipStream_t stream);
int floats_to_counts(uint32_t* p, int64_t n, hipStream_t stream);
// mode: 0 select-and-add (weighted sums), 1 select-and-add with counts, 2 subset-sum tables;
// plus kEccMode for the same on the ELL1 track
// n_words: the widest staged row of the launch (sizes the rows' LDS region).
int launch_plain(const PlainLaunch& p, int64_t blocks, int lanes, int chunk, int mode, int n_words,
                 hipStream_t stream);
// persistent: blocks pull units from *counter (zeroed beforehand); else one block per unit.
int launch_batch(const ItemDesc* items, const WorkUnit* units, int64_t n_units, uint32_t* counter,
                 int blocks, int lanes, int chunk, int mode, int n_words, bool persistent, hipStream_t stream);
// Resident blocks per CU of the persistent form (or, persistent false, of one block per unit).
int batch_blocks_per_cu(int lanes, int chunk, int mode, int n_words, bool persistent = true);
// The table variant's launchers (bsh_count_table.hip); lds: the block's LDS bytes.
int launch_plain_table(const PlainLaunch& p, int64_t blocks, int lanes, int chunk, int mode, size_t lds,
                       hipStream_t stream);
int launch_batch_table(const ItemDesc* items, const WorkUnit* units, int64_t n_units, uint32_t* counter, int blocks,
                       int lanes, int chunk, int mode, size_t lds, bool persistent, hipStream_t stream);
int occupancy_table(int lanes, int chunk, int mode, size_t lds, bool persistent);
int allow_lds(const void* kernel, size_t bytes);
int kernel_mode(int variant, bool with_count);
// kEccMode for a grid with an eccentricity pair, else 0 (added to kernel_mode's value)
int ecc_mode(const bsh_grid* g);
// For a table mode: when proven_window holds for the item, stores the proof's bounds in its
// descriptor and returns true (the launch may then take mode + kProvenMode).
bool prove_item(int mode, ItemDesc& d, const bsh_segments* seg, const bsh_grid* grid);
bool valid_tile_shape(int lanes, int chunk);

}  // namespace bsh
