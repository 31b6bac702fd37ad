// Internal interfaces between the C ABI (das_api.cpp) and the kernels
// (das_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <hip/hip_vector_types.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "das_device_params.h"

namespace das {

constexpr int kWaves = 4;               // waves per workgroup tile
constexpr int kLanes = 64;              // gfx950 wavefront
constexpr int kSlots = kWaves * kLanes; // voxel slots per tile

// Host-side voxel tiling: slot -> voxel index (-1 = empty slot).
struct Tiling {
    int32_t tile_dims[3] = {0, 0, 0};   // lattice points per tile (0: not a lattice)
    int32_t wave_dims[3] = {0, 0, 0};   // lattice points per wave
    int64_t n_tiles = 0;
    std::vector<int32_t> slot_to_vox;   // n_tiles * kSlots
    std::vector<int32_t> tile_xyz;      // n_tiles * 3 tile coordinates (lattice), else (index, 0, 0)
};

// Returns 0 or a negative das_status; err receives a message.
int tile_points(const float* xyz, int64_t n, const char* override_spec, Tiling& out, std::string& err);

struct PlanDev {
    das_kparams kp;
    float* vx = nullptr;       // [n_slots]
    float* vy = nullptr;
    float* vz = nullptr;
    float* tx = nullptr;       // [T][n_slots]
    int32_t* slot_vox = nullptr;  // [n_slots]
    double* elemd = nullptr;   // [E][3] element coordinates (float32 inputs held in FP64)
    const void* zrow = nullptr; // 64 zero bytes (inside the elemd allocation): read for samples outside a record
    int32_t* windows = nullptr; // [n_tiles][T][E][2]: (first row, rows); plan-time only
    int4* items = nullptr;      // per tile, the (t, e, first row, rows) work items, e-major, in stages:
                                // two int4 per stage for variants that pair (the second may be empty:
                                // rows = 0), one otherwise
    int32_t* item_off = nullptr;  // [n_tiles + 1] offsets into items, in stages
    int32_t* wg_unit = nullptr;   // [n_tiles * chunks] workgroup -> tile * chunks + frame chunk
    int32_t fc = 0, pitch = 0, groups = 1;  // kernel variant: frames per workgroup, LDS row pitch, element groups
    int64_t n_vox = 0;                      // voxels (per-transmit output stride: n_vox * F)
};

// Workgroup -> (tile, frame chunk) order: each of the 8 XCDs gets a lateral
// region of tile columns (all depths), heaviest units first inside a region,
// regions interleaved so that workgroup w runs on XCD w % 8.
std::vector<int32_t> order_units(const Tiling& tl, const std::vector<int32_t>& item_off, int chunks, bool xcd_runs);

// Kernel variant for F frames, the largest tile window (rows), the tile count and the average number of
// (transmit, element) items per tile.
struct Variant {
    int fc, pitch, groups;
};
Variant choose_variant(int frames, int max_window, int64_t n_tiles, double items_per_tile);

// The compiled variants as (fc, pitch, groups) triples: writes min(count, capacity) of them to out (when not
// null) and returns the count.
int list_variants(int32_t* out, int capacity);

// Whether a variant stages two items per step (the plan packs stages only for such variants): with 16 or
// more frames per workgroup the saved fill and barrier outweigh the extra registers.  At 8 frames the unpaired
// variant at 6 waves per SIMD beats the paired one at 4 (c3: 5.13 against 6.78 ms).
constexpr bool stage_pairs(int fc) { return fc >= 16; }

// Window rows each fill thread stages for a variant (the largest over the IQ types: complex64, which packs
// the fewest frames into a 16-byte load); the second window of a stage starts at a multiple of it.
constexpr int fill_rows_per_thread(int fc, int pitch) {
    const int fpt = fc < 2 ? fc : 2;
    return ((pitch - 1) * (fc / fpt) + kSlots - 1) / kSlots;
}

// Computes per (tile, transmit, element) sample windows and counts.
// counts[0] = active (slot, e, t) triples (w > 0, inside the record);
// counts[1] = processed triples (valid slots of tiles whose window is not
// empty); counts[2] = largest window.
hipError_t launch_windows(const PlanDev& p, unsigned long long* counts_dev, hipStream_t s);

// Raises the dynamic LDS limit of the plan's kernel variant (all IQ types).
hipError_t prepare_variant(const PlanDev& p);

hipError_t launch_das(const PlanDev& p, const void* iq, int dtype, void* out, hipStream_t s);
// Per-transmit output [T][V][F] (variants with at most 2 frames per workgroup, T <= 4).
bool per_tx_supported(const PlanDev& p);
hipError_t launch_das_per_tx(const PlanDev& p, const void* iq, int dtype, void* out, hipStream_t s);

hipError_t launch_tx_plane_wave(float* tx_out, const float* vox_xyz, int64_t n_vox, const double* normals_host,
                                int32_t n_tx, double inv_c, hipStream_t s);

}  // namespace das
