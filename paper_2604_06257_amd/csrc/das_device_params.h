// Kernel parameter block (plain data shared by host and device code).
#pragma once

#include <stdint.h>

struct das_kparams {
    int32_t T, E, S, F;
    int64_t n_slots;     // tiles * slots per tile
    int32_t n_tiles;
    int32_t use_apod;    // f# > 0
    double fs_c;         // fs / c: samples per metre of receive path
    double fd_c;         // fd / c: carrier cycles per metre of receive path
    double fs;
    double fd;
    double t0fs;         // t0 * fs
    float two_fnum;      // 2 f#
    float alpha;         // Tukey taper fraction
    float inv_2alpha;    // 1 / (2 alpha), 0 when alpha = 0
    float edge_2alpha;   // (1 - alpha) / (2 alpha), 0 when alpha = 0
    int32_t planar;      // every element lies in the plane z = z0
    double z0;           // that plane's depth (when planar)
    int32_t vec_ok;      // frame rows are 16-byte aligned (F multiple of the vector width)
};
