// C ABI of the delay-and-sum beamformer: argument checks, plan lifecycle,
// voxel tiling (host) and kernel dispatch.  See include/das.h for the
// contract of every entry point.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <utility>
#include <numeric>
#include <string>
#include <unordered_set>
#include <vector>

#include "das.h"
#include "das_internal.h"

namespace {

thread_local std::string g_err;

int fail(int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return status;
}

int fail_hip(hipError_t e, const char* what) {
    return fail(DAS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

constexpr uint64_t kMagic = 0x6461735f706c616eull;  // "das_plan"

std::mutex g_mu;
std::unordered_set<const void*> g_live;  // plans created and not yet destroyed

}  // namespace

struct das_plan {
    uint64_t magic = kMagic;
    das_params p{};
    das::PlanDev dev;
    das::Tiling tiling;  // slot_to_vox kept on host for queries
    int64_t active_triples = 0;
    int64_t processed_triples = 0;
    int32_t max_window = 0;
};

// ---------------------------------------------------------------- tiling
namespace das {

static bool parse_spec(const char* spec, int32_t tile[3], int32_t wave[3]) {
    int v[6];
    if (!spec || std::sscanf(spec, "%d,%d,%d,%d,%d,%d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) != 6) return false;
    for (int i = 0; i < 3; ++i) {
        if (v[i] <= 0 || v[i + 3] <= 0 || v[i] % v[i + 3] != 0) return false;
        tile[i] = v[i];
        wave[i] = v[i + 3];
    }
    return tile[0] * tile[1] * tile[2] == kSlots && wave[0] * wave[1] * wave[2] == kLanes;
}

// Default tile shapes.  Depth (z) is the fast axis of the sample index (about
// two samples of round trip per voxel step), lateral axes the slow ones, so
// waves are 16 lateral x 4 deep in 2D and 8 x 8 lateral x 1 deep in 3D.
static void default_dims(const int64_t n_ax[3], int32_t tile[3], int32_t wave[3]) {
    const bool big[3] = {n_ax[0] > 1, n_ax[1] > 1, n_ax[2] > 1};
    const int nbig = big[0] + big[1] + big[2];
    for (int i = 0; i < 3; ++i) tile[i] = wave[i] = 1;
    if (nbig == 3) {
        tile[0] = 8; tile[1] = 8; tile[2] = 4;
        wave[0] = 8; wave[1] = 8; wave[2] = 1;
    } else if (nbig == 2) {
        if (big[2]) {
            const int lat = big[0] ? 0 : 1;
            tile[lat] = 32; tile[2] = 8;
            wave[lat] = 16; wave[2] = 4;
        } else {
            tile[0] = 32; tile[1] = 8;
            wave[0] = 16; wave[1] = 4;
        }
    } else {
        const int ax = big[0] ? 0 : (big[1] ? 1 : 2);
        tile[ax] = kSlots;
        wave[ax] = kLanes;
    }
}

static uint64_t spread21(uint64_t x) {
    x &= 0x1fffff;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

int tile_points(const float* xyz, int64_t n, const char* spec, Tiling& out, std::string& err) {
    out = Tiling();
    if (n == 0) return DAS_OK;
    if (n > (int64_t)INT32_MAX) {
        err = "more than 2^31 - 1 voxels";
        return DAS_ESHAPE;
    }
    for (int64_t i = 0; i < 3 * n; ++i)
        if (!std::isfinite(xyz[i])) {
            err = "non-finite voxel coordinate";
            return DAS_EINVAL;
        }
    std::vector<float> uniq[3];
    int64_t n_ax[3];
    for (int a = 0; a < 3; ++a) {
        uniq[a].resize(n);
        for (int64_t i = 0; i < n; ++i) uniq[a][i] = xyz[3 * i + a];
        std::sort(uniq[a].begin(), uniq[a].end());
        uniq[a].erase(std::unique(uniq[a].begin(), uniq[a].end()), uniq[a].end());
        n_ax[a] = (int64_t)uniq[a].size();
    }
    const double cells = (double)n_ax[0] * (double)n_ax[1] * (double)n_ax[2];
    bool lattice = cells <= 2.0 * (double)n + 64.0 && (n_ax[0] > 1 || n_ax[1] > 1 || n_ax[2] > 1);
    std::vector<int32_t> cell;
    std::vector<int32_t> idx3;
    if (lattice) {
        cell.assign((size_t)cells, -1);
        idx3.resize(3 * n);
        for (int64_t i = 0; i < n && lattice; ++i) {
            int64_t id = 0;
            for (int a = 2; a >= 0; --a) {
                const int64_t k = std::lower_bound(uniq[a].begin(), uniq[a].end(), xyz[3 * i + a]) - uniq[a].begin();
                idx3[3 * i + a] = (int32_t)k;
            }
            id = ((int64_t)idx3[3 * i + 2] * n_ax[1] + idx3[3 * i + 1]) * n_ax[0] + idx3[3 * i];
            if (cell[id] >= 0) lattice = false;  // repeated point: not a lattice
            else cell[id] = (int32_t)i;
        }
    }
    if (lattice) {
        int32_t tile[3], wave[3];
        if (!parse_spec(spec, tile, wave)) default_dims(n_ax, tile, wave);
        const int64_t nt[3] = {(n_ax[0] + tile[0] - 1) / tile[0], (n_ax[1] + tile[1] - 1) / tile[1],
                               (n_ax[2] + tile[2] - 1) / tile[2]};
        const int wpt[3] = {tile[0] / wave[0], tile[1] / wave[1], tile[2] / wave[2]};
        std::vector<int32_t> slots(kSlots);
        for (int64_t bz = 0; bz < nt[2]; ++bz)
            for (int64_t by = 0; by < nt[1]; ++by)
                for (int64_t bx = 0; bx < nt[0]; ++bx) {
                    bool any = false;
                    for (int s = 0; s < kSlots; ++s) {
                        const int w = s / kLanes, l = s % kLanes;
                        const int wx = w % wpt[0], wy = (w / wpt[0]) % wpt[1], wz = w / (wpt[0] * wpt[1]);
                        const int lx = l % wave[0], ly = (l / wave[0]) % wave[1], lz = l / (wave[0] * wave[1]);
                        const int64_t ix = bx * tile[0] + wx * wave[0] + lx;
                        const int64_t iy = by * tile[1] + wy * wave[1] + ly;
                        const int64_t iz = bz * tile[2] + wz * wave[2] + lz;
                        int32_t v = -1;
                        if (ix < n_ax[0] && iy < n_ax[1] && iz < n_ax[2]) v = cell[(iz * n_ax[1] + iy) * n_ax[0] + ix];
                        slots[s] = v;
                        any |= v >= 0;
                    }
                    if (any) {
                        out.slot_to_vox.insert(out.slot_to_vox.end(), slots.begin(), slots.end());
                        out.tile_xyz.push_back((int32_t)bx);
                        out.tile_xyz.push_back((int32_t)by);
                        out.tile_xyz.push_back((int32_t)bz);
                        ++out.n_tiles;
                    }
                }
        for (int a = 0; a < 3; ++a) {
            out.tile_dims[a] = tile[a];
            out.wave_dims[a] = wave[a];
        }
        return DAS_OK;
    }
    // Not a lattice: group points along a Morton curve of their bounding box.
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = uniq[a].front();
        hi[a] = uniq[a].back();
    }
    std::vector<uint64_t> code(n);
    for (int64_t i = 0; i < n; ++i) {
        uint64_t c = 0;
        for (int a = 0; a < 3; ++a) {
            const double span = (double)hi[a] - (double)lo[a];
            const double q = span > 0 ? ((double)xyz[3 * i + a] - lo[a]) / span * 2097151.0 : 0.0;
            c |= spread21((uint64_t)std::llround(q)) << a;
        }
        code[i] = c;
    }
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return code[a] < code[b]; });
    out.n_tiles = (n + kSlots - 1) / kSlots;
    out.slot_to_vox.assign(out.n_tiles * kSlots, -1);
    for (int64_t t = 0; t < out.n_tiles; ++t) {
        out.tile_xyz.push_back((int32_t)t);
        out.tile_xyz.push_back(0);
        out.tile_xyz.push_back(0);
    }
    std::copy(order.begin(), order.end(), out.slot_to_vox.begin());
    return DAS_OK;
}

}  // namespace das

namespace das {

std::vector<int32_t> order_units(const Tiling& tl, const std::vector<int32_t>& item_off, int chunks, bool xcd_runs) {
    const int64_t n = tl.n_tiles;
    std::vector<int32_t> units;
    units.reserve((size_t)(n * chunks));
    auto cost = [&](int32_t t) { return item_off[t + 1] - item_off[t]; };
    if (xcd_runs) {  // contiguous runs of tiles per XCD (kept for comparison)
        const int64_t q = n / 8, r = n % 8;
        for (int64_t b = 0; b < n; ++b) {
            const int64_t x = b % 8, kk = b / 8;
            const int32_t t = (int32_t)(x < r ? x * (q + 1) + kk : r * (q + 1) + (x - r) * q + kk);
            for (int c = 0; c < chunks; ++c) units.push_back(t * chunks + c);
        }
        return units;
    }
    // columns = tiles sharing (x, y) tile coordinates; in row-major (y, x) order
    std::vector<int32_t> idx((size_t)n);
    std::iota(idx.begin(), idx.end(), 0);
    auto col_key = [&](int32_t t) { return std::make_pair(tl.tile_xyz[3 * t + 1], tl.tile_xyz[3 * t]); };
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return col_key(a) < col_key(b); });
    int64_t total = 0;
    for (int32_t t : idx) total += cost(t);
    // split the column sequence into 8 regions of about equal work (whole columns)
    std::vector<std::vector<int32_t>> region(8);
    int64_t acc = 0;
    int r = 0;
    for (size_t i = 0; i < idx.size();) {
        size_t j = i;
        int64_t col_cost = 0;
        while (j < idx.size() && col_key(idx[j]) == col_key(idx[i])) col_cost += cost(idx[j++]);
        if (r < 7 && acc > 0 && acc + col_cost / 2 > (total * (r + 1)) / 8) ++r;
        for (size_t k = i; k < j; ++k) region[r].push_back(idx[k]);
        acc += col_cost;
        i = j;
    }
    size_t longest = 0;
    for (auto& g : region) {
        std::stable_sort(g.begin(), g.end(), [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
        longest = std::max(longest, g.size() * (size_t)chunks);
    }
    for (size_t k = 0; k < longest; ++k)
        for (int x = 0; x < 8; ++x)
            if (k < region[x].size() * (size_t)chunks)
                units.push_back(region[x][k / chunks] * chunks + (int32_t)(k % chunks));
    return units;
}

}  // namespace das

// ---------------------------------------------------------------- checks
static int check_params(const das_params* p) {
    if (!p) return fail(DAS_EINVAL, "params is NULL");
    if (p->n_tx < 1 || p->n_elem < 1 || p->n_samples < 1 || p->n_frames < 1 || p->n_vox < 0)
        return fail(DAS_ESHAPE, "sizes must satisfy T, E, S, F >= 1 and V >= 0 (got T=%d E=%d S=%d F=%d V=%lld)",
                    p->n_tx, p->n_elem, p->n_samples, p->n_frames, (long long)p->n_vox);
    if ((double)p->n_tx * p->n_elem * p->n_samples * p->n_frames > 9.0e15)
        return fail(DAS_ESHAPE, "channel data larger than 2^53 samples");
    if (p->n_vox > (int64_t)INT32_MAX) return fail(DAS_ESHAPE, "more than 2^31 - 1 voxels");
    if ((double)p->n_tx * (double)p->n_elem > (double)INT32_MAX)
        return fail(DAS_ESHAPE, "T * E must fit in 31 bits");
    // one (t, e) record is addressed with 32-bit byte offsets (plus a window margin)
    if (((double)p->n_samples + 4200.0) * (double)p->n_frames * 8.0 > (double)INT32_MAX)
        return fail(DAS_ESHAPE, "a (transmit, element) record of S * F samples must stay below 2 GiB");
    if (!(std::isfinite(p->sound_speed) && p->sound_speed > 0)) return fail(DAS_EINVAL, "sound_speed must be finite and > 0");
    if (!(std::isfinite(p->fs) && p->fs > 0)) return fail(DAS_EINVAL, "fs must be finite and > 0");
    if (!(std::isfinite(p->f_demod) && p->f_demod >= 0)) return fail(DAS_EINVAL, "f_demod must be finite and >= 0");
    if (!std::isfinite(p->t0)) return fail(DAS_EINVAL, "t0 must be finite");
    if (!(std::isfinite(p->f_number) && p->f_number >= 0)) return fail(DAS_EINVAL, "f_number must be finite and >= 0");
    if (!(p->tukey_alpha >= 0 && p->tukey_alpha <= 1)) return fail(DAS_EINVAL, "tukey_alpha must be in [0, 1]");
    return DAS_OK;
}

static bool plan_live(const das_plan* plan) {
    std::lock_guard<std::mutex> g(g_mu);
    return plan && g_live.count(plan) && plan->magic == kMagic;
}

static void free_dev(das::PlanDev& d) {
    void* ptrs[] = {d.vx, d.vy, d.vz, d.tx, d.slot_vox, d.elemd, d.windows, d.items, d.item_off, d.wg_unit};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    d = das::PlanDev();
}

template <typename T>
static hipError_t upload(T** dst, const std::vector<T>& src, hipStream_t s) {
    hipError_t e = hipMalloc((void**)dst, std::max<size_t>(src.size(), 1) * sizeof(T));
    if (e != hipSuccess) return e;
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

extern "C" {

int das_version(void) { return (1 << 16) | 4; }

int das_kernel_variants(int32_t* fc_pitch_groups, int32_t capacity) {
    g_err.clear();
    if (capacity < 0) return fail(DAS_EINVAL, "capacity < 0");
    if (capacity > 0 && !fc_pitch_groups) return fail(DAS_EINVAL, "fc_pitch_groups is NULL");
    return das::list_variants(fc_pitch_groups, capacity);
}

int das_choose_kernel_variant(int32_t n_frames, int32_t max_window, int64_t n_tiles, double items_per_tile,
                              int32_t* fc_pitch_groups) {
    g_err.clear();
    if (!fc_pitch_groups) return fail(DAS_EINVAL, "fc_pitch_groups is NULL");
    if (n_frames < 1 || max_window < 0 || n_tiles < 1 || !(items_per_tile >= 0.0))
        return fail(DAS_EINVAL, "need n_frames >= 1, max_window >= 0, n_tiles >= 1, items_per_tile >= 0");
    const das::Variant v = das::choose_variant(n_frames, max_window, n_tiles, items_per_tile);
    if (v.fc == 0) return fail(DAS_ESHAPE, "no compiled variant for %d frames", (int)n_frames);
    fc_pitch_groups[0] = v.fc;
    fc_pitch_groups[1] = v.pitch;
    fc_pitch_groups[2] = v.groups;
    return DAS_OK;
}

const char* das_last_error(void) { return g_err.c_str(); }

const char* das_status_string(int status) {
    switch (status) {
        case DAS_OK: return "ok";
        case DAS_EINVAL: return "invalid argument";
        case DAS_ESHAPE: return "invalid shape";
        case DAS_EDTYPE: return "invalid dtype";
        case DAS_EALIGN: return "misaligned pointer";
        case DAS_EHIP: return "HIP runtime error";
        case DAS_ENOMEM: return "out of memory";
        default: return "unknown status";
    }
}

int das_plan_create(das_plan** out, const das_params* p, const float* elem_xyz, const float* vox_xyz,
                    const float* tx_arrival, void* stream) {
    g_err.clear();
    if (!out) return fail(DAS_EINVAL, "out is NULL");
    *out = nullptr;
    int st = check_params(p);
    if (st) return st;
    if (!elem_xyz) return fail(DAS_EINVAL, "elem_xyz is NULL");
    if (p->n_vox > 0 && (!vox_xyz || !tx_arrival)) return fail(DAS_EINVAL, "vox_xyz / tx_arrival is NULL");
    if (!aligned(elem_xyz, 4) || (vox_xyz && !aligned(vox_xyz, 4)) || (tx_arrival && !aligned(tx_arrival, 4)))
        return fail(DAS_EALIGN, "geometry pointers must be 4-byte aligned");

    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int64_t V = p->n_vox, T = p->n_tx, E = p->n_elem;
    std::vector<float> vox(3 * V), tx(T * V), elem(3 * E);
    hipError_t e;
    if (V > 0) {
        if ((e = hipMemcpyAsync(vox.data(), vox_xyz, vox.size() * 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
            return fail_hip(e, "copying vox_xyz");
        if ((e = hipMemcpyAsync(tx.data(), tx_arrival, tx.size() * 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
            return fail_hip(e, "copying tx_arrival");
    }
    if ((e = hipMemcpyAsync(elem.data(), elem_xyz, elem.size() * 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return fail_hip(e, "copying elem_xyz");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail_hip(e, "synchronising");
    for (float x : elem)
        if (!std::isfinite(x)) return fail(DAS_EINVAL, "non-finite element coordinate");
    for (float x : tx)
        if (!std::isfinite(x)) return fail(DAS_EINVAL, "non-finite transmit arrival time");

    das_plan* plan = new (std::nothrow) das_plan();
    if (!plan) return fail(DAS_ENOMEM, "host allocation failed");
    plan->p = *p;
    std::string err;
    st = das::tile_points(vox.data(), V, std::getenv("DAS_TILE"), plan->tiling, err);
    if (st) {
        delete plan;
        return fail(st, "%s", err.c_str());
    }
    const das::Tiling& tl = plan->tiling;
    const int64_t n_slots = tl.n_tiles * das::kSlots;
    if (tl.n_tiles > (int64_t)INT32_MAX / das::kSlots || tl.n_tiles * (int64_t)p->n_frames > (int64_t)INT32_MAX) {
        delete plan;
        return fail(DAS_ESHAPE, "too many tiles");
    }
    std::vector<float> vx(n_slots), vy(n_slots), vz(n_slots), txs(T * n_slots, 0.0f);
    for (int64_t t = 0; t < tl.n_tiles; ++t) {
        // empty slots take the coordinates of a valid point of their tile
        int32_t ref = -1;
        for (int k = 0; k < das::kSlots && ref < 0; ++k) ref = tl.slot_to_vox[t * das::kSlots + k];
        for (int k = 0; k < das::kSlots; ++k) {
            const int64_t sl = t * das::kSlots + k;
            const int32_t v = tl.slot_to_vox[sl];
            const int32_t src = v >= 0 ? v : ref;
            vx[sl] = vox[3 * src];
            vy[sl] = vox[3 * src + 1];
            vz[sl] = vox[3 * src + 2];
            if (v >= 0)
                for (int64_t k2 = 0; k2 < T; ++k2) txs[k2 * n_slots + sl] = tx[k2 * V + v];
        }
    }
    das::PlanDev& d = plan->dev;
    das_kparams& kp = d.kp;
    kp.T = p->n_tx;
    kp.E = p->n_elem;
    kp.S = p->n_samples;
    kp.F = p->n_frames;
    kp.n_slots = n_slots;
    d.n_vox = p->n_vox;
    kp.n_tiles = (int32_t)tl.n_tiles;
    kp.use_apod = p->f_number > 0 ? 1 : 0;
    kp.fs_c = p->fs / p->sound_speed;
    kp.fd_c = p->f_demod / p->sound_speed;
    kp.fs = p->fs;
    kp.fd = p->f_demod;
    kp.t0fs = p->t0 * p->fs;
    kp.two_fnum = (float)(2.0 * p->f_number);
    kp.alpha = (float)p->tukey_alpha;
    kp.inv_2alpha = p->tukey_alpha > 0 ? (float)(0.5 / p->tukey_alpha) : 0.0f;
    kp.edge_2alpha = p->tukey_alpha > 0 ? (float)((1.0 - p->tukey_alpha) * 0.5 / p->tukey_alpha) : 0.0f;
    // elements in one depth plane (linear and matrix arrays): the depth terms are per voxel
    kp.planar = 1;
    for (int64_t k = 1; k < E; ++k)
        if (elem[3 * k + 2] != elem[2]) kp.planar = 0;
    kp.z0 = kp.planar ? (double)elem[2] : 0.0;

    // element coordinates, then a 64-byte zero row (16-byte aligned) that the beamforming kernel reads in place of
    // samples outside a record
    const size_t zoff = (3 * (size_t)E + 1) / 2 * 2;
    std::vector<double> elemd(zoff + 8, 0.0);
    for (int64_t k = 0; k < 3 * E; ++k) elemd[(size_t)k] = (double)elem[k];
    unsigned long long* counts = nullptr;
    unsigned long long hc[3] = {0, 0, 0};
    if ((e = upload(&d.vx, vx, s)) != hipSuccess || (e = upload(&d.vy, vy, s)) != hipSuccess ||
        (e = upload(&d.vz, vz, s)) != hipSuccess || (e = upload(&d.tx, txs, s)) != hipSuccess ||
        (e = upload(&d.slot_vox, tl.slot_to_vox, s)) != hipSuccess || (e = upload(&d.elemd, elemd, s)) != hipSuccess)
        goto hip_fail;
    d.zrow = d.elemd + zoff;
    if ((e = hipMalloc((void**)&d.windows, std::max<int64_t>(1, 2 * tl.n_tiles * T * E) * sizeof(int32_t))) !=
        hipSuccess)
        goto hip_fail;
    if ((e = hipMalloc((void**)&counts, sizeof(hc))) != hipSuccess) goto hip_fail;
    if ((e = hipMemcpyAsync(counts, hc, sizeof(hc), hipMemcpyHostToDevice, s)) != hipSuccess) goto hip_fail;
    if ((e = das::launch_windows(d, counts, s)) != hipSuccess) goto hip_fail;
    if ((e = hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, s)) != hipSuccess) goto hip_fail;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) goto hip_fail;
    (void)hipFree(counts);
    counts = nullptr;
    plan->active_triples = (int64_t)hc[0];
    plan->processed_triples = (int64_t)hc[1];
    plan->max_window = (int32_t)hc[2];
    {
        // Work items per tile: the non-empty (t, e) windows, cut into pieces of at
        // most pitch - 1 rows, element-major so consecutive items share the
        // receive geometry.
        // average (transmit, element) pairs with a non-empty window per tile: processed triples per valid slot
        const double items_per_tile = p->n_vox > 0 ? (double)plan->processed_triples / (double)p->n_vox : 0.0;
        const das::Variant var = das::choose_variant(p->n_frames, plan->max_window, tl.n_tiles, items_per_tile);
        d.fc = var.fc;
        d.pitch = var.pitch;
        d.groups = var.groups;
        const int rows = var.pitch > 0 ? var.pitch - 1 : INT32_MAX;  // the direct kernel takes whole windows
        std::vector<int32_t> win((size_t)2 * tl.n_tiles * T * E);
        if (!win.empty() &&
            ((e = hipMemcpyAsync(win.data(), d.windows, win.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s)) !=
                 hipSuccess ||
             (e = hipStreamSynchronize(s)) != hipSuccess))
            goto hip_fail;
        std::vector<int4> items;
        std::vector<int32_t> off((size_t)tl.n_tiles + 1, 0);
        for (int64_t t = 0; t < tl.n_tiles; ++t) {
            off[t] = (int32_t)items.size();
            for (int64_t el = 0; el < E; ++el)
                for (int64_t k = 0; k < T; ++k) {
                    const int32_t* w = &win[2 * ((t * T + k) * E + el)];
                    for (int32_t r = 0; r < w[1]; r += rows)
                        items.push_back(make_int4((int)k, (int)el, w[0] + r, std::min(rows, w[1] - r)));
                }
            if (items.size() > (size_t)INT32_MAX) {
                e = hipErrorInvalidValue;
                goto hip_fail;
            }
        }
        off[tl.n_tiles] = (int32_t)items.size();
        if (das::stage_pairs(var.fc)) {
            // Stages: consecutive items of a tile whose windows fit one LDS buffer together (at most pitch - 1
            // rows) share a stage, i.e. one fill and one barrier.  Two int4 per stage; an absent second item
            // has zero rows.  DAS_PAIR=0 keeps one item per stage (same layout).  Variants that do not pair
            // keep one int4 per item.
            const char* pair_env = std::getenv("DAS_PAIR");
            const bool pair = !(pair_env != nullptr && std::strcmp(pair_env, "0") == 0);
            const int slack = das::fill_rows_per_thread(var.fc, var.pitch) - 1;
            std::vector<int4> stages;
            std::vector<int32_t> soff((size_t)tl.n_tiles + 1, 0);
            for (int64_t t = 0; t < tl.n_tiles; ++t) {
                soff[t] = (int32_t)(stages.size() / 2);
                for (int32_t i = off[t]; i < off[t + 1];) {
                    const int4 a = items[(size_t)i];
                    // the second window starts at a multiple of the fill rows per thread (at most
                    // slack + 1): reserve the slack
                    if (pair && i + 1 < off[t + 1] && a.w + slack + items[(size_t)i + 1].w <= rows) {
                        stages.push_back(a);
                        stages.push_back(items[(size_t)i + 1]);
                        i += 2;
                    } else {
                        stages.push_back(a);
                        stages.push_back(make_int4(0, 0, 0, 0));
                        i += 1;
                    }
                }
            }
            soff[tl.n_tiles] = (int32_t)(stages.size() / 2);
            items.swap(stages);
            off.swap(soff);
        }
        const int chunks = (p->n_frames + var.fc - 1) / var.fc;
        const char* ord = std::getenv("DAS_ORDER");
        const std::vector<int32_t> order =
            das::order_units(tl, off, chunks, ord != nullptr && std::strcmp(ord, "xcd") == 0);
        (void)hipFree(d.windows);
        d.windows = nullptr;
        if ((e = upload(&d.items, items, s)) != hipSuccess || (e = upload(&d.item_off, off, s)) != hipSuccess ||
            (e = upload(&d.wg_unit, order, s)) != hipSuccess)
            goto hip_fail;
        if ((e = das::prepare_variant(d)) != hipSuccess) goto hip_fail;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) goto hip_fail;
    }
    {
        std::lock_guard<std::mutex> g(g_mu);
        g_live.insert(plan);
    }
    *out = plan;
    return DAS_OK;

hip_fail:
    if (counts) (void)hipFree(counts);
    free_dev(d);
    delete plan;
    if (e == hipErrorOutOfMemory) return fail(DAS_ENOMEM, "device allocation failed");
    return fail_hip(e, "creating plan");
}

int das_plan_destroy(das_plan* plan) {
    g_err.clear();
    if (!plan) return DAS_OK;
    {
        std::lock_guard<std::mutex> g(g_mu);
        if (!g_live.count(plan)) return fail(DAS_EINVAL, "not a live plan (already destroyed?)");
        g_live.erase(plan);
    }
    free_dev(plan->dev);
    plan->magic = 0;
    delete plan;
    return DAS_OK;
}

int das_execute(const das_plan* plan, const void* iq, int dtype, void* out, void* stream) {
    g_err.clear();
    if (!plan_live(plan)) return fail(DAS_EINVAL, "plan is NULL or not live");
    if (dtype != DAS_IQ_C64 && dtype != DAS_IQ_C16F && dtype != DAS_IQ_C16BF)
        return fail(DAS_EDTYPE, "unknown IQ dtype %d", dtype);
    if (plan->p.n_vox == 0) return DAS_OK;
    if (!iq || !out) return fail(DAS_EINVAL, "iq / out is NULL");
    const size_t iq_align = dtype == DAS_IQ_C64 ? 8 : 4;
    if (!aligned(iq, iq_align)) return fail(DAS_EALIGN, "iq must be %zu-byte aligned", iq_align);
    if (!aligned(out, 8)) return fail(DAS_EALIGN, "out must be 8-byte aligned");
    const hipError_t e = das::launch_das(plan->dev, iq, dtype, out, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "launching das kernel");
    return DAS_OK;
}

int das_execute_per_tx(const das_plan* plan, const void* iq, int dtype, void* out, void* stream) {
    g_err.clear();
    if (!plan_live(plan)) return fail(DAS_EINVAL, "plan is NULL or not live");
    if (dtype != DAS_IQ_C64 && dtype != DAS_IQ_C16F && dtype != DAS_IQ_C16BF)
        return fail(DAS_EDTYPE, "unknown IQ dtype %d", dtype);
    if (plan->p.n_vox > 0 && !das::per_tx_supported(plan->dev))
        return fail(DAS_ESHAPE, "per-transmit output needs at most 4 transmits and at most 2 frames (plan: T=%d F=%d)",
                    plan->p.n_tx, plan->p.n_frames);
    if (plan->p.n_vox == 0) return DAS_OK;
    if (!iq || !out) return fail(DAS_EINVAL, "iq / out is NULL");
    const size_t iq_align = dtype == DAS_IQ_C64 ? 8 : 4;
    if (!aligned(iq, iq_align)) return fail(DAS_EALIGN, "iq must be %zu-byte aligned", iq_align);
    if (!aligned(out, 8)) return fail(DAS_EALIGN, "out must be 8-byte aligned");
    const hipError_t e = das::launch_das_per_tx(plan->dev, iq, dtype, out, reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "launching per-transmit das kernel");
    return DAS_OK;
}

int das_tx_plane_wave(float* tx_out, const float* vox_xyz, int64_t n_vox, const double* angles, int32_t n_tx,
                      double sound_speed, void* stream) {
    g_err.clear();
    if (n_tx < 1 || n_vox < 0) return fail(DAS_ESHAPE, "need n_tx >= 1 and n_vox >= 0");
    if (!angles) return fail(DAS_EINVAL, "angles is NULL");
    if (!(std::isfinite(sound_speed) && sound_speed > 0)) return fail(DAS_EINVAL, "sound_speed must be finite and > 0");
    if (n_vox > 0 && (!tx_out || !vox_xyz)) return fail(DAS_EINVAL, "tx_out / vox_xyz is NULL");
    if (n_vox > 0 && (!aligned(tx_out, 4) || !aligned(vox_xyz, 4))) return fail(DAS_EALIGN, "pointers must be 4-byte aligned");
    std::vector<double> nrm(3 * (size_t)n_tx);
    for (int32_t t = 0; t < n_tx; ++t) {
        const double th = angles[2 * t], ph = angles[2 * t + 1];
        if (!std::isfinite(th) || !std::isfinite(ph)) return fail(DAS_EINVAL, "non-finite angle");
        nrm[3 * t] = std::sin(th) * std::cos(ph);
        nrm[3 * t + 1] = std::sin(ph);
        nrm[3 * t + 2] = std::cos(th) * std::cos(ph);
    }
    const hipError_t e = das::launch_tx_plane_wave(tx_out, vox_xyz, n_vox, nrm.data(), n_tx, 1.0 / sound_speed,
                                                   reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "launching plane-wave kernel");
    return DAS_OK;
}

int das_plan_query(const das_plan* plan, das_plan_info* info) {
    g_err.clear();
    if (!plan_live(plan)) return fail(DAS_EINVAL, "plan is NULL or not live");
    if (!info) return fail(DAS_EINVAL, "info is NULL");
    info->n_vox = plan->p.n_vox;
    info->n_slots = plan->tiling.n_tiles * das::kSlots;
    info->n_tiles = plan->tiling.n_tiles;
    info->total_triples = plan->p.n_vox * (int64_t)plan->p.n_elem * plan->p.n_tx;
    info->active_triples = plan->active_triples;
    info->processed_triples = plan->processed_triples;
    for (int a = 0; a < 3; ++a) info->tile_dims[a] = plan->tiling.tile_dims[a];
    info->max_window = plan->max_window;
    info->kernel_fc = plan->dev.fc;
    info->kernel_pitch = plan->dev.pitch;
    info->kernel_groups = plan->dev.groups;
    return DAS_OK;
}

int das_tile_order(const float* vox_xyz, int64_t n_vox, int32_t* slot_to_vox, int64_t capacity, int64_t* n_slots,
                   int32_t* tile_dims) {
    g_err.clear();
    if (!n_slots) return fail(DAS_EINVAL, "n_slots is NULL");
    if (n_vox < 0) return fail(DAS_ESHAPE, "n_vox < 0");
    if (n_vox > 0 && !vox_xyz) return fail(DAS_EINVAL, "vox_xyz is NULL");
    das::Tiling tl;
    std::string err;
    const int st = das::tile_points(vox_xyz, n_vox, std::getenv("DAS_TILE"), tl, err);
    if (st) return fail(st, "%s", err.c_str());
    *n_slots = tl.n_tiles * das::kSlots;
    if (tile_dims)
        for (int a = 0; a < 3; ++a) tile_dims[a] = tl.tile_dims[a];
    if (slot_to_vox) {
        if (capacity < *n_slots) return fail(DAS_ESHAPE, "capacity %lld < n_slots %lld", (long long)capacity, (long long)*n_slots);
        std::copy(tl.slot_to_vox.begin(), tl.slot_to_vox.end(), slot_to_vox);
    }
    return DAS_OK;
}

}  // extern "C"
