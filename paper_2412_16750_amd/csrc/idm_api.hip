// Host runtime behind the C ABI declared in include/idm.h: validation, lane
// packing into work-group bundles, workspace layout, kernel dispatch, HIP
// graph capture/replay of the step and fit sequences, and the autotuner.
#include "idm.h"
#include "idm_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace idmx;

// Device scratch of idm_sim_backward_noalloc (its workspace), one copy per
// GPU.  Host code never uses this name as an address: the device address of
// each GPU's copy comes from hipGetSymbolAddress (static_scratch below).
static __device__ __align__(256) char scratch[IDM_STATIC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err = "no error";

idm_status fail(idm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

idm_status hip_fail(hipError_t e, const char *what) {
    return fail(IDM_ERR_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

constexpr size_t kAlign = 256;
// Resident work-group model used to size launch levels: MI355X has 256 compute
// units of at most 2048 resident threads (the forward kernels reach it).
constexpr int64_t kRoundCUs = 256;
constexpr int kThreadsPerCU = 2048;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Shape {
    int threads = 0, per_thread = 0;
    int K = 0;   // checkpoint interval
    int KB = 0;  // backward register block (divides K)
    int grid = 0;
    bool stored = false;  // the forward keeps every step's states for the backward
    int tile = 0;         // J > 0: halo tiles advancing J steps per launch (stored, one
                          // vehicle per thread)
};

bool valid_threads(int t) { return t == 64 || t == 128 || t == 256 || t == 512 || t == 1024; }
bool valid_per_thread(int r) { return r == 1 || r == 2 || r == 4; }

// Backward register blocks instantiated for each vehicles-per-thread count.
std::vector<int> kbs_for(int r) {
    if (r == 1) return {8, 16, 32};
    if (r == 2) return {8, 16, 32};
    return {4, 8};
}

bool kb_ok(int r, int KB) {
    auto v = kbs_for(r);
    return std::find(v.begin(), v.end(), KB) != v.end();
}

// Default register block for a checkpoint interval: the largest instantiated
// block that divides K and keeps the kernel free of register spills (16 for
// one or two vehicles per thread, 8 for four); 0 if none divides K.
int default_kb(int r, int K) {
    const int cap = r == 4 ? 8 : 16;
    int best = 0;
    for (int kb : kbs_for(r))
        if (kb <= cap && K % kb == 0) best = kb;
    return best;
}

}  // namespace

struct idm_plan {
    idm_problem pb{};
    std::vector<int32_t> offsets;
    int32_t max_lane = 0;
    Shape sh;
    // bundle layout
    int32_t n_bundles = 0;
    int64_t n_slots = 0;
    int32_t n_bnd = 0;                  // piece boundaries of lanes longer than a bundle
    std::vector<int32_t> level_start;   // bundles of launch level l: [start[l], start[l+1])
    int32_t *d_gidx = nullptr;
    uint8_t *d_flags = nullptr;
    int32_t *d_bnd = nullptr;           // [2][n_bundles]: bnd_in, bnd_out (null if n_bnd = 0)
    float *d_zero = nullptr;  // 64 zero floats read in place of absent upstream inputs
    uint8_t *d_head = nullptr;  // [N] 1 = first vehicle of its lane (feature kernel)
    int32_t *d_lane_off = nullptr;  // [L+1] lane offsets on the device
    int32_t *d_lane_of = nullptr;   // [N] lane of every vehicle
    // graphs
    hipGraphExec_t step_exec = nullptr;
    idm_step_args step_key{};
    hipGraphExec_t fit_exec = nullptr;
    std::vector<unsigned char> fit_key;
    // graphs cannot be captured on the legacy null stream: null-stream callers
    // get a plan-owned side stream (default priority), joined by events
    hipStream_t side = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int32_t tuned_cached = 0;  // the last autotune took its shape from the cache
    int32_t store_pref = 0;    // idm_tuning.store_states: 0, 1, or 2 = the autotuner chooses
    int32_t n_tiles = 0;       // halo tiles (= n_bundles) when sh.tile > 0, else 0
};

namespace {

int32_t nblk_of(const idm_plan *p) {
    return p->pb.n_steps == 0 ? 0 : (p->pb.n_steps + p->sh.K - 1) / p->sh.K;
}

// Piece boundaries when lanes are cut into bundles of `cap` slots: a lane of
// n > cap vehicles has ceil(n / cap) pieces.
int64_t count_boundaries(const std::vector<int32_t> &offsets, int L, int64_t cap) {
    int64_t n = 0;
    for (int l = 0; l < L; ++l) {
        const int64_t sz = offsets[l + 1] - offsets[l];
        if (sz > cap) n += (sz + cap - 1) / cap - 1;
    }
    return n;
}

// Workspace dimensions of a launch shape: checkpoint interval, piece
// boundaries, kept states and halo tiles.
struct WsDims {
    int K = 0;
    int64_t nbnd = 0;
    bool stored = false;
    int64_t ntile = 0;  // halo tiles, 0 for bundles
};

WsDims dims_of(const idm_plan *p) {
    WsDims w;
    w.K = p->sh.K;
    w.nbnd = p->n_bnd;
    w.stored = p->sh.stored;
    w.ntile = p->n_tiles;
    return w;
}

WsDims dims(int K, int64_t nbnd, bool stored, int64_t ntile = 0) {
    WsDims w;
    w.K = K;
    w.nbnd = nbnd;
    w.stored = stored;
    w.ntile = ntile;
    return w;
}

// Per-work-group partials: one per bundle (at most one per lane piece), or
// one per halo tile.
int64_t n_parts(const idm_plan *p, const WsDims &w) {
    return w.ntile > 0 ? w.ntile : (int64_t)p->pb.n_lanes + w.nbnd;
}

// Workspace layout: [loss partials: one double per bundle or tile][forward
// diagnostics: two uint64 per bundle or tile][fit: 7N doubles][checkpoints]
// [boundary states: n_bnd x (S+1) float2][boundary adjoint contributions:
// n_bnd x S float2][stored states: (S+1) x N displacements, then (S+1) x N
// speeds][halo tiles: carried adjoints 2 x [2][N] floats, gp0 sums [N]
// floats, parameter and loss sums [6][N] doubles].  A plan that keeps every
// step's states has no checkpoints and no piece boundaries; any other has no
// stored states; only halo tiles have the last part.
size_t ws_loss_off(const idm_plan *) { return 0; }
size_t ws_diag_off(const idm_plan *p, const WsDims &w) {
    return align_up(sizeof(double) * (size_t)n_parts(p, w));
}
size_t ws_fit_off(const idm_plan *p, const WsDims &w) {
    return ws_diag_off(p, w) + align_up(2 * sizeof(uint64_t) * (size_t)n_parts(p, w));
}
size_t ws_ckpt_off(const idm_plan *p, const WsDims &w) {
    return ws_fit_off(p, w) + align_up(sizeof(double) * 7 * (size_t)p->pb.n_vehicles);
}
size_t ckpt_bytes(const idm_plan *p, const WsDims &w) {
    if (w.stored) return 0;
    size_t nb = p->pb.n_steps == 0 ? 0 : (size_t)(p->pb.n_steps + w.K - 1) / w.K;
    return align_up(nb * 2 * sizeof(float) * (size_t)p->pb.n_vehicles);
}
size_t ws_ext_off(const idm_plan *p, const WsDims &w) { return ws_ckpt_off(p, w) + ckpt_bytes(p, w); }
size_t state_rows_bytes(const idm_plan *p) {
    return align_up(((size_t)p->pb.n_steps + 1) * sizeof(float) * (size_t)p->pb.n_vehicles);
}
size_t ext_state_bytes(const idm_plan *p, int64_t nbnd) {
    return align_up((size_t)nbnd * ((size_t)p->pb.n_steps + 1) * 2 * sizeof(float));
}
size_t ws_states_off(const idm_plan *p, const WsDims &w) {
    return ws_ext_off(p, w) + ext_state_bytes(p, w.nbnd) +
           align_up((size_t)w.nbnd * (size_t)p->pb.n_steps * 2 * sizeof(float));
}
size_t ws_tile_off(const idm_plan *p, const WsDims &w) {
    return ws_states_off(p, w) + (w.stored ? 2 * state_rows_bytes(p) : 0);
}
size_t tile_carry_bytes(const idm_plan *p) {
    return align_up(2 * sizeof(float) * (size_t)p->pb.n_vehicles);
}
size_t tile_gp0_bytes(const idm_plan *p) {
    return align_up(sizeof(float) * (size_t)p->pb.n_vehicles);
}
size_t tile_bytes(const idm_plan *p, const WsDims &w) {
    if (w.ntile == 0) return 0;
    return 2 * tile_carry_bytes(p) + tile_gp0_bytes(p) +
           align_up(6 * sizeof(double) * (size_t)p->pb.n_vehicles);
}
size_t ws_total(const idm_plan *p, const WsDims &w) { return ws_tile_off(p, w) + tile_bytes(p, w); }
size_t ws_total(const idm_plan *p) { return ws_total(p, dims_of(p)); }
size_t ws_fit_off(const idm_plan *p) { return ws_fit_off(p, dims_of(p)); }
size_t ws_diag_off(const idm_plan *p) { return ws_diag_off(p, dims_of(p)); }
size_t ws_ckpt_off(const idm_plan *p) { return ws_ckpt_off(p, dims_of(p)); }
size_t ws_states_off(const idm_plan *p) { return ws_states_off(p, dims_of(p)); }

void drop_graphs(idm_plan *p) {
    if (p->step_exec) hipGraphExecDestroy(p->step_exec);
    if (p->fit_exec) hipGraphExecDestroy(p->fit_exec);
    p->step_exec = nullptr;
    p->fit_exec = nullptr;
    p->fit_key.clear();
    memset(&p->step_key, 0, sizeof p->step_key);
}

// Pack lanes into bundles of `cap` slots.  A lane longer than `cap` is cut
// into pieces of exactly `cap` vehicles and a remainder; piece j opens its own
// bundle and runs in launch level j (the forward walks the levels upwards, the
// backward downwards), the boundary between pieces j-1 and j getting one row of
// the boundary buffers.  Whole lanes then go best-fit decreasing (ties keep
// lane order) into the room left by remainders or into new bundles, and the
// bundles of whole lanes only fill up each level's last round of resident
// work-groups.  Within a level, bundles are sorted by fill (largest first), so
// a persistent grid starts with the most work.
// Deterministic; host only.
struct Layout {
    int64_t n_bundles = 0, cap = 0;
    int32_t n_bnd = 0;
    std::vector<int32_t> gidx;
    std::vector<uint8_t> flags;
    std::vector<int32_t> bnd_in, bnd_out;  // per bundle, -1 = none
    std::vector<int32_t> level, level_start;
};

// Halo tiles of T = `threads` slots advancing J steps per launch.  Lanes of
// n <= T vehicles share tiles (pack_whole_lanes).  A longer lane is cut into
// the fewest tiles of at most T - 1 slots that hold it, m = ceil((n - J) /
// (T - 1 - J)): the forward's first tile (the lane head) and the backward's
// last (the lane tail) need no halo on that side, so each direction splits
// the lane on its own, the m tiles' slot counts (owned vehicles plus halo) as
// equal as integers allow.  A cut tile never fills its work-group: in the
// backward the last thread gathers the contribution of thread 0 (the slot
// after it, modulo T), which is exactly zero only for padding or a lane
// head, so the slot after a lane tail must be padding or a lane head.
// fn(lane start, lane end, tile j, m, forward owned [lo, hi), backward owned
// [lo, hi)) for every cut tile, lane by lane.
template <class F>
void for_each_tile(const std::vector<int32_t> &offsets, int L, int threads, int J, F fn) {
    for (int l = 0; l < L; ++l) {
        const int32_t s0 = offsets[l], e0 = offsets[l + 1];
        const int64_t n = e0 - s0;
        if (n <= threads) continue;
        const int64_t cap = threads - 1;  // J < T, both even: cap - J >= 1
        const int64_t m = (n - J + (cap - J) - 1) / (cap - J);
        const int64_t q = n + (m - 1) * J;  // slots over all tiles
        const int64_t base = q / m, rem = q % m;
        auto slots = [&](int64_t j) { return base + (j < rem ? 1 : 0); };
        // forward: tile 0 has no halo ahead; backward: tile m - 1 none behind
        int32_t flo = s0, blo = s0;
        for (int64_t j = 0; j < m; ++j) {
            const int32_t fhi = flo + (int32_t)(slots(j) - (j > 0 ? J : 0));
            const int32_t bhi = blo + (int32_t)(slots(m - 1 - j) - (j < m - 1 ? J : 0));
            fn(s0, e0, (int)j, (int)m, flo, fhi, blo, bhi);
            flo = fhi;
            blo = bhi;
        }
    }
}

// Lanes of at most T vehicles share tiles of T slots: best-fit decreasing
// (ties keep lane order), as bundles of whole lanes are packed; a tile holds
// its lanes one after another, in the order they were placed.  Each such tile
// starts with a lane head, so even a full one gives its last thread an exactly
// zero contribution from thread 0, and every vehicle in it is owned for any
// number of steps (no halo).  Returns the lanes of each tile.
std::vector<std::vector<int>> pack_whole_lanes(const std::vector<int32_t> &offsets, int L,
                                               int threads) {
    std::vector<int> order;
    for (int l = 0; l < L; ++l) {
        const int64_t sz = offsets[l + 1] - offsets[l];
        if (sz > 0 && sz <= threads) order.push_back(l);
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return (offsets[x + 1] - offsets[x]) > (offsets[y + 1] - offsets[y]);
    });
    std::vector<std::vector<int>> tiles;
    std::vector<int64_t> fill;
    std::multimap<int64_t, int> room;  // free slots -> tile
    for (int l : order) {
        const int64_t sz = offsets[l + 1] - offsets[l];
        auto it = room.lower_bound(sz);
        int b;
        if (it == room.end()) {
            b = (int)tiles.size();
            tiles.emplace_back();
            fill.push_back(0);
        } else {
            b = it->second;
            room.erase(it);
        }
        tiles[b].push_back(l);
        fill[b] += sz;
        if (threads - fill[b] > 0) room.emplace(threads - fill[b], b);
    }
    return tiles;
}

int64_t count_tiles(const std::vector<int32_t> &offsets, int L, int threads, int J) {
    int64_t n = 0;
    for_each_tile(offsets, L, threads, J,
                  [&](int32_t, int32_t, int, int, int32_t, int32_t, int32_t, int32_t) { ++n; });
    return n + (int64_t)pack_whole_lanes(offsets, L, threads).size();
}

// Slot tables of halo tiles: tiles x threads forward slots, then tiles x
// threads backward slots; the cut lanes' tiles first, then the shared tiles of
// whole lanes.  A cut tile's forward slots hold up to J halo vehicles ahead of
// the owned ones, the first slot flagged as a lane head; its backward slots
// the owned vehicles, then up to J halo vehicles behind them, the head flag
// only on a true lane head.  Tile b of the forward and tile b of the backward
// cover the same lane but may own different vehicles.  A shared tile is the
// same in both tables: its lanes whole, every vehicle owned.
idm_status compute_tiles(const std::vector<int32_t> &offsets, int L, const Shape &sh, Layout &out) {
    const int NT = sh.threads, J = sh.tile;
    const int64_t nb = count_tiles(offsets, L, NT, J);
    if (2 * nb * NT >= ((int64_t)1 << 40) || nb >= ((int64_t)1 << 31))
        return fail(IDM_ERR_LAYOUT, "layout too large");
    out.n_bundles = nb;
    out.cap = NT;
    out.n_bnd = 0;
    out.gidx.assign((size_t)(2 * nb * NT), -1);
    out.flags.assign((size_t)(2 * nb * NT), 0);
    out.bnd_in.assign((size_t)nb, -1);
    out.bnd_out.assign((size_t)nb, -1);
    out.level.assign((size_t)nb, 0);
    out.level_start = {0, (int32_t)nb};
    int64_t b = 0;
    for_each_tile(offsets, L, NT, J,
                  [&](int32_t ls, int32_t le, int, int, int32_t flo, int32_t fhi, int32_t blo,
                      int32_t bhi) {
                      int64_t s = b * NT;
                      const int32_t f0 = std::max<int32_t>(ls, flo - J);
                      for (int32_t i = f0; i < fhi; ++i, ++s) {
                          out.gidx[(size_t)s] = i;
                          uint8_t f = SLOT_VALID;
                          if (i == f0) f |= SLOT_HEAD;
                          if (i >= flo) f |= SLOT_OWNED;
                          if (i == le - 1) f |= SLOT_TAIL;
                          out.flags[(size_t)s] = f;
                      }
                      s = (nb + b) * NT;
                      const int32_t b1 = (int32_t)std::min<int64_t>(le, (int64_t)bhi + J);
                      for (int32_t i = blo; i < b1; ++i, ++s) {
                          out.gidx[(size_t)s] = i;
                          uint8_t f = SLOT_VALID;
                          if (i == ls) f |= SLOT_HEAD;
                          if (i < bhi) f |= SLOT_OWNED;
                          if (i == le - 1) f |= SLOT_TAIL;
                          out.flags[(size_t)s] = f;
                      }
                      ++b;
                  });
    for (const std::vector<int> &lanes : pack_whole_lanes(offsets, L, NT)) {
        int64_t s = b * NT;
        for (int l : lanes) {
            for (int32_t i = offsets[l]; i < offsets[l + 1]; ++i, ++s) {
                uint8_t f = SLOT_VALID | SLOT_OWNED;
                if (i == offsets[l]) f |= SLOT_HEAD;
                if (i == offsets[l + 1] - 1) f |= SLOT_TAIL;
                out.gidx[(size_t)s] = out.gidx[(size_t)(s + nb * NT)] = i;
                out.flags[(size_t)s] = out.flags[(size_t)(s + nb * NT)] = f;
            }
        }
        ++b;
    }
    return IDM_OK;
}

idm_status compute_layout(const std::vector<int32_t> &offsets, int L, const Shape &sh, Layout &out) {
    if (sh.tile > 0) return compute_tiles(offsets, L, sh, out);
    const int64_t cap = (int64_t)sh.threads * sh.per_thread;
    struct Item {
        int32_t lo, hi;
        bool lane_head, lane_tail;
    };
    std::vector<std::vector<Item>> bundles;
    std::vector<int64_t> fill;
    std::vector<int32_t> level, bin, bout;
    std::multimap<int64_t, int> room;  // remaining capacity -> bundle
    auto open = [&](int32_t lv, int32_t in) {
        bundles.emplace_back();
        fill.push_back(0);
        level.push_back(lv);
        bin.push_back(in);
        bout.push_back(-1);
        return (int)bundles.size() - 1;
    };
    int64_t nbnd = 0;
    int32_t n_levels = 1;
    for (int l = 0; l < L; ++l) {
        const int64_t sz = offsets[l + 1] - offsets[l];
        if (sz <= cap) continue;
        const int64_t np = (sz + cap - 1) / cap;
        if (np >= ((int64_t)1 << 20) || nbnd + np >= ((int64_t)1 << 30))
            return fail(IDM_ERR_LAYOUT, "lane %d: too many pieces", l);
        n_levels = std::max<int32_t>(n_levels, (int32_t)np);
        int prev = -1;
        for (int64_t j = 0; j < np; ++j) {
            const int32_t lo = (int32_t)(offsets[l] + j * cap);
            const int32_t hi = (int32_t)std::min<int64_t>(lo + cap, offsets[l + 1]);
            int32_t in = -1;
            if (j > 0) {
                in = (int32_t)nbnd++;
                bout[prev] = in;
            }
            const int b = open((int32_t)j, in);
            bundles[b].push_back({lo, hi, j == 0, j == np - 1});
            fill[b] = hi - lo;
            if (cap - fill[b] > 0) room.emplace(cap - fill[b], b);
            prev = b;
        }
    }
    std::vector<int> order;
    order.reserve(L);
    for (int l = 0; l < L; ++l) {
        const int64_t sz = offsets[l + 1] - offsets[l];
        if (sz > 0 && sz <= cap) order.push_back(l);
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return (offsets[x + 1] - offsets[x]) > (offsets[y + 1] - offsets[y]);
    });
    for (int l : order) {
        const int64_t sz = offsets[l + 1] - offsets[l];
        auto it = room.lower_bound(sz);
        int b;
        if (it == room.end()) {
            b = open(-1, -1);
        } else {
            b = it->second;
            room.erase(it);
        }
        bundles[b].push_back({offsets[l], offsets[l + 1], true, true});
        fill[b] += sz;
        if (cap - fill[b] > 0) room.emplace(cap - fill[b], b);
    }
    const int64_t nb = (int64_t)bundles.size();
    if (nb * cap >= ((int64_t)1 << 40) || nb >= ((int64_t)1 << 31))
        return fail(IDM_ERR_LAYOUT, "layout too large");
    // bundles of whole lanes only, fullest first: into the room left in the
    // last round of resident work-groups of each level (level 0 first), the
    // rest into level 0, so that the levels take as few rounds as one launch
    // of all bundles would
    const int64_t q = kRoundCUs * std::max(1, kThreadsPerCU / sh.threads);
    std::vector<int64_t> count((size_t)n_levels, 0);
    std::vector<int> free_b;
    for (int64_t b = 0; b < nb; ++b) {
        if (level[b] >= 0)
            ++count[level[b]];
        else
            free_b.push_back((int)b);
    }
    std::stable_sort(free_b.begin(), free_b.end(), [&](int x, int y) { return fill[x] > fill[y]; });
    size_t next = 0;
    for (int32_t lv = 0; lv < n_levels && next < free_b.size(); ++lv) {
        const int64_t room_lv = (count[lv] + q - 1) / q * q - count[lv];
        for (int64_t i = 0; i < room_lv && next < free_b.size(); ++i) {
            level[free_b[next++]] = lv;
            ++count[lv];
        }
    }
    for (; next < free_b.size(); ++next) level[free_b[next]] = 0;
    std::vector<int> border((size_t)nb);
    for (int64_t i = 0; i < nb; ++i) border[i] = (int)i;
    std::stable_sort(border.begin(), border.end(), [&](int x, int y) {
        return level[x] != level[y] ? level[x] < level[y] : fill[x] > fill[y];
    });
    out.n_bundles = nb;
    out.cap = cap;
    out.n_bnd = (int32_t)nbnd;
    out.gidx.assign((size_t)(nb * cap), -1);
    out.flags.assign((size_t)(nb * cap), 0);
    out.bnd_in.assign((size_t)nb, -1);
    out.bnd_out.assign((size_t)nb, -1);
    out.level.assign((size_t)nb, 0);
    out.level_start.assign((size_t)n_levels + 1, 0);
    for (int64_t bi = 0; bi < nb; ++bi) {
        const int b = border[bi];
        out.bnd_in[bi] = bin[b];
        out.bnd_out[bi] = bout[b];
        out.level[bi] = level[b];
        ++out.level_start[level[b] + 1];
        int64_t s = bi * cap;
        for (const Item &it : bundles[b]) {
            for (int32_t i = it.lo; i < it.hi; ++i, ++s) {
                out.gidx[s] = i;
                uint8_t f = SLOT_VALID;
                if (i == it.lo && it.lane_head) f |= SLOT_HEAD;
                if (i == it.hi - 1 && it.lane_tail) f |= SLOT_TAIL;
                out.flags[s] = f;
            }
        }
    }
    for (int32_t lv = 0; lv < n_levels; ++lv) out.level_start[lv + 1] += out.level_start[lv];
    if (sh.stored && out.n_bnd > 0)
        return fail(IDM_ERR_UNSUPPORTED,
                    "keeping every step's states needs whole lanes in a bundle: a %d x %d bundle "
                    "cuts the longest lane into pieces",
                    sh.threads, sh.per_thread);
    return IDM_OK;
}

idm_status build_layout(idm_plan *p, const Shape &sh) {
    Layout lay;
    idm_status r = compute_layout(p->offsets, p->pb.n_lanes, sh, lay);
    if (r != IDM_OK) return r;
    int32_t *dg = nullptr;
    uint8_t *df = nullptr;
    size_t n = lay.gidx.size() ? lay.gidx.size() : 1;
    hipError_t e = hipMalloc(&dg, n * sizeof(int32_t));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(slot table)");
    e = hipMalloc(&df, n);
    if (e != hipSuccess) {
        hipFree(dg);
        return hip_fail(e, "hipMalloc(slot flags)");
    }
    if (!lay.gidx.empty()) {
        e = hipMemcpy(dg, lay.gidx.data(), lay.gidx.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(df, lay.flags.data(), lay.flags.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            hipFree(dg);
            hipFree(df);
            return hip_fail(e, "hipMemcpy(slot table)");
        }
    }
    int32_t *db = nullptr;
    if (lay.n_bnd > 0) {
        const size_t nb = (size_t)lay.n_bundles;
        e = hipMalloc(&db, 2 * nb * sizeof(int32_t));
        if (e == hipSuccess)
            e = hipMemcpy(db, lay.bnd_in.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(db + nb, lay.bnd_out.data(), nb * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            hipFree(dg);
            hipFree(df);
            if (db) hipFree(db);
            return hip_fail(e, "boundary table");
        }
    }
    // the tables below are made once per plan; a failure frees this layout
    auto fail_tables = [&](hipError_t err, const char *what) {
        hipFree(dg);
        hipFree(df);
        if (db) hipFree(db);
        return hip_fail(err, what);
    };
    if (!p->d_lane_off) {
        std::vector<int32_t> lane_of((size_t)p->pb.n_vehicles, 0);
        for (int l = 0; l < p->pb.n_lanes; ++l)
            for (int32_t i = p->offsets[l]; i < p->offsets[l + 1]; ++i) lane_of[(size_t)i] = l;
        e = hipMalloc(&p->d_lane_off, p->offsets.size() * sizeof(int32_t));
        if (e == hipSuccess)
            e = hipMemcpy(p->d_lane_off, p->offsets.data(), p->offsets.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc(&p->d_lane_of, lane_of.size() * sizeof(int32_t));
        if (e == hipSuccess)
            e = hipMemcpy(p->d_lane_of, lane_of.data(), lane_of.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail_tables(e, "lane tables");
    }
    if (!p->d_head) {
        std::vector<uint8_t> head((size_t)p->pb.n_vehicles, 0);
        for (int l = 0; l < p->pb.n_lanes; ++l)
            if (p->offsets[l + 1] > p->offsets[l]) head[(size_t)p->offsets[l]] = 1;
        e = hipMalloc(&p->d_head, head.size());
        if (e == hipSuccess) e = hipMemcpy(p->d_head, head.data(), head.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail_tables(e, "head flags");
    }
    if (!p->d_zero) {
        e = hipMalloc(&p->d_zero, 64 * sizeof(float));
        if (e == hipSuccess) e = hipMemset(p->d_zero, 0, 64 * sizeof(float));
        if (e != hipSuccess) return fail_tables(e, "hipMalloc(zero word)");
    }
    if (p->d_gidx) hipFree(p->d_gidx);
    if (p->d_flags) hipFree(p->d_flags);
    if (p->d_bnd) hipFree(p->d_bnd);
    p->d_gidx = dg;
    p->d_flags = df;
    p->d_bnd = db;
    p->n_bundles = (int32_t)lay.n_bundles;
    p->n_slots = lay.n_bundles * lay.cap;
    p->n_bnd = lay.n_bnd;
    p->level_start = lay.level_start;
    p->sh = sh;
    p->n_tiles = sh.tile > 0 ? p->n_bundles : 0;
    if (p->sh.grid > p->n_bundles) p->sh.grid = p->n_bundles;
    drop_graphs(p);
    return IDM_OK;
}

// Default launch shape: one vehicle per thread when K allows it (most
// work-groups), the smallest bundle that holds the longest lane, or 1024
// threads with longer lanes cut into pieces; K from the problem.
idm_status choose_shape(const idm_plan *p, const idm_tuning *tu, Shape &sh) {
    int K = p->pb.ckpt_every;
    if (tu && tu->ckpt_every > 0) K = tu->ckpt_every;
    const int KB_req = tu ? tu->block : 0;
    if (K <= 0) K = KB_req > 0 ? KB_req : 32;
    if (tu && (tu->threads || tu->per_thread)) {
        // 576, 640 and 768 threads: halo tiles only (checked below)
        const bool tile_threads =
            tu->threads == 576 || tu->threads == 640 || tu->threads == 768;
        if (!(valid_threads(tu->threads) || (tile_threads && tu->tile_steps > 0)) ||
            !valid_per_thread(tu->per_thread))
            return fail(IDM_ERR_UNSUPPORTED, "tuning threads=%d per_thread=%d not supported",
                        tu->threads, tu->per_thread);
        sh.threads = tu->threads;
        sh.per_thread = tu->per_thread;
        if ((int64_t)sh.threads * sh.per_thread < p->max_lane && sh.per_thread != 1)
            return fail(IDM_ERR_UNSUPPORTED,
                        "a %d-vehicle lane does not fit %d x %d slots: lanes cut into pieces "
                        "need one vehicle per thread",
                        p->max_lane, sh.threads, sh.per_thread);
    } else {
        const int64_t need = std::max<int64_t>(p->max_lane, 1);
        bool found = false;
        for (int r : {1, 2, 4}) {
            if (KB_req > 0 ? !(kb_ok(r, KB_req) && K % KB_req == 0) : default_kb(r, K) == 0) continue;
            // lanes cut into pieces need one vehicle per thread
            if (r > 1 && need > 1024 * r) continue;
            sh.threads = 1024;
            sh.per_thread = r;
            for (int t : {64, 128, 256, 512, 1024}) {
                if ((int64_t)t * r >= need) {
                    sh.threads = t;
                    break;
                }
            }
            found = true;
            break;
        }
        if (!found)
            return fail(IDM_ERR_UNSUPPORTED,
                        "no launch shape for K=%d and a %d-vehicle lane: K needs a backward block "
                        "that divides it (8, 16 or 32 for lanes cut into pieces)",
                        K, p->max_lane);
    }
    const int KB = KB_req > 0 ? KB_req : default_kb(sh.per_thread, K);
    if (KB <= 0 || !kb_ok(sh.per_thread, KB) || K % KB != 0)
        return fail(IDM_ERR_UNSUPPORTED,
                    "checkpoint interval K=%d needs a backward block (8/16/32 for 1-2 vehicles per "
                    "thread, 4/8 for 4) that divides it; got block %d, per_thread %d",
                    K, KB_req, sh.per_thread);
    sh.K = K;
    sh.KB = KB;
    sh.grid = (tu && tu->grid > 0) ? tu->grid : 0;
    sh.stored = tu && tu->store_states == 1;  // 2: checkpoints until the autotuner chooses
    sh.tile = tu ? tu->tile_steps : 0;
    if (sh.tile < 0) return fail(IDM_ERR_INVALID_ARG, "tuning: tile_steps < 0");
    if (sh.tile > 0) {
        if (!sh.stored)
            return fail(IDM_ERR_UNSUPPORTED, "halo tiles (tile_steps %d) need store_states = 1",
                        sh.tile);
        if (!forward_tiled_kernel(p->pb.bound, tu->threads) || tu->per_thread != 1)
            return fail(IDM_ERR_UNSUPPORTED,
                        "halo tiles need threads of 256, 512, 576, 640, 768 or 1024 and "
                        "per_thread = 1 in the tuning; got %d x %d",
                        tu->threads, tu->per_thread);
        if (sh.tile >= sh.threads || sh.tile % 2 != 0 || sh.tile % K != 0)
            return fail(IDM_ERR_UNSUPPORTED,
                        "tile_steps %d must be even, a multiple of K = %d and below threads = %d",
                        sh.tile, K, sh.threads);
        if (sh.grid > 0)
            return fail(IDM_ERR_UNSUPPORTED, "halo tiles run one work-group per tile (grid 0)");
    }
    return IDM_OK;
}

SimArgs base_args(const idm_plan *p) {
    SimArgs a;
    memset(&a, 0, sizeof a);
    a.n = p->pb.n_vehicles;
    a.n_steps = p->pb.n_steps;
    a.K = p->sh.K;
    a.dt = p->pb.dt;
    a.inv_dt = 1.0f / p->pb.dt;
    a.a_min = p->pb.a_min;
    a.gap_floor = p->pb.gap_floor;
    a.slot_gidx = p->d_gidx;
    a.slot_flags = p->d_flags;
    a.n_bundles = p->n_bundles;
    a.zero = p->d_zero;
    return a;
}

idm_status check_params(const idm_params *prm) {
    if (!prm || !prm->v0 || !prm->T || !prm->a || !prm->b || !prm->s0 || !prm->length)
        return fail(IDM_ERR_INVALID_ARG, "params: null pointer");
    return IDM_OK;
}

idm_status check_obs(const idm_plan *p, const idm_obs *obs) {
    if (!obs) return IDM_OK;
    if (!obs->target) return fail(IDM_ERR_INVALID_ARG, "obs.target is null");
    if (obs->n_obs < 1 || obs->obs_first < 0 || obs->obs_stride < 1)
        return fail(IDM_ERR_INVALID_ARG, "obs: n_obs=%d first=%d stride=%d invalid", obs->n_obs,
                    obs->obs_first, obs->obs_stride);
    int64_t last = (int64_t)obs->obs_first + (int64_t)(obs->n_obs - 1) * obs->obs_stride;
    if (last > p->pb.n_steps)
        return fail(IDM_ERR_INVALID_ARG, "obs: last observed step %lld > n_steps %d", (long long)last,
                    p->pb.n_steps);
    return IDM_OK;
}

int grid_of(const idm_plan *p, int32_t n) { return p->sh.grid > 0 ? std::min(p->sh.grid, n) : n; }
int grid_of(const idm_plan *p) { return grid_of(p, p->n_bundles); }

int32_t n_levels(const idm_plan *p) { return (int32_t)p->level_start.size() - 1; }

// Launch level `lv`: its bundle tables (and the first of its loss partials
// or diagnostic counts); returns its bundle count.
int32_t level_args(const idm_plan *p, int32_t lv, SimArgs &a, double *loss_base,
                   uint64_t *diag_base = nullptr) {
    const int32_t b0 = p->level_start[lv], b1 = p->level_start[lv + 1];
    const int64_t cap = (int64_t)p->sh.threads * p->sh.per_thread;
    a.slot_gidx = p->d_gidx + b0 * cap;
    a.slot_flags = p->d_flags + b0 * cap;
    a.n_bundles = b1 - b0;
    if (p->d_bnd) {
        a.bnd_in = p->d_bnd + b0;
        a.bnd_out = p->d_bnd + p->n_bundles + b0;
    }
    if (loss_base) a.loss_part = loss_base + b0;
    if (diag_base) a.diag = diag_base + 2 * (int64_t)b0;
    return b1 - b0;
}

void ext_args(const idm_plan *p, void *ws, SimArgs &a) {
    if (p->n_bnd == 0) return;
    char *base = (char *)ws + ws_ext_off(p, dims_of(p));
    a.ext_state = (float2 *)base;
    a.ext_adj = (float2 *)(base + ext_state_bytes(p, p->n_bnd));
}

// Launches of a halo-tile plan: blocks of J steps, [j J, min((j + 1) J, S)),
// at least one (S = 0 writes the initial row).
int32_t tile_launches(const idm_plan *p) {
    const int32_t S = p->pb.n_steps, J = p->sh.tile;
    return S == 0 ? 1 : (S + J - 1) / J;
}

// Where a forward that keeps every step's states writes them: the
// workspace's rows, or with `direct` (forward + backward of one step, whose
// backward reads them where they are) the caller's trajectory outputs where
// given, which then need no copy.
void kept_rows(const idm_plan *p, void *ws, bool direct, float *&traj_d, float *&traj_v,
               float *&st_d, float *&st_v) {
    st_d = (float *)((char *)ws + ws_states_off(p));
    st_v = (float *)((char *)st_d + state_rows_bytes(p));
    if (!direct) return;
    if (traj_d) st_d = traj_d;
    if (traj_v) st_v = traj_v;
    traj_d = traj_v = nullptr;
}

// The halo-tile forward: every launch advances every tile J steps, reading
// the states its halo starts from in the rows the previous launch wrote.
idm_status run_forward_tiled(idm_plan *p, SimArgs a, float *traj_d, float *traj_v, void *ws,
                             hipStream_t s, bool direct) {
    float *st_d = nullptr, *st_v = nullptr;
    if (ws) {
        kept_rows(p, ws, direct, traj_d, traj_v, st_d, st_v);
    } else if (traj_d && traj_v) {
        st_d = traj_d;  // no workspace: the caller's rows hold the states
        st_v = traj_v;
        traj_d = traj_v = nullptr;
    } else {
        return fail(IDM_ERR_WORKSPACE,
                    "a halo-tile forward reads each launch's start states from the trajectory "
                    "rows: pass the workspace or both trajectory outputs");
    }
    a.traj_d = st_d;
    a.traj_v = st_v;
    a.ckpt = nullptr;
    a.diag = ws ? (uint64_t *)((char *)ws + ws_diag_off(p)) : nullptr;
    KernelFn fn = forward_tiled_kernel(p->pb.bound, p->sh.threads);
    if (!fn) return fail(IDM_ERR_UNSUPPORTED, "no halo-tile forward for %d threads", p->sh.threads);
    const int32_t S = p->pb.n_steps, J = p->sh.tile;
    for (int32_t j = 0; j < tile_launches(p); ++j) {
        a.k_lo = j * J;
        a.k_hi = std::min(S, (j + 1) * J);
        hipError_t e = launch_sim(fn, p->n_tiles, p->sh.threads, a, s);
        if (e != hipSuccess) return hip_fail(e, "halo-tile forward launch");
    }
    const size_t rows = ((size_t)S + 1) * sizeof(float) * (size_t)p->pb.n_vehicles;
    for (int i = 0; i < 2; ++i) {
        float *dst = i ? traj_v : traj_d;
        const float *src = i ? st_v : st_d;
        if (!dst || rows == 0) continue;
        hipError_t e = hipMemcpyAsync(dst, src, rows, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "trajectory copy");
    }
    return IDM_OK;
}

idm_status run_forward(idm_plan *p, const idm_params *prm, const double *p0, const float *v_init,
                       float *traj_d, float *traj_v, void *ws, hipStream_t s,
                       bool direct = false) {
    SimArgs a = base_args(p);
    a.v0 = prm->v0; a.T = prm->T; a.a = prm->a; a.b = prm->b; a.s0 = prm->s0; a.len = prm->length;
    a.p0 = p0;
    a.v_init = v_init;
    if (p->sh.tile > 0) return run_forward_tiled(p, a, traj_d, traj_v, ws, s, direct);
    a.traj_d = traj_d;
    a.traj_v = traj_v;
    a.ckpt = ws ? (float *)((char *)ws + ws_ckpt_off(p)) : nullptr;
    if (p->pb.n_steps == 0 && a.ckpt) a.ckpt = nullptr;
    // a plan that keeps every step's states writes them into the workspace
    // (no checkpoints) and copies them out for a caller that asked for them
    float *st_d = nullptr, *st_v = nullptr;
    if (p->sh.stored && ws) {
        kept_rows(p, ws, direct, traj_d, traj_v, st_d, st_v);
        a.traj_d = st_d;
        a.traj_v = st_v;
        a.ckpt = nullptr;
    }
    if (p->n_bnd > 0) {
        if (!ws)
            return fail(IDM_ERR_WORKSPACE,
                        "lanes longer than a bundle exchange boundary states through the "
                        "workspace; the forward needs it");
        ext_args(p, ws, a);
    }
    // bundle-edge waves store through the cache when both rows are written by
    // a launch that fills the chip (there the half-written boundary lines of
    // streamed stores cost HBM write rate); a launch of few work-groups is
    // bound by each step's latency, which streamed stores keep lower
    const bool edge_cached = a.traj_d && a.traj_v && p->n_bundles >= kRoundCUs;
    KernelFn fn = forward_kernel(p->pb.bound, p->sh.per_thread, p->sh.threads, p->n_bnd > 0,
                                 edge_cached);
    if (!fn) return fail(IDM_ERR_UNSUPPORTED, "no forward kernel for this shape");
    uint64_t *diag = ws ? (uint64_t *)((char *)ws + ws_diag_off(p)) : nullptr;
    // pieces of long lanes: level l reads the boundary states level l-1 wrote
    for (int32_t lv = 0; lv < n_levels(p); ++lv) {
        const int32_t nb = level_args(p, lv, a, nullptr, diag);
        if (nb == 0) continue;
        hipError_t e = launch_sim(fn, grid_of(p, nb), p->sh.threads, a, s);
        if (e != hipSuccess) return hip_fail(e, "forward launch");
    }
    const size_t rows = ((size_t)p->pb.n_steps + 1) * sizeof(float) * (size_t)p->pb.n_vehicles;
    for (int i = 0; i < 2; ++i) {
        float *dst = i ? traj_v : traj_d;
        const float *src = i ? st_v : st_d;
        if (!src || !dst || rows == 0) continue;
        hipError_t e = hipMemcpyAsync(dst, src, rows, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "trajectory copy");
    }
    return IDM_OK;
}

idm_status run_backward_stored(idm_plan *p, const idm_params *prm, const double *p0,
                               const float *traj_d, const float *traj_v, const float *gd,
                               const float *gv, const idm_obs *obs, double *g_prm,
                               double *g_p0, double *g_v0, double *loss_out, void *ws,
                               hipStream_t s);

idm_status run_backward(idm_plan *p, const idm_params *prm, const double *p0, const float *v_init,
                        const float *gd, const float *gv, const idm_obs *obs, double *g_prm,
                        double *g_p0, double *g_v0, double *loss_out, void *ws, hipStream_t s) {
    if (p->sh.stored) {
        // the states the forward kept in the workspace
        const float *st_d = (const float *)((char *)ws + ws_states_off(p));
        const float *st_v = (const float *)((const char *)st_d + state_rows_bytes(p));
        return run_backward_stored(p, prm, p0, st_d, st_v, gd, gv, obs, g_prm, g_p0, g_v0,
                                   loss_out, ws, s);
    }
    SimArgs a = base_args(p);
    a.v0 = prm->v0; a.T = prm->T; a.a = prm->a; a.b = prm->b; a.s0 = prm->s0; a.len = prm->length;
    a.p0 = p0;
    a.v_init = v_init;
    a.ckpt = (float *)((char *)ws + ws_ckpt_off(p));
    a.gd = gd;
    a.gv = gv;
    if (obs) {
        a.target = obs->target;
        a.n_obs = obs->n_obs;
        a.obs_first = obs->obs_first;
        a.obs_stride = obs->obs_stride;
        a.inv_count = 1.0 / ((double)obs->n_obs * (double)p->pb.n_vehicles);
        a.two_inv_count = 2.0 * a.inv_count;
    } else {
        a.obs_stride = 1;
    }
    a.g_prm = g_prm;
    a.g_p0 = g_p0;
    a.g_v0 = g_v0;
    double *loss_base = (double *)((char *)ws + ws_loss_off(p));
    ext_args(p, ws, a);
    KernelFn fn = backward_kernel(p->pb.bound, p->sh.per_thread, p->sh.threads, p->sh.KB, p->sh.K,
                                  gd || gv, p->n_bnd > 0);
    if (!fn) return fail(IDM_ERR_UNSUPPORTED, "no backward kernel for this shape");
    // pieces of long lanes: level l reads the adjoint contributions level l+1 wrote
    for (int32_t lv = n_levels(p) - 1; lv >= 0; --lv) {
        const int32_t nb = level_args(p, lv, a, loss_base);
        if (nb == 0) continue;
        hipError_t e = launch_sim(fn, grid_of(p, nb), p->sh.threads, a, s);
        if (e != hipSuccess) return hip_fail(e, "backward launch");
    }
    if (loss_out) {
        hipError_t e = launch_loss_finalize(loss_base, p->n_bundles, obs ? a.inv_count : 0.0,
                                            loss_out, s);
        if (e != hipSuccess) return hip_fail(e, "loss finalize launch");
    }
    return IDM_OK;
}

// The adjoint from the forward's stored trajectory (whole lanes: one launch
// level).  The workspace holds the loss partials only.
idm_status run_backward_stored(idm_plan *p, const idm_params *prm, const double *p0,
                               const float *traj_d, const float *traj_v, const float *gd,
                               const float *gv, const idm_obs *obs, double *g_prm,
                               double *g_p0, double *g_v0, double *loss_out, void *ws,
                               hipStream_t s) {
    if (p->n_bnd > 0 || n_levels(p) != 1)
        return fail(IDM_ERR_UNSUPPORTED,
                    "the backward from stored states handles whole lanes only; this plan cuts "
                    "lanes longer than a bundle into pieces (use idm_sim_backward)");
    SimArgs a = base_args(p);
    a.v0 = prm->v0; a.T = prm->T; a.a = prm->a; a.b = prm->b; a.s0 = prm->s0; a.len = prm->length;
    a.p0 = p0;
    a.traj_d = const_cast<float *>(traj_d);
    a.traj_v = const_cast<float *>(traj_v);
    a.gd = gd;
    a.gv = gv;
    if (obs) {
        a.target = obs->target;
        a.n_obs = obs->n_obs;
        a.obs_first = obs->obs_first;
        a.obs_stride = obs->obs_stride;
        a.inv_count = 1.0 / ((double)obs->n_obs * (double)p->pb.n_vehicles);
        a.two_inv_count = 2.0 * a.inv_count;
    } else {
        a.obs_stride = 1;
    }
    a.g_prm = g_prm;
    a.g_p0 = g_p0;
    a.g_v0 = g_v0;
    double *loss_base = (double *)((char *)ws + ws_loss_off(p));
    if (p->sh.tile > 0) {
        // halo tiles: blocks of J steps from the last to the first, the
        // adjoints carried between launches through two alternating buffers
        KernelFn fn = backward_tiled_kernel(p->pb.bound, p->sh.threads, gd || gv);
        if (!fn)
            return fail(IDM_ERR_UNSUPPORTED, "no halo-tile backward for %d threads", p->sh.threads);
        char *tb = (char *)ws + ws_tile_off(p, dims_of(p));
        float *carry[2] = {(float *)tb, (float *)(tb + tile_carry_bytes(p))};
        a.t_gp0 = (float *)(tb + 2 * tile_carry_bytes(p));
        a.t_acc = (double *)(tb + 2 * tile_carry_bytes(p) + tile_gp0_bytes(p));
        const int64_t cap = (int64_t)p->sh.threads;
        a.slot_gidx = p->d_gidx + (int64_t)p->n_tiles * cap;  // the backward tables
        a.slot_flags = p->d_flags + (int64_t)p->n_tiles * cap;
        a.n_bundles = p->n_tiles;
        a.loss_part = loss_base;
        const int32_t S = p->pb.n_steps, J = p->sh.tile, nl = tile_launches(p);
        for (int32_t i = 0; i < nl; ++i) {
            const int32_t j = nl - 1 - i;
            a.k_lo = j * J;
            a.k_hi = std::min(S, (j + 1) * J);
            a.tc_in = carry[i & 1];
            a.tc_out = carry[(i + 1) & 1];
            hipError_t e = launch_sim(fn, p->n_tiles, p->sh.threads, a, s);
            if (e != hipSuccess) return hip_fail(e, "halo-tile backward launch");
        }
        if (loss_out) {
            hipError_t e = launch_loss_finalize(loss_base, p->n_tiles, obs ? a.inv_count : 0.0,
                                                loss_out, s);
            if (e != hipSuccess) return hip_fail(e, "loss finalize launch");
        }
        return IDM_OK;
    }
    KernelFn fn = backward_stored_kernel(p->pb.bound, p->sh.per_thread, p->sh.threads, gd || gv);
    if (!fn) return fail(IDM_ERR_UNSUPPORTED, "no stored-state backward kernel for this shape");
    const int32_t nb = level_args(p, 0, a, loss_base);
    if (nb > 0) {
        hipError_t e = launch_sim(fn, grid_of(p, nb), p->sh.threads, a, s);
        if (e != hipSuccess) return hip_fail(e, "stored-state backward launch");
    }
    if (loss_out) {
        hipError_t e = launch_loss_finalize(loss_base, p->n_bundles, obs ? a.inv_count : 0.0,
                                            loss_out, s);
        if (e != hipSuccess) return hip_fail(e, "loss finalize launch");
    }
    return IDM_OK;
}

AdamArgs adam_args(const idm_plan *p, const idm_fit_state *st, const double *grad) {
    AdamArgs a;
    memset(&a, 0, sizeof a);
    a.n = p->pb.n_vehicles;
    a.u = st->u;
    a.m = st->m;
    a.v = st->v;
    a.params = st->params;
    a.grad = grad;
    a.step = st->step;
    a.step_rw = st->step;
    for (int i = 0; i < 5; ++i) {
        a.lo[i] = st->lo[i];
        a.hi[i] = st->hi[i];
    }
    a.lr0 = st->lr0;
    a.lr1 = st->lr1;
    a.lr_steps = st->lr_steps;
    a.beta1 = st->beta1;
    a.beta2 = st->beta2;
    a.eps = st->eps;
    a.raw = st->raw_units ? 1 : 0;
    return a;
}

idm_status check_fit(const idm_plan *p, const idm_fit_state *st, const double *p0,
                     const float *v_init, const idm_obs *obs, void *ws) {
    if (!st || !st->u || !st->m || !st->v || !st->params || !st->length || !st->step ||
        !st->loss_hist)
        return fail(IDM_ERR_INVALID_ARG, "fit state: null pointer");
    if (st->hist_len < 1 || st->lr_steps < 1)
        return fail(IDM_ERR_INVALID_ARG, "fit state: hist_len and lr_steps must be >= 1");
    for (int i = 0; i < 5; ++i)
        if (!(st->hi[i] > st->lo[i]) || !std::isfinite(st->lo[i]) || !std::isfinite(st->hi[i]))
            return fail(IDM_ERR_INVALID_ARG, "fit state: box %d invalid", i);
    if (!(st->beta1 >= 0 && st->beta1 < 1 && st->beta2 >= 0 && st->beta2 < 1 && st->eps > 0) ||
        !std::isfinite(st->lr0) || !std::isfinite(st->lr1))
        return fail(IDM_ERR_INVALID_ARG, "fit state: Adam hyper-parameters invalid");
    if (!p0 || !v_init) return fail(IDM_ERR_INVALID_ARG, "p0 / v_init null");
    if (!obs) return fail(IDM_ERR_INVALID_ARG, "fit needs observations");
    if (!ws) return fail(IDM_ERR_WORKSPACE, "workspace is null");
    return check_obs(p, obs);
}

idm_status run_fit_step(idm_plan *p, const idm_fit_state *st, const double *p0, const float *v_init,
                        const idm_obs *obs, void *ws, hipStream_t s) {
    const int64_t N = p->pb.n_vehicles;
    idm_params prm;
    prm.v0 = st->params;
    prm.T = st->params + N;
    prm.a = st->params + 2 * N;
    prm.b = st->params + 3 * N;
    prm.s0 = st->params + 4 * N;
    prm.length = st->length;
    double *grad = (double *)((char *)ws + ws_fit_off(p));
    double *gp0 = grad + 5 * N, *gv0 = grad + 6 * N;
    idm_status r = run_forward(p, &prm, p0, v_init, nullptr, nullptr, ws, s);
    if (r != IDM_OK) return r;
    r = run_backward(p, &prm, p0, v_init, nullptr, nullptr, obs, grad, gp0, gv0, nullptr, ws, s);
    if (r != IDM_OK) return r;
    double scale = 1.0 / ((double)obs->n_obs * (double)N);
    hipError_t e = launch_fit_finalize((double *)((char *)ws + ws_loss_off(p)), p->n_bundles, scale,
                                       st->step, st->loss_hist, st->hist_len, s);
    if (e != hipSuccess) return hip_fail(e, "fit finalize launch");
    AdamArgs aa = adam_args(p, st, grad);
    e = launch_adam(aa, s);
    if (e != hipSuccess) return hip_fail(e, "adam launch");
    return IDM_OK;
}

idm_status run_step(idm_plan *p, const idm_step_args *a, hipStream_t s) {
    // a plan that keeps states writes them straight into the trajectory
    // outputs the caller asked for, and the backward reads them there
    idm_status r = run_forward(p, &a->prm, a->p0, a->v_init, a->traj_d, a->traj_v, a->workspace,
                               s, true);
    if (r != IDM_OK) return r;
    idm_obs obs{a->obs_target, a->n_obs, a->obs_first, a->obs_stride};
    if (p->sh.stored) {
        float *td = a->traj_d, *tv = a->traj_v, *st_d = nullptr, *st_v = nullptr;
        kept_rows(p, a->workspace, true, td, tv, st_d, st_v);
        return run_backward_stored(p, &a->prm, a->p0, st_d, st_v, a->grad_traj_d, a->grad_traj_v,
                                   a->obs_target ? &obs : nullptr, a->grad_params, a->grad_p0,
                                   a->grad_v0, a->loss_out, a->workspace, s);
    }
    return run_backward(p, &a->prm, a->p0, a->v_init, a->grad_traj_d, a->grad_traj_v,
                        a->obs_target ? &obs : nullptr, a->grad_params, a->grad_p0, a->grad_v0,
                        a->loss_out, a->workspace, s);
}

idm_status check_step(const idm_plan *p, const idm_step_args *a) {
    if (!a) return fail(IDM_ERR_INVALID_ARG, "args is null");
    idm_status r = check_params(&a->prm);
    if (r != IDM_OK) return r;
    if (!a->p0 || !a->v_init) return fail(IDM_ERR_INVALID_ARG, "p0 / v_init null");
    if (!a->grad_params || !a->grad_p0 || !a->grad_v0)
        return fail(IDM_ERR_INVALID_ARG, "gradient outputs null");
    if (!a->workspace) return fail(IDM_ERR_WORKSPACE, "workspace is null");
    if (a->obs_target) {
        idm_obs obs{a->obs_target, a->n_obs, a->obs_first, a->obs_stride};
        return check_obs(p, &obs);
    }
    return IDM_OK;
}

// Capture `fn` (which launches on the given stream) into a graph.
template <class F>
idm_status capture(hipStream_t s, hipGraphExec_t *out, F fn) {
    if (!s) return fail(IDM_ERR_INVALID_ARG, "graph capture needs a non-default stream");
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    idm_status r = fn();
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s, &g);
    if (r != IDM_OK) {
        if (g) hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    *out = ex;
    return IDM_OK;
}

// Validation of the problem and choice of the launch shape (host only).
idm_status host_plan(const idm_problem *pb, const idm_tuning *tu, idm_plan *p, Shape &sh) {
    if (!pb) return fail(IDM_ERR_INVALID_ARG, "null argument");
    if (pb->n_vehicles < 1 || pb->n_lanes < 1 || pb->n_steps < 0 || pb->n_steps > IDM_MAX_STEPS)
        return fail(IDM_ERR_INVALID_ARG, "sizes: N=%d L=%d S=%d (S <= %d)", pb->n_vehicles,
                    pb->n_lanes, pb->n_steps, IDM_MAX_STEPS);
    // a per-step row of N floats is addressed with 32-bit buffer offsets
    if (pb->n_vehicles > IDM_MAX_VEHICLES)
        return fail(IDM_ERR_INVALID_ARG, "N=%d exceeds %d vehicles", pb->n_vehicles,
                    IDM_MAX_VEHICLES);
    if (!(pb->dt > 0.0f) || !std::isfinite(pb->dt))
        return fail(IDM_ERR_INVALID_ARG, "dt must be positive and finite");
    if (!std::isfinite(pb->a_min) || !(pb->a_min < 0.0f))
        return fail(IDM_ERR_INVALID_ARG, "a_min must be negative and finite");
    if (!(pb->gap_floor >= 0.0f) || !std::isfinite(pb->gap_floor))
        return fail(IDM_ERR_INVALID_ARG, "gap_floor must be >= 0");
    if (pb->delta != 4.0f)
        return fail(IDM_ERR_UNSUPPORTED, "delta=%g: only delta = 4 is implemented", pb->delta);
    if (pb->bound != IDM_BOUND_SOFTPLUS && pb->bound != IDM_BOUND_CLAMP)
        return fail(IDM_ERR_INVALID_ARG, "bound must be IDM_BOUND_SOFTPLUS or IDM_BOUND_CLAMP");
    if (pb->ckpt_every < 0) return fail(IDM_ERR_INVALID_ARG, "ckpt_every < 0");
    if (!pb->lane_offsets_host) return fail(IDM_ERR_INVALID_ARG, "lane_offsets_host is null");
    const int32_t *off = pb->lane_offsets_host;
    if (off[0] != 0 || off[pb->n_lanes] != pb->n_vehicles)
        return fail(IDM_ERR_LAYOUT, "lane offsets must start at 0 and end at N");
    int32_t max_lane = 0;
    for (int l = 0; l < pb->n_lanes; ++l) {
        if (off[l + 1] < off[l]) return fail(IDM_ERR_LAYOUT, "lane offsets decrease at lane %d", l);
        max_lane = std::max(max_lane, off[l + 1] - off[l]);
    }
    if (tu && (tu->grid < 0 || tu->ckpt_every < 0 || tu->block < 0))
        return fail(IDM_ERR_INVALID_ARG, "tuning: negative grid, ckpt_every or block");
    if (tu && (tu->store_states < 0 || tu->store_states > 2))
        return fail(IDM_ERR_INVALID_ARG, "tuning: store_states must be 0, 1 or 2");
    p->pb = *pb;
    p->offsets.assign(off, off + pb->n_lanes + 1);
    p->pb.lane_offsets_host = nullptr;
    p->max_lane = max_lane;
    p->store_pref = tu ? tu->store_states : 0;
    return choose_shape(p, tu, sh);
}

// The stream graph work runs on: the caller's, or the side stream for the
// null stream (made to wait for the null stream's prior work).
template <class PL>
idm_status graph_stream_enter(PL *p, hipStream_t caller, hipStream_t *out) {
    if (caller) {
        *out = caller;
        return IDM_OK;
    }
    hipError_t e = hipSuccess;
    if (!p->side) {
        e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "side stream creation");
    }
    e = hipEventRecord(p->ev_in, nullptr);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->ev_in, 0);
    if (e != hipSuccess) return hip_fail(e, "side stream join");
    *out = p->side;
    return IDM_OK;
}

// Make the null stream wait for the side stream's graph work.
template <class PL>
idm_status graph_stream_leave(PL *p, hipStream_t caller) {
    if (caller) return IDM_OK;
    hipError_t e = hipEventRecord(p->ev_out, p->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(nullptr, p->ev_out, 0);
    if (e != hipSuccess) return hip_fail(e, "side stream join");
    return IDM_OK;
}

}  // namespace

namespace idmx {
idm_status set_error(idm_status st, const char *msg) { return fail(st, "%s", msg); }
const uint8_t *plan_head_flags(const idm_plan *p) { return p ? p->d_head : nullptr; }
int64_t plan_vehicles(const idm_plan *p) { return p ? p->pb.n_vehicles : 0; }
int32_t plan_steps(const idm_plan *p) { return p ? p->pb.n_steps : 0; }
float plan_dt(const idm_plan *p) { return p ? p->pb.dt : 0.0f; }
}  // namespace idmx

namespace {

// Autotuner cache: the shape chosen for a problem signature, kept for the
// process.  The signature is the sorted lane sizes (the lane-size histogram)
// followed by S, the bound mode, a fixed K (0 = free), the kind of upstream
// gradient and the device's compute-unit count, compared in full.
std::mutex g_tune_mu;
std::map<std::vector<int64_t>, Shape> g_tune_cache;

std::vector<int64_t> tune_key(const idm_plan *p, bool dense, bool obs, int cus) {
    std::vector<int64_t> k((size_t)p->pb.n_lanes);
    for (int l = 0; l < p->pb.n_lanes; ++l) k[(size_t)l] = p->offsets[l + 1] - p->offsets[l];
    std::sort(k.begin(), k.end());
    k.push_back(p->pb.n_steps);
    k.push_back((int64_t)p->pb.bound);
    k.push_back(p->pb.ckpt_every);
    k.push_back(dense ? 1 : 0);
    k.push_back(obs ? 1 : 0);
    k.push_back(cus);
    k.push_back(p->store_pref);
    return k;
}

// Device address of the current GPU's copy of `scratch`, looked up once per
// device (hipGetSymbolAddress, with that device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

idm_status static_scratch(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(IDM_ERR_UNSUPPORTED, "device index %d", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(IDM_ERR_HIP, "hipGetSymbolAddress(scratch) gave no address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return IDM_OK;
}

}  // namespace

extern "C" {

const char *idm_last_error(void) { return g_err.c_str(); }

const char *idm_version(void) { return "idmx 0.1 gfx950"; }

idm_status idm_copy_bytes(void *dst, const void *src, size_t bytes, void *stream) {
    if (!dst || !src) return fail(IDM_ERR_INVALID_ARG, "null pointer");
    if (bytes % 16 || ((uintptr_t)dst % 16) || ((uintptr_t)src % 16))
        return fail(IDM_ERR_INVALID_ARG, "copy needs 16-byte aligned pointers and sizes");
    if (bytes == 0) return IDM_OK;
    int64_t n16 = (int64_t)(bytes / 16);
    int64_t g = (n16 + 1023) / 1024;  // chunks of 1024 16-byte words per work-group
    int grid = (int)std::min<int64_t>(g, 256 * 16);
    hipError_t e = launch_copy(src, dst, n16, grid, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "copy launch");
    return IDM_OK;
}

idm_status idm_plan_create(const idm_problem *pb, const idm_tuning *tu, idm_plan **out) {
    if (!out) return fail(IDM_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    idm_plan *p = new idm_plan();
    Shape sh;
    idm_status r = host_plan(pb, tu, p, sh);
    if (r == IDM_OK) r = build_layout(p, sh);
    if (r != IDM_OK) {
        idm_plan_destroy(p);
        return r;
    }
    *out = p;
    return IDM_OK;
}

idm_status idm_problem_check(const idm_problem *pb, const idm_tuning *tu, idm_plan_info *info,
                             size_t *workspace_bytes) {
    idm_plan p;
    Shape sh;
    idm_status r = host_plan(pb, tu, &p, sh);
    if (r != IDM_OK) return r;
    Layout lay;
    r = compute_layout(p.offsets, p.pb.n_lanes, sh, lay);
    if (r != IDM_OK) return r;
    p.sh = sh;
    p.n_bundles = (int32_t)lay.n_bundles;
    p.n_slots = lay.n_bundles * lay.cap;
    p.n_bnd = lay.n_bnd;
    p.level_start = lay.level_start;
    if (p.sh.grid > p.n_bundles) p.sh.grid = p.n_bundles;
    p.n_tiles = sh.tile > 0 ? p.n_bundles : 0;
    if (workspace_bytes) *workspace_bytes = ws_total(&p);
    if (info) return idm_plan_get_info(&p, info);
    return IDM_OK;
}

idm_status idm_problem_layout(const idm_problem *pb, const idm_tuning *tu, int32_t *slot_vehicle_host,
                              uint8_t *slot_flags_host, int64_t capacity) {
    if (!slot_vehicle_host || !slot_flags_host) return fail(IDM_ERR_INVALID_ARG, "null output");
    idm_plan p;
    Shape sh;
    idm_status r = host_plan(pb, tu, &p, sh);
    if (r != IDM_OK) return r;
    Layout lay;
    r = compute_layout(p.offsets, p.pb.n_lanes, sh, lay);
    if (r != IDM_OK) return r;
    if ((int64_t)lay.gidx.size() > capacity)
        return fail(IDM_ERR_INVALID_ARG, "capacity %lld < %lld slots", (long long)capacity,
                    (long long)lay.gidx.size());
    std::copy(lay.gidx.begin(), lay.gidx.end(), slot_vehicle_host);
    std::copy(lay.flags.begin(), lay.flags.end(), slot_flags_host);
    return IDM_OK;
}

idm_status idm_problem_bundles(const idm_problem *pb, const idm_tuning *tu, int32_t *bnd_in_host,
                               int32_t *bnd_out_host, int32_t *level_host, int64_t capacity) {
    if (!bnd_in_host || !bnd_out_host || !level_host)
        return fail(IDM_ERR_INVALID_ARG, "null output");
    idm_plan p;
    Shape sh;
    idm_status r = host_plan(pb, tu, &p, sh);
    if (r != IDM_OK) return r;
    Layout lay;
    r = compute_layout(p.offsets, p.pb.n_lanes, sh, lay);
    if (r != IDM_OK) return r;
    if (lay.n_bundles > capacity)
        return fail(IDM_ERR_INVALID_ARG, "capacity %lld < %lld bundles", (long long)capacity,
                    (long long)lay.n_bundles);
    std::copy(lay.bnd_in.begin(), lay.bnd_in.end(), bnd_in_host);
    std::copy(lay.bnd_out.begin(), lay.bnd_out.end(), bnd_out_host);
    std::copy(lay.level.begin(), lay.level.end(), level_host);
    return IDM_OK;
}

idm_status idm_plan_destroy(idm_plan *p) {
    if (!p) return IDM_OK;
    drop_graphs(p);
    if (p->d_gidx) hipFree(p->d_gidx);
    if (p->d_flags) hipFree(p->d_flags);
    if (p->d_bnd) hipFree(p->d_bnd);
    if (p->d_zero) hipFree(p->d_zero);
    if (p->d_head) hipFree(p->d_head);
    if (p->d_lane_off) hipFree(p->d_lane_off);
    if (p->d_lane_of) hipFree(p->d_lane_of);
    if (p->side) hipStreamDestroy(p->side);
    if (p->ev_in) hipEventDestroy(p->ev_in);
    if (p->ev_out) hipEventDestroy(p->ev_out);
    delete p;
    return IDM_OK;
}

size_t idm_workspace_bytes(const idm_plan *p) { return p ? ws_total(p) : 0; }

idm_status idm_plan_get_info(const idm_plan *p, idm_plan_info *o) {
    if (!p || !o) return fail(IDM_ERR_INVALID_ARG, "null argument");
    o->threads = p->sh.threads;
    o->per_thread = p->sh.per_thread;
    o->ckpt_every = p->sh.K;
    o->block = p->sh.KB;
    o->grid = grid_of(p);
    o->n_bundles = p->n_bundles;
    o->max_lane = p->max_lane;
    o->n_slots = p->n_slots;
    o->fill = p->n_slots ? (double)p->pb.n_vehicles / (double)p->n_slots : 0.0;
    o->n_levels = n_levels(p);
    o->n_boundaries = p->n_bnd;
    o->autotune_cached = p->tuned_cached;
    o->store_states = p->sh.stored ? 1 : 0;
    o->tile_steps = p->sh.tile;
    return IDM_OK;
}

idm_status idm_sim_forward(idm_plan *p, const idm_params *prm, const double *p0, const float *v_init,
                           float *traj_d, float *traj_v, void *ws, void *stream) {
    if (!p) return fail(IDM_ERR_INVALID_ARG, "plan is null");
    idm_status r = check_params(prm);
    if (r != IDM_OK) return r;
    if (!p0 || !v_init) return fail(IDM_ERR_INVALID_ARG, "p0 / v_init null");
    return run_forward(p, prm, p0, v_init, traj_d, traj_v, ws, (hipStream_t)stream);
}

idm_status idm_plan_diagnostics(idm_plan *p, const void *ws, int64_t *counts_out, void *stream) {
    if (!p) return fail(IDM_ERR_INVALID_ARG, "plan is null");
    if (!ws) return fail(IDM_ERR_WORKSPACE, "workspace is null");
    if (!counts_out) return fail(IDM_ERR_INVALID_ARG, "counts_out is null");
    hipError_t e = launch_diag_finalize((const uint64_t *)((const char *)ws + ws_diag_off(p)),
                                        p->n_bundles, counts_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "diagnostics launch");
    return IDM_OK;
}

idm_status idm_sim_backward(idm_plan *p, const idm_params *prm, const double *p0,
                            const float *v_init, const float *gd, const float *gv,
                            const idm_obs *obs, double *g_prm, double *g_p0, double *g_v0,
                            double *loss_out, void *ws, void *stream) {
    if (!p) return fail(IDM_ERR_INVALID_ARG, "plan is null");
    idm_status r = check_params(prm);
    if (r != IDM_OK) return r;
    if (!p0 || !v_init) return fail(IDM_ERR_INVALID_ARG, "p0 / v_init null");
    if (!g_prm || !g_p0 || !g_v0) return fail(IDM_ERR_INVALID_ARG, "gradient outputs null");
    if (!ws) return fail(IDM_ERR_WORKSPACE, "workspace is null");
    r = check_obs(p, obs);
    if (r != IDM_OK) return r;
    return run_backward(p, prm, p0, v_init, gd, gv, obs, g_prm, g_p0, g_v0, loss_out, ws,
                        (hipStream_t)stream);
}

idm_status idm_sim_backward_stored(idm_plan *p, const idm_params *prm, const double *p0,
                                   const float *traj_d, const float *traj_v, const float *gd,
                                   const float *gv, const idm_obs *obs, double *g_prm,
                                   double *g_p0, double *g_v0, double *loss_out, void *ws,
                                   void *stream) {
    if (!p) return fail(IDM_ERR_INVALID_ARG, "plan is null");
    idm_status r = check_params(prm);
    if (r != IDM_OK) return r;
    if (!p0) return fail(IDM_ERR_INVALID_ARG, "p0 null");
    if (!traj_d || !traj_v)
        return fail(IDM_ERR_INVALID_ARG, "traj_d / traj_v null: the stored trajectory is required");
    if (!g_prm || !g_p0 || !g_v0) return fail(IDM_ERR_INVALID_ARG, "gradient outputs null");
    if (!ws) return fail(IDM_ERR_WORKSPACE, "workspace is null");
    r = check_obs(p, obs);
    if (r != IDM_OK) return r;
    return run_backward_stored(p, prm, p0, traj_d, traj_v, gd, gv, obs, g_prm, g_p0, g_v0,
                               loss_out, ws, (hipStream_t)stream);
}

idm_status idm_sim_backward_noalloc(idm_plan *p, const idm_params *prm, const double *p0,
                                    const float *v_init, const float *gd, const float *gv,
                                    const idm_obs *obs, double *g_prm, double *g_p0,
                                    double *g_v0, double *loss_out, void *stream) {
    if (!p) return fail(IDM_ERR_INVALID_ARG, "plan is null");
    idm_status r = check_params(prm);
    if (r != IDM_OK) return r;
    if (!p0 || !v_init) return fail(IDM_ERR_INVALID_ARG, "p0 / v_init null");
    if (!g_prm || !g_p0 || !g_v0) return fail(IDM_ERR_INVALID_ARG, "gradient outputs null");
    r = check_obs(p, obs);
    if (r != IDM_OK) return r;
    const size_t need = ws_total(p);
    if (need > IDM_STATIC_SCRATCH_BYTES)
        return fail(IDM_ERR_WORKSPACE,
                    "the problem needs a %zu-byte workspace; the static scratch holds %zu bytes "
                    "(use idm_sim_forward / idm_sim_backward with a caller workspace)",
                    need, (size_t)IDM_STATIC_SCRATCH_BYTES);
    void *ws = nullptr;
    r = static_scratch(&ws);
    if (r != IDM_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    r = run_forward(p, prm, p0, v_init, nullptr, nullptr, ws, s);
    if (r != IDM_OK) return r;
    return run_backward(p, prm, p0, v_init, gd, gv, obs, g_prm, g_p0, g_v0, loss_out, ws, s);
}

idm_status idm_fit_init(idm_plan *p, const idm_fit_state *st, const float *init_params,
                        void *stream) {
    if (!p) return fail(IDM_ERR_INVALID_ARG, "plan is null");
    if (!init_params) return fail(IDM_ERR_INVALID_ARG, "init_params is null");
    if (!st || !st->u || !st->m || !st->v || !st->params || !st->step)
        return fail(IDM_ERR_INVALID_ARG, "fit state: null pointer");
    for (int i = 0; i < 5; ++i)
        if (!(st->hi[i] > st->lo[i]) || !std::isfinite(st->lo[i]) || !std::isfinite(st->hi[i]))
            return fail(IDM_ERR_INVALID_ARG, "fit state: box %d invalid", i);
    AdamArgs aa = adam_args(p, st, nullptr);
    hipError_t e = launch_fit_init(aa, init_params, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fit init launch");
    return IDM_OK;
}

idm_status idm_fit_init_normalized(idm_plan *p, const idm_fit_state *st, const float *u_rows,
                                   int32_t ld, void *stream) {
    if (!p) return fail(IDM_ERR_INVALID_ARG, "plan is null");
    if (!u_rows || ld < 5) return fail(IDM_ERR_INVALID_ARG, "u_rows null or ld < 5");
    if (!st || !st->u || !st->m || !st->v || !st->params || !st->step)
        return fail(IDM_ERR_INVALID_ARG, "fit state: null pointer");
    for (int i = 0; i < 5; ++i)
        if (!(st->hi[i] > st->lo[i]) || !std::isfinite(st->lo[i]) || !std::isfinite(st->hi[i]))
            return fail(IDM_ERR_INVALID_ARG, "fit state: box %d invalid", i);
    AdamArgs aa = adam_args(p, st, nullptr);
    hipError_t e = launch_fit_init_u(aa, u_rows, ld, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fit init launch");
    return IDM_OK;
}

idm_status idm_observe(idm_plan *p, const float *traj_d, const double *p0, const float *noise,
                       int32_t n_obs, int32_t obs_first, int32_t obs_stride, float *target_out,
                       void *stream) {
    if (!p || !traj_d || !p0 || !target_out) return fail(IDM_ERR_INVALID_ARG, "null argument");
    idm_obs o{target_out, n_obs, obs_first, obs_stride};
    idm_status r = check_obs(p, &o);
    if (r != IDM_OK) return r;
    hipError_t e = launch_observe(traj_d, p0, noise, n_obs, obs_first, obs_stride,
                                  p->pb.n_vehicles, target_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "observe launch");
    return IDM_OK;
}

idm_status idm_lane_loss(idm_plan *p, const float *traj_d, const double *p0, const idm_obs *obs,
                         double *lane_loss, void *stream) {
    if (!p || !traj_d || !p0 || !lane_loss) return fail(IDM_ERR_INVALID_ARG, "null argument");
    if (!obs) return fail(IDM_ERR_INVALID_ARG, "obs is null");
    idm_status r = check_obs(p, obs);
    if (r != IDM_OK) return r;
    hipError_t e = launch_lane_loss(traj_d, p0, obs->target, obs->n_obs, obs->obs_first,
                                    obs->obs_stride, p->pb.n_vehicles, p->d_lane_off,
                                    p->pb.n_lanes, lane_loss, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lane loss launch");
    return IDM_OK;
}

idm_status idm_select_by_lane(idm_plan *p, const double *loss_a, const double *loss_b,
                              const float *params_a, const float *params_b, float *params_out,
                              int32_t *chose_a, void *stream) {
    if (!p || !loss_a || !loss_b || !params_a || !params_b || !params_out)
        return fail(IDM_ERR_INVALID_ARG, "null argument");
    hipError_t e = launch_select_by_lane(loss_a, loss_b, p->d_lane_of, params_a, params_b,
                                         p->pb.n_vehicles, params_out, chose_a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "select launch");
    return IDM_OK;
}

idm_status idm_fit_step(idm_plan *p, const idm_fit_state *st, const double *p0, const float *v_init,
                        const idm_obs *obs, void *ws, void *stream) {
    if (!p) return fail(IDM_ERR_INVALID_ARG, "plan is null");
    idm_status r = check_fit(p, st, p0, v_init, obs, ws);
    if (r != IDM_OK) return r;
    return run_fit_step(p, st, p0, v_init, obs, ws, (hipStream_t)stream);
}

idm_status idm_fit_run(idm_plan *p, const idm_fit_state *st, const double *p0, const float *v_init,
                       const idm_obs *obs, int32_t n_iters, void *ws, void *stream) {
    if (!p) return fail(IDM_ERR_INVALID_ARG, "plan is null");
    if (n_iters < 0) return fail(IDM_ERR_INVALID_ARG, "n_iters < 0");
    idm_status r = check_fit(p, st, p0, v_init, obs, ws);
    if (r != IDM_OK) return r;
    hipStream_t s = nullptr;
    r = graph_stream_enter(p, (hipStream_t)stream, &s);
    if (r != IDM_OK) return r;
    std::vector<unsigned char> key(sizeof(idm_fit_state) + sizeof(idm_obs) + 3 * sizeof(void *));
    unsigned char *k = key.data();
    memcpy(k, st, sizeof(idm_fit_state));
    memcpy(k + sizeof(idm_fit_state), obs, sizeof(idm_obs));
    const void *ptrs[3] = {p0, v_init, ws};
    memcpy(k + sizeof(idm_fit_state) + sizeof(idm_obs), ptrs, sizeof ptrs);
    if (!p->fit_exec || p->fit_key != key) {
        if (p->fit_exec) hipGraphExecDestroy(p->fit_exec);
        p->fit_exec = nullptr;
        r = capture(s, &p->fit_exec, [&]() { return run_fit_step(p, st, p0, v_init, obs, ws, s); });
        if (r != IDM_OK) return r;
        p->fit_key = key;
    }
    for (int32_t i = 0; i < n_iters; ++i) {
        hipError_t e = hipGraphLaunch(p->fit_exec, s);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch(fit)");
    }
    return graph_stream_leave(p, (hipStream_t)stream);
}

idm_status idm_step_graph_launch(idm_plan *p, const idm_step_args *a, void *stream) {
    if (!p) return fail(IDM_ERR_INVALID_ARG, "plan is null");
    idm_status r = check_step(p, a);
    if (r != IDM_OK) return r;
    hipStream_t s = nullptr;
    r = graph_stream_enter(p, (hipStream_t)stream, &s);
    if (r != IDM_OK) return r;
    if (!p->step_exec || memcmp(&p->step_key, a, sizeof *a) != 0) {
        if (p->step_exec) hipGraphExecDestroy(p->step_exec);
        p->step_exec = nullptr;
        r = capture(s, &p->step_exec, [&]() { return run_step(p, a, s); });
        if (r != IDM_OK) return r;
        p->step_key = *a;
    }
    hipError_t e = hipGraphLaunch(p->step_exec, s);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch(step)");
    return graph_stream_leave(p, (hipStream_t)stream);
}

idm_status idm_plan_autotune(idm_plan *p, const idm_step_args *a, size_t ws_bytes, int32_t reps,
                             void *stream) {
    if (!p) return fail(IDM_ERR_INVALID_ARG, "plan is null");
    idm_status r = check_step(p, a);
    if (r != IDM_OK) return r;
    if (reps < 1) return fail(IDM_ERR_INVALID_ARG, "reps must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    const bool dense = a->grad_traj_d || a->grad_traj_v;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus <= 0) cus = 256;
    const std::vector<int64_t> key = tune_key(p, dense, a->obs_target != nullptr, cus);
    {
        bool hit = false;
        Shape c;
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                hit = true;
                c = it->second;
            }
        }
        if (hit) {
            const int64_t nb = c.tile > 0 ? 0
                                          : count_boundaries(p->offsets, p->pb.n_lanes,
                                                             (int64_t)c.threads * c.per_thread);
            const int64_t nt =
                c.tile > 0 ? count_tiles(p->offsets, p->pb.n_lanes, c.threads, c.tile) : 0;
            // the cached shape is taken when its workspace fits and its layout
            // builds; otherwise the shapes are timed again
            if (ws_total(p, dims(c.K, nb, c.stored, nt)) <= ws_bytes &&
                build_layout(p, c) == IDM_OK) {
                p->tuned_cached = 1;
                return IDM_OK;
            }
        }
    }
    std::vector<Shape> cands, spilling;
    // the checkpoint interval the caller fixed is kept; otherwise K = KB
    const bool k_fixed = p->pb.ckpt_every > 0;
    for (int t : {64, 128, 256, 512, 1024})
        for (int rr : {1, 2, 4}) {
            // bundles up to 8 times the longest lane; a shorter bundle cuts lanes
            // into pieces (one vehicle per thread, at most 8 pieces below 1024
            // threads)
            const int64_t cap = (int64_t)t * rr;
            if (cap < p->max_lane && (rr != 1 || (cap * 8 < p->max_lane && t < 1024))) continue;
            if (cap > 8 * std::max<int64_t>(p->max_lane, 64)) continue;
            const int64_t nbnd = count_boundaries(p->offsets, p->pb.n_lanes, cap);
            // keeping every step's states (a plan made with store_states = 1,
            // or 2: the autotuner weighs both backwards): whole lanes, the
            // plan's K (it only groups the FP32 gradient sums), no register
            // block to choose
            if (p->store_pref >= 1 && nbnd == 0 && ws_total(p, dims(p->sh.K, 0, true)) <= ws_bytes &&
                backward_stored_kernel(p->pb.bound, rr, t, dense)) {
                Shape sh;
                sh.threads = t;
                sh.per_thread = rr;
                sh.K = p->sh.K;
                sh.KB = default_kb(rr, sh.K) > 0 ? default_kb(rr, sh.K) : kbs_for(rr)[0];
                sh.grid = 0;
                sh.stored = true;
                cands.push_back(sh);
            }
            if (p->store_pref == 1) continue;
            for (int KB : kbs_for(rr)) {
                // K = KB, and K = 2 KB where a stash variant exists for the shape
                for (int twice = 0; twice < 2; ++twice) {
                    const int K = k_fixed ? p->pb.ckpt_every : (twice ? 2 * KB : KB);
                    if (k_fixed && twice) break;
                    if (K % KB != 0 || ws_total(p, dims(K, nbnd, false)) > ws_bytes) continue;
                    KernelFn fb = backward_kernel(p->pb.bound, rr, t, KB, K, dense, nbnd > 0);
                    if (twice && fb == backward_kernel(p->pb.bound, rr, t, KB, KB, dense, nbnd > 0))
                        continue;
                    hipFuncAttributes fa;
                    if (!fb || hipFuncGetAttributes(&fa, fb) != hipSuccess) continue;
                    Shape sh;
                    sh.threads = t;
                    sh.per_thread = rr;
                    sh.K = K;
                    sh.KB = KB;
                    sh.grid = 0;
                    // shapes whose backward spills more than a few registers (small
                    // spills sit outside the step loops) are timed only when no other
                    // shape holds the longest lane
                    (fa.localSizeBytes > 128 ? spilling : cands).push_back(sh);
                }
            }
        }
    // halo tiles (kept states, one vehicle per thread) where some lane is
    // longer than the work-group (otherwise they are whole-lane bundles with
    // more launches): J steps per launch, J a multiple of the plan's K
    if (p->store_pref >= 1) {
        const int tile_cands[][2] = {{256, 64},  {256, 128}, {512, 128}, {512, 256},
                                     {576, 128}, {640, 128}, {640, 256}, {768, 256},
                                     {1024, 256}};
        for (const auto &tc : tile_cands) {
            const int t = tc[0], J = tc[1];
            if (p->max_lane <= t || J % p->sh.K != 0) continue;
            const int64_t nt = count_tiles(p->offsets, p->pb.n_lanes, t, J);
            if (ws_total(p, dims(p->sh.K, 0, true, nt)) > ws_bytes) continue;
            if (!forward_tiled_kernel(p->pb.bound, t) ||
                !backward_tiled_kernel(p->pb.bound, t, dense))
                continue;
            Shape sh;
            sh.threads = t;
            sh.per_thread = 1;
            sh.K = p->sh.K;
            sh.KB = default_kb(1, sh.K) > 0 ? default_kb(1, sh.K) : kbs_for(1)[0];
            sh.grid = 0;
            sh.stored = true;
            sh.tile = J;
            cands.push_back(sh);
        }
    }
    if (cands.empty()) cands.swap(spilling);
    if (cands.empty()) return fail(IDM_ERR_WORKSPACE, "no launch shape fits the workspace");
    const Shape orig = p->sh;
    // every candidate is timed as replays of its captured forward + backward
    // (the way the step and fit graphs run it: a shape with more launches per
    // pass pays only their in-graph gaps), on the caller's stream or, for the
    // null stream, the plan's side stream
    hipStream_t gs = nullptr;
    r = graph_stream_enter(p, s, &gs);
    if (r != IDM_OK) return r;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    float best = INFINITY;
    Shape best_sh = orig;
    for (Shape sh : cands) {
        for (int persistent = 0; persistent < 2; ++persistent) {
            Shape s2 = sh;
            if (persistent && sh.tile > 0) continue;  // one work-group per tile
            if (persistent) {
                KernelFn fb =
                    sh.stored
                        ? backward_stored_kernel(p->pb.bound, sh.per_thread, sh.threads, dense)
                        : backward_kernel(p->pb.bound, sh.per_thread, sh.threads, sh.KB, sh.K,
                                          dense,
                                          count_boundaries(p->offsets, p->pb.n_lanes,
                                                           (int64_t)sh.threads * sh.per_thread) > 0);
                int occ = 0;
                if (!fb || hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fb, sh.threads, 0) !=
                               hipSuccess || occ < 1)
                    continue;
                s2.grid = cus * occ;
            }
            r = build_layout(p, s2);
            if (r != IDM_OK) continue;
            if (persistent && p->n_bundles <= s2.grid) continue;  // same as non-persistent
            hipGraphExec_t ex = nullptr;
            r = capture(gs, &ex, [&]() { return run_step(p, a, gs); });
            if (r != IDM_OK) break;
            // as many untimed replays first (a shape's first replays can run
            // several per cent slower, measured on halo tiles), then the best
            // of three timed batches (single batches of close shapes swapped
            // places from run to run)
            hipError_t he = hipSuccess;
            for (int i = 0; i < reps && he == hipSuccess; ++i) he = hipGraphLaunch(ex, gs);
            float ms = INFINITY;
            for (int batch = 0; batch < 3 && he == hipSuccess; ++batch) {
                he = hipEventRecord(e0, gs);
                for (int i = 0; i < reps && he == hipSuccess; ++i) he = hipGraphLaunch(ex, gs);
                if (he == hipSuccess) he = hipEventRecord(e1, gs);
                if (he == hipSuccess) he = hipEventSynchronize(e1);
                float bm = 0.0f;
                if (he == hipSuccess) he = hipEventElapsedTime(&bm, e0, e1);
                if (he == hipSuccess) ms = std::min(ms, bm);
            }
            hipGraphExecDestroy(ex);
            if (he != hipSuccess) {
                r = hip_fail(he, "autotune timing");
                break;
            }
            if (ms < best) {
                best = ms;
                best_sh = s2;
            }
        }
        if (r != IDM_OK) break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    idm_status r2 = build_layout(p, r == IDM_OK ? best_sh : orig);
    if (r != IDM_OK) return r;
    r = graph_stream_leave(p, s);
    if (r != IDM_OK) return r;
    if (r2 == IDM_OK) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache[key] = best_sh;
        p->tuned_cached = 0;
    }
    return r2;
}

}  // extern "C"

// ---------------------------------------------------------------- ego-only reconstruction

struct idm_ego_plan {
    idm_ego_problem pb{};
    int32_t K = 32;
    hipGraphExec_t fit_exec = nullptr;
    std::vector<unsigned char> fit_key;
    hipStream_t side = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int32_t tuned_cached = 0;  // the last autotune took its shape from the cache
};

namespace {

int32_t ego_nblk(const idm_ego_plan *p) {
    return p->pb.n_steps == 0 ? 0 : (p->pb.n_steps + p->K - 1) / p->K;
}
size_t ego_sn(const idm_ego_plan *p) { return (size_t)p->pb.n_steps * (size_t)p->pb.n_traj; }
// Workspace: [loss parts N doubles][dL/dparams 5N doubles][dL/dG SN floats]
//            [dL/dD SN floats][checkpoints nblk x 2 x N floats]
size_t ego_ws_grad_prm(const idm_ego_plan *p) { return align_up(sizeof(double) * (size_t)p->pb.n_traj); }
size_t ego_ws_grad_gap(const idm_ego_plan *p) {
    return ego_ws_grad_prm(p) + align_up(sizeof(double) * 5 * (size_t)p->pb.n_traj);
}
size_t ego_ws_grad_dv(const idm_ego_plan *p) {
    return ego_ws_grad_gap(p) + align_up(sizeof(float) * ego_sn(p));
}
size_t ego_ws_ckpt(const idm_ego_plan *p) { return ego_ws_grad_dv(p) + align_up(sizeof(float) * ego_sn(p)); }
size_t ego_ws_total(const idm_ego_plan *p) {
    return ego_ws_ckpt(p) + align_up(sizeof(float) * 2 * (size_t)ego_nblk(p) * (size_t)p->pb.n_traj);
}

idm_status ego_check_vars(const idm_ego_plan *p, const idm_ego_vars *x, const float *v_init,
                          const void *ws) {
    if (!x || !v_init || !ws) return fail(IDM_ERR_INVALID_ARG, "null argument");
    if (!x->v0 || !x->T || !x->a || !x->b || !x->s0)
        return fail(IDM_ERR_INVALID_ARG, "null parameter array");
    if (p->pb.n_steps > 0 && (!x->gap || !x->dv))
        return fail(IDM_ERR_INVALID_ARG, "null gap or speed-difference array");
    return IDM_OK;
}

EgoArgs ego_args(const idm_ego_plan *p, const idm_ego_vars *x, const float *v_init, void *ws) {
    EgoArgs a{};
    a.n = p->pb.n_traj;
    a.n_steps = p->pb.n_steps;
    a.K = p->K;
    a.dt = p->pb.dt;
    a.inv_dt = 1.0f / p->pb.dt;
    a.a_min = p->pb.a_min;
    a.gap_floor = p->pb.gap_floor;
    a.v0 = x->v0; a.T = x->T; a.a = x->a; a.b = x->b; a.s0 = x->s0;
    a.gap = x->gap;
    a.dv = x->dv;
    a.v_init = v_init;
    // no checkpoint is kept without steps (the region is empty)
    a.ckpt = p->pb.n_steps > 0 ? (float *)((char *)ws + ego_ws_ckpt(p)) : nullptr;
    return a;
}

idm_status ego_run_forward(idm_ego_plan *p, const EgoArgs &a, hipStream_t s) {
    hipError_t e = launch_ego_forward(p->pb.bound, a, s);
    return e == hipSuccess ? IDM_OK : hip_fail(e, "ego forward launch");
}

idm_status ego_run_backward(idm_ego_plan *p, EgoArgs a, const idm_ego_obs *obs, double *g_prm,
                            float *g_gap, float *g_dv, double *g_v0, void *ws, hipStream_t s) {
    a.obs_off = obs->offsets;
    a.obs_step = obs->step;
    a.obs_pos = obs->pos;
    a.g_prm = g_prm;
    a.g_gap = g_gap;
    a.g_dv = g_dv;
    a.g_v0 = g_v0;
    a.loss_part = (double *)ws;
    hipError_t e = launch_ego_backward(p->pb.bound, a, s);
    return e == hipSuccess ? IDM_OK : hip_fail(e, "ego backward launch");
}

idm_status ego_check_obs(const idm_ego_obs *obs) {
    if (!obs || !obs->offsets || obs->n_obs < 0 || (obs->n_obs > 0 && (!obs->step || !obs->pos)))
        return fail(IDM_ERR_INVALID_ARG, "observations: null arrays or negative count");
    return IDM_OK;
}

EgoAdamArgs ego_adam_args(const idm_ego_plan *p, const idm_ego_fit_state *st, void *ws) {
    EgoAdamArgs a{};
    a.n = p->pb.n_traj;
    a.sn = (int64_t)ego_sn(p);
    a.params = st->params;
    a.gap = st->gap;
    a.dv = st->dv;
    a.m = st->m;
    a.v = st->v;
    if (ws) {
        a.g_prm = (const double *)((char *)ws + ego_ws_grad_prm(p));
        a.g_gap = (const float *)((char *)ws + ego_ws_grad_gap(p));
        a.g_dv = (const float *)((char *)ws + ego_ws_grad_dv(p));
    }
    a.step = st->step;
    a.step_rw = st->step;
    for (int j = 0; j < 5; ++j) {
        a.lo[j] = st->lo[j];
        a.hi[j] = st->hi[j];
    }
    a.lr0 = st->lr0;
    a.lr1 = st->lr1;
    a.lr_steps = st->lr_steps;
    a.beta1 = st->beta1;
    a.beta2 = st->beta2;
    a.eps = st->eps;
    return a;
}

idm_status ego_check_fit(const idm_ego_plan *p, const idm_ego_fit_state *st, const float *v_init,
                         const idm_ego_obs *obs, const void *ws) {
    if (!p || !st || !v_init || !ws) return fail(IDM_ERR_INVALID_ARG, "null argument");
    if (!st->params || !st->gap || !st->dv || !st->m || !st->v || !st->step || !st->loss_hist ||
        st->hist_len < 1)
        return fail(IDM_ERR_INVALID_ARG, "fit state: null arrays or hist_len < 1");
    if (st->lr_steps < 1) return fail(IDM_ERR_INVALID_ARG, "fit state: lr_steps < 1");
    for (int j = 0; j < 5; ++j)
        if (!(st->lo[j] <= st->hi[j])) return fail(IDM_ERR_INVALID_ARG, "fit state: box %d empty", j);
    return ego_check_obs(obs);
}

// forward (checkpoints only) -> backward into the workspace gradients ->
// loss history + step counter -> Adam
idm_status ego_run_fit_step(idm_ego_plan *p, const idm_ego_fit_state *st, const float *v_init,
                            const idm_ego_obs *obs, void *ws, hipStream_t s) {
    idm_ego_vars x{st->params, st->params + p->pb.n_traj, st->params + 2 * (size_t)p->pb.n_traj,
                   st->params + 3 * (size_t)p->pb.n_traj, st->params + 4 * (size_t)p->pb.n_traj,
                   st->gap, st->dv};
    EgoArgs a = ego_args(p, &x, v_init, ws);
    idm_status r = ego_run_forward(p, a, s);
    if (r != IDM_OK) return r;
    r = ego_run_backward(p, a, obs, (double *)((char *)ws + ego_ws_grad_prm(p)),
                         (float *)((char *)ws + ego_ws_grad_gap(p)),
                         (float *)((char *)ws + ego_ws_grad_dv(p)), nullptr, ws, s);
    if (r != IDM_OK) return r;
    hipError_t e = launch_fit_finalize((const double *)ws, p->pb.n_traj, 1.0, st->step,
                                       st->loss_hist, st->hist_len, s);
    if (e != hipSuccess) return hip_fail(e, "ego fit finalize launch");
    e = launch_ego_adam(ego_adam_args(p, st, ws), s);
    return e == hipSuccess ? IDM_OK : hip_fail(e, "ego Adam launch");
}

}  // namespace

extern "C" {

idm_status idm_ego_plan_create(const idm_ego_problem *pb, idm_ego_plan **out) {
    if (!pb || !out) return fail(IDM_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (pb->n_traj < 1 || pb->n_traj > IDM_MAX_VEHICLES || pb->n_steps < 0)
        return fail(IDM_ERR_INVALID_ARG, "sizes: N=%d S=%d", pb->n_traj, pb->n_steps);
    if (!(pb->dt > 0.0f) || !std::isfinite(pb->dt))
        return fail(IDM_ERR_INVALID_ARG, "dt must be positive and finite");
    if (!std::isfinite(pb->a_min) || !(pb->a_min < 0.0f))
        return fail(IDM_ERR_INVALID_ARG, "a_min must be negative and finite");
    if (!(pb->gap_floor >= 0.0f) || !std::isfinite(pb->gap_floor))
        return fail(IDM_ERR_INVALID_ARG, "gap_floor must be >= 0");
    if (pb->delta != 4.0f)
        return fail(IDM_ERR_UNSUPPORTED, "delta=%g: only delta = 4 is implemented", pb->delta);
    if (pb->bound != IDM_BOUND_SOFTPLUS && pb->bound != IDM_BOUND_CLAMP)
        return fail(IDM_ERR_INVALID_ARG, "bound must be IDM_BOUND_SOFTPLUS or IDM_BOUND_CLAMP");
    const int32_t K = pb->ckpt_every == 0 ? 32 : pb->ckpt_every;
    if (K != 8 && K != 16 && K != 32)
        return fail(IDM_ERR_UNSUPPORTED, "ego checkpoint interval %d: 8, 16 or 32", pb->ckpt_every);
    idm_ego_plan *p = new idm_ego_plan();
    p->pb = *pb;
    p->K = K;
    *out = p;
    return IDM_OK;
}

idm_status idm_ego_plan_destroy(idm_ego_plan *p) {
    if (!p) return IDM_OK;
    if (p->fit_exec) hipGraphExecDestroy(p->fit_exec);
    if (p->side) hipStreamDestroy(p->side);
    if (p->ev_in) hipEventDestroy(p->ev_in);
    if (p->ev_out) hipEventDestroy(p->ev_out);
    delete p;
    return IDM_OK;
}

size_t idm_ego_workspace_bytes(const idm_ego_plan *p) { return p ? ego_ws_total(p) : 0; }

idm_status idm_ego_match_steps(const double *t, int32_t m, double dt, int32_t n_steps,
                               int32_t *step_out, void *stream) {
    if (m < 0 || (m > 0 && (!t || !step_out)) || !(dt > 0.0) || n_steps < 0)
        return fail(IDM_ERR_INVALID_ARG, "match_steps: bad arguments");
    if (m == 0) return IDM_OK;
    hipError_t e = launch_ego_match_steps(t, m, dt, n_steps, step_out, (hipStream_t)stream);
    return e == hipSuccess ? IDM_OK : hip_fail(e, "match_steps launch");
}

idm_status idm_ego_initial_speed(const int32_t *offsets, const double *t, const float *pos,
                                 int32_t n, float *v_init_out, void *stream) {
    if (n < 1 || !offsets || !t || !pos || !v_init_out)
        return fail(IDM_ERR_INVALID_ARG, "initial_speed: bad arguments");
    hipError_t e = launch_ego_initial_speed(offsets, t, pos, n, v_init_out, (hipStream_t)stream);
    return e == hipSuccess ? IDM_OK : hip_fail(e, "initial_speed launch");
}

idm_status idm_ego_forward(idm_ego_plan *p, const idm_ego_vars *x, const float *v_init,
                           float *traj_p, float *traj_v, float *traj_a, void *ws, void *stream) {
    if (!p) return fail(IDM_ERR_INVALID_ARG, "plan is null");
    idm_status r = ego_check_vars(p, x, v_init, ws);
    if (r != IDM_OK) return r;
    EgoArgs a = ego_args(p, x, v_init, ws);
    a.traj_p = traj_p;
    a.traj_v = traj_v;
    a.traj_a = traj_a;
    return ego_run_forward(p, a, (hipStream_t)stream);
}

idm_status idm_ego_backward(idm_ego_plan *p, const idm_ego_vars *x, const float *v_init,
                            const idm_ego_obs *obs, double *grad_params, float *grad_gap,
                            float *grad_dv, double *grad_v0, double *loss_out, void *ws,
                            void *stream) {
    if (!p) return fail(IDM_ERR_INVALID_ARG, "plan is null");
    idm_status r = ego_check_vars(p, x, v_init, ws);
    if (r != IDM_OK) return r;
    r = ego_check_obs(obs);
    if (r != IDM_OK) return r;
    if (!grad_params || (p->pb.n_steps > 0 && (!grad_gap || !grad_dv)))
        return fail(IDM_ERR_INVALID_ARG, "null gradient output");
    hipStream_t s = (hipStream_t)stream;
    EgoArgs a = ego_args(p, x, v_init, ws);
    r = ego_run_backward(p, a, obs, grad_params, grad_gap, grad_dv, grad_v0, ws, s);
    if (r != IDM_OK) return r;
    if (loss_out) {
        hipError_t e = launch_loss_finalize((const double *)ws, p->pb.n_traj, 1.0, loss_out, s);
        if (e != hipSuccess) return hip_fail(e, "ego loss finalize launch");
    }
    return IDM_OK;
}

idm_status idm_ego_fit_init(idm_ego_plan *p, const idm_ego_fit_state *st, const float init_params[5],
                            float gap0, float dv0, void *stream) {
    if (!p || !st || !init_params || !st->params || !st->gap || !st->dv || !st->m || !st->v ||
        !st->step)
        return fail(IDM_ERR_INVALID_ARG, "null argument");
    hipError_t e = launch_ego_fit_init(ego_adam_args(p, st, nullptr), init_params, gap0, dv0,
                                       (hipStream_t)stream);
    return e == hipSuccess ? IDM_OK : hip_fail(e, "ego fit init launch");
}

idm_status idm_ego_fit_step(idm_ego_plan *p, const idm_ego_fit_state *st, const float *v_init,
                            const idm_ego_obs *obs, void *ws, void *stream) {
    idm_status r = ego_check_fit(p, st, v_init, obs, ws);
    if (r != IDM_OK) return r;
    return ego_run_fit_step(p, st, v_init, obs, ws, (hipStream_t)stream);
}

idm_status idm_ego_fit_run(idm_ego_plan *p, const idm_ego_fit_state *st, const float *v_init,
                           const idm_ego_obs *obs, int32_t n_iters, void *ws, void *stream) {
    idm_status r = ego_check_fit(p, st, v_init, obs, ws);
    if (r != IDM_OK) return r;
    if (n_iters < 0) return fail(IDM_ERR_INVALID_ARG, "n_iters < 0");
    hipStream_t s = nullptr;
    r = graph_stream_enter(p, (hipStream_t)stream, &s);
    if (r != IDM_OK) return r;
    std::vector<unsigned char> key(sizeof(idm_ego_fit_state) + sizeof(idm_ego_obs) + 2 * sizeof(void *));
    memcpy(key.data(), st, sizeof(idm_ego_fit_state));
    memcpy(key.data() + sizeof(idm_ego_fit_state), obs, sizeof(idm_ego_obs));
    const void *ptrs[2] = {v_init, ws};
    memcpy(key.data() + sizeof(idm_ego_fit_state) + sizeof(idm_ego_obs), ptrs, sizeof ptrs);
    if (!p->fit_exec || p->fit_key != key) {
        if (p->fit_exec) hipGraphExecDestroy(p->fit_exec);
        p->fit_exec = nullptr;
        r = capture(s, &p->fit_exec, [&]() { return ego_run_fit_step(p, st, v_init, obs, ws, s); });
        if (r != IDM_OK) return r;
        p->fit_key = key;
    }
    for (int32_t i = 0; i < n_iters; ++i) {
        hipError_t e = hipGraphLaunch(p->fit_exec, s);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch(ego fit)");
    }
    return graph_stream_leave(p, (hipStream_t)stream);
}

}  // extern "C"
