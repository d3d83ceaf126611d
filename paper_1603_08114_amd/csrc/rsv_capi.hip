// rsv_capi.hip -- host side of the C ABI declared in include/rsv_hmc.h.
//
// Owns no device memory: carves the caller's workspace, builds the tile
// decomposition of every chain on the host (re-built only when the leapfrog
// knobs change), and enqueues the kernels (rsv_kernels.hip, rsv_traj_*.hip,
// rsv_resident.hip) on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rsv_hmc.h"
#include "rsv_internal.h"

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace rsv {
rsv_status set_error(rsv_status code, const char* where, const char* what) {
    g_last_error = std::string(where) + ": " + what;
    return code;
}
}  // namespace rsv

using namespace rsv;

namespace {

rsv_status fail(rsv_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define RSV_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) return fail(RSV_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Each momentum step (kick) invalidates one more site at each tile cut: the
// halo covers the kicks of a trajectory plus the bond to the next site.
int halo_for(int n_kicks) { return (n_kicks + 1 + 3) & ~3; }

// Kicks per trajectory of n_steps: one per leapfrog step, two per Omelyan
// step, three per Forest-Ruth step.
int kicks_for(int32_t flags, int n_steps) {
    if (flags & RSV_FLAG_OMELYAN) return 2 * n_steps;
    if (flags & RSV_FLAG_FOREST_RUTH) return 3 * n_steps;
    return n_steps;
}

// Tile decomposition of one chain of length T for tiles of NW wavefronts
// with S sites per lane and a trajectory of n_kicks: tiles of 64*NW*S loaded
// sites whose exact ranges [a, b) partition [0, T).  Returns false if the
// halo does not fit.
bool tile_chain(int32_t chain, int32_t T, int S, int NW, int n_kicks,
                std::vector<TileDesc>& body, std::vector<TileDesc>& edges) {
    const int L = 64 * NW * S;
    const int H = halo_for(n_kicks);
    if (T <= L) {
        const TileDesc t{chain, 0, 0, T, T % S != 0 ? 1 : 0, {0, 0, 0}};
        if (t.edge) edges.push_back(t); else body.push_back(t);
        return true;
    }
    if (L <= 2 * H) return false;
    int32_t a = 0, b = L - H;
    body.push_back(TileDesc{chain, 0, a, b, 0, {0, 0, 0}});
    for (;;) {
        a = b;
        const int32_t la = a - H;
        if (la + L >= T) {
            const TileDesc t{chain, la, a, T, (T - la) % S != 0 ? 1 : 0, {0, 0, 0}};
            if (t.edge) edges.push_back(t); else body.push_back(t);
            return true;
        }
        b = la + L - H;
        body.push_back(TileDesc{chain, la, a, b, 0, {0, 0, 0}});
    }
}

int32_t count_tiles(int32_t T, int S, int NW, int n_kicks) {
    std::vector<TileDesc> b, e;
    if (!tile_chain(0, T, S, NW, n_kicks, b, e)) return -1;
    return static_cast<int32_t>(b.size() + e.size());
}

struct Layout {
    size_t y2_d = 0, y2_f = 0, lrv_f = 0, h_prop = 0, tiles = 0, chains = 0, partials = 0,
           edge = 0, accept = 0, shift = 0, mass_sqrt = 0, acc = 0, counters = 0,
           bins = 0, bin_chains = 0, bin_tiles = 0, slices = 0, arrive = 0, total = 0;
    int32_t max_tiles = 0;
};

rsv_status check_problem(const rsv_problem* pb, int64_t* n_data, int64_t* n_state) {
    if (!pb) return fail(RSV_EINVAL, "problem is NULL");
    if (pb->n_series < 1) return fail(RSV_EINVAL, "n_series must be >= 1");
    if (pb->chains_per_series < 1) return fail(RSV_EINVAL, "chains_per_series must be >= 1");
    const int64_t n_chains = static_cast<int64_t>(pb->n_series) * pb->chains_per_series;
    if (n_chains > 65535) return fail(RSV_EINVAL, "at most 65535 chains");
    if (!pb->offsets) return fail(RSV_EINVAL, "offsets is NULL");
    if (pb->offsets[0] != 0) return fail(RSV_EINVAL, "offsets[0] must be 0");
    for (int s = 0; s < pb->n_series; ++s) {
        const int64_t T = pb->offsets[s + 1] - pb->offsets[s];
        if (T < 3) return fail(RSV_EINVAL, "series %d has T = %lld < 3", s, (long long)T);
        if (T > (int64_t(1) << 30)) return fail(RSV_EINVAL, "series %d is too long", s);
    }
    if (pb->precision != RSV_F64 && pb->precision != RSV_F32_MIXED)
        return fail(RSV_EINVAL, "unknown precision %d", pb->precision);
    if (pb->terms < 1 || pb->terms > RSV_TERMS_RSV)
        return fail(RSV_EINVAL, "terms must be a non-empty subset of RSV_TERMS_RSV");
    if (pb->max_steps < 1) return fail(RSV_EINVAL, "max_steps must be >= 1");
    if (!(pb->dtau_jitter >= 0.0 && pb->dtau_jitter < 1.0))
        return fail(RSV_EINVAL, "dtau_jitter must be in [0, 1)");
    if (pb->flags & ~(RSV_FLAG_RESIDENT | RSV_FLAG_LEVEL_MOVE | RSV_FLAG_OMELYAN |
                      RSV_FLAG_FOREST_RUTH))
        return fail(RSV_EINVAL, "unknown flags 0x%x", pb->flags);
    if ((pb->flags & RSV_FLAG_OMELYAN) && (pb->flags & RSV_FLAG_FOREST_RUTH))
        return fail(RSV_EINVAL, "at most one integrator flag");
    const rsv_prior& p = pb->prior;
    if (!(p.mu_var > 0 && p.xi_var > 0 && p.eta_shape > 0 && p.eta_scale > 0 && p.u_shape > 0 &&
          p.u_scale > 0 && std::isfinite(p.mu_mean) && std::isfinite(p.xi_mean) &&
          std::isfinite(p.mu_var) && std::isfinite(p.xi_var)))
        return fail(RSV_EINVAL, "prior variances, shapes and scales must be finite and > 0");
    *n_data = pb->offsets[pb->n_series];
    *n_state = *n_data * pb->chains_per_series;
    return RSV_OK;
}

rsv_status tile_shape(const rsv_problem* pb, int* S, int* NW) {
    traj_default_shape(pb->precision, S, NW);
    if (pb->sites_per_lane) *S = pb->sites_per_lane;
    if (pb->waves_per_tile) *NW = pb->waves_per_tile;
    if (!traj_shape_available(pb->precision, *S, *NW))
        return fail(RSV_EINVAL, "tile shape (sites_per_lane %d, waves_per_tile %d) is not "
                                "compiled for this precision", *S, *NW);
    return RSV_OK;
}

rsv_status make_layout(const rsv_problem* pb, Layout* L) {
    int64_t n_data = 0, n_state = 0;
    rsv_status st = check_problem(pb, &n_data, &n_state);
    if (st != RSV_OK) return st;
    int S = 0, NW = 0;
    rsv_status sh = tile_shape(pb, &S, &NW);
    if (sh != RSV_OK) return sh;
    int64_t tiles = 0;
    for (int s = 0; s < pb->n_series; ++s) {
        const int32_t T = static_cast<int32_t>(pb->offsets[s + 1] - pb->offsets[s]);
        const int32_t n = count_tiles(T, S, NW, kicks_for(pb->flags, pb->max_steps));
        if (n < 0)
            return fail(RSV_EINVAL, "max_steps = %d needs a halo wider than a tile (%d sites)",
                        pb->max_steps, 64 * NW * S);
        tiles += static_cast<int64_t>(n) * pb->chains_per_series;
    }
    if (tiles > (int64_t(1) << 30)) return fail(RSV_EINVAL, "too many tiles");
    const int64_t n_chains = static_cast<int64_t>(pb->n_series) * pb->chains_per_series;
    const size_t elem = pb->precision == RSV_F64 ? sizeof(double) : sizeof(float);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    L->y2_d = take(n_data * sizeof(double));
    if (pb->precision == RSV_F32_MIXED) {
        L->y2_f = take(n_data * sizeof(float));
        L->lrv_f = take(n_data * sizeof(float));
    }
    L->h_prop = take(n_state * elem);
    L->tiles = take(tiles * sizeof(TileDesc));
    L->chains = take(n_chains * sizeof(ChainDesc));
    L->partials = take(tiles * kPart * sizeof(double));
    L->edge = take(n_chains * kEdge * sizeof(double));
    L->accept = take(n_chains * sizeof(int32_t));
    L->shift = take(n_chains * sizeof(double));
    L->mass_sqrt = take(n_data * elem);
    L->acc = take(2 * n_state * sizeof(float));
    L->counters = take(kNumCounters * sizeof(uint32_t));
    L->bins = take(n_chains * sizeof(BinDesc));
    L->bin_chains = take(n_chains * sizeof(int32_t));
    L->bin_tiles = take(tiles * sizeof(int32_t));
    L->slices = take((tiles / kSliceTiles + n_chains) * 2 * kNQ * sizeof(double));
    L->arrive = take(n_chains * sizeof(uint32_t));
    L->total = off;
    L->max_tiles = static_cast<int32_t>(tiles);
    return RSV_OK;
}

}  // namespace

struct rsv_ctx {
    rsv_problem pb;
    std::vector<int64_t> offsets;
    int32_t n_chains = 0, C = 0, S = 0, NW = 0, max_T = 0;
    int64_t n_data = 0, n_state = 0;
    void* h = nullptr;
    rsv_theta* theta = nullptr;
    const float* log_mass = nullptr;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    Layout lay;
    // contexts of rsv_hmc_init_static: the device whose static workspace they
    // use and the generation they hold (-1: the caller's workspace)
    int static_dev = -1;
    uint64_t static_gen = 0;
    // device views into the workspace
    double* y2_d = nullptr;
    float* y2_f = nullptr;
    float* lrv_f = nullptr;
    void* h_prop = nullptr;
    TileDesc* tiles = nullptr;
    ChainDesc* chains = nullptr;
    double* partials = nullptr;
    double* edge = nullptr;
    int32_t* accept = nullptr;  // per chain: 1 if its current state is in h_prop
    double* shift = nullptr;    // per chain: pending level shift of the current state
    void* mass_sqrt = nullptr;    // per data site sqrt(m_t) (with a diagonal mass), in the
                                  // state's precision
    float* acc_f = nullptr;       // per state entry: FP32 batch sum, then batch sum of squares
    uint32_t* counters = nullptr;
    double* slices = nullptr;     // split finalize: slice sums
    uint32_t* arrive = nullptr;   // split finalize: per-chain arrival counts
    BinDesc* bins = nullptr;          // resident sweeps: bins of chains, one per block
    int32_t* bin_chains = nullptr;
    int32_t* bin_tiles = nullptr;
    // host mirrors of the current decomposition
    std::vector<rsv_leapfrog> lf;
    std::vector<TileDesc> h_tiles;
    std::vector<ChainDesc> h_chains;
    int32_t n_body = 0, n_edge = 0;
    int32_t max_tiles_per_chain = 0;
    int32_t n_bins = 0;        // bins of the resident kernel (0: not available)
    // kernel timing: event pairs around each trajectory-kernel launch (a
    // resident launch is one pair covering all its sweeps)
    std::vector<hipEvent_t> ev_start, ev_stop;
    std::vector<int64_t> ev_trajectories;  // trajectories each recorded pair covers
    size_t ev_used = 0;
    // Sweeps in two chain groups: chains [0, split) on `stream` and
    // [split, n_chains) on `side`, forked from and joined to `stream` by
    // events at each rsv_hmc_sweep call, so that one group's finalize (a
    // short, latency-bound launch) and the tail of its trajectory launch run
    // beside the other group's trajectory.  The tiles of each group are
    // contiguous in the tile list (group_tile_first / group_tiles).
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int32_t split = 0;  // == n_chains: one group
    int32_t group_tile_first[2] = {0, 0}, group_tiles[2] = {0, 0};

    ~rsv_ctx() {
        for (hipEvent_t e : ev_start) (void)hipEventDestroy(e);
        for (hipEvent_t e : ev_stop) (void)hipEventDestroy(e);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (side) (void)hipStreamDestroy(side);
    }
};

// ---------------------------------------------------------------------------
// Static workspace of rsv_hmc_init_static: one array per device, taken by the
// newest static context on that device.  In host code `scratch` names a
// host-side stand-in; its device address comes from hipGetSymbolAddress,
// once per device, and only that address is passed to kernels and copies.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[RSV_STATIC_WORKSPACE_BYTES];

namespace {

std::mutex g_static_mu;
std::vector<void*> g_static_ptr;     // per device: device address of `scratch`
std::vector<uint64_t> g_static_gen;  // per device: generation of the newest static context

// A context may be used: not NULL, and (for a static context) still the
// newest static context of its device.
rsv_status usable(const rsv_ctx* c) {
    if (!c) return fail(RSV_ESTATE, "context is NULL");
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_gen[c->static_dev] != c->static_gen)
            return fail(RSV_ESTATE, "this static-workspace context was superseded by a newer "
                                    "rsv_hmc_init_static on device %d", c->static_dev);
    }
    return RSV_OK;
}

}  // namespace

namespace {

bool level_moves(const rsv_ctx* c) { return (c->pb.flags & RSV_FLAG_LEVEL_MOVE) != 0; }

// Packs whole chains into bins for the resident kernel: a block integrates
// its bin's tiles in rounds of kTPB tiles (four single-wavefront tiles, or
// one tile of four wavefronts), so a bin holds up to kTPB * rounds tiles,
// with rounds just enough for the longest chain.  Chains are placed largest
// first into the bin with the least room that still fits them (best fit
// decreasing); bins with more tiles come first.
constexpr int kBinMaxChainTiles = 64;  // longer chains run one launch per kernel

void pack_bins(const std::vector<ChainDesc>& chains, int tiles_per_round,
               std::vector<BinDesc>& bins, std::vector<int32_t>& bin_chains,
               std::vector<int32_t>& bin_tiles) {
    struct Item { int32_t chain, tiles; };
    std::vector<Item> items;
    int32_t max_tiles = 1;
    for (int32_t ch = 0; ch < static_cast<int32_t>(chains.size()); ++ch) {
        const ChainDesc& d = chains[ch];
        items.push_back(Item{ch, d.tile_count + (d.edge_tile >= 0 ? 1 : 0)});
        max_tiles = std::max(max_tiles, items.back().tiles);
    }
    const int32_t cap = tiles_per_round * ((max_tiles + tiles_per_round - 1) / tiles_per_round);
    std::stable_sort(items.begin(), items.end(),
                     [](const Item& a, const Item& b) { return a.tiles > b.tiles; });
    std::vector<std::vector<int32_t>> members;   // chains of each bin
    std::vector<int32_t> used;
    std::vector<std::vector<int32_t>> by_room(cap + 1);  // open bins by free tiles
    for (const Item& it : items) {
        int32_t b = -1;
        for (int room = it.tiles; room <= cap && b < 0; ++room) {
            if (!by_room[room].empty()) {
                b = by_room[room].front();
                by_room[room].erase(by_room[room].begin());
            }
        }
        if (b < 0) {
            b = static_cast<int32_t>(members.size());
            members.emplace_back();
            used.push_back(0);
        }
        members[b].push_back(it.chain);
        used[b] += it.tiles;
        if (used[b] < cap) by_room[cap - used[b]].push_back(b);
    }
    std::vector<int32_t> order(members.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int32_t>(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return used[a] > used[b]; });
    for (int32_t b : order) {
        BinDesc d{static_cast<int32_t>(bin_chains.size()), static_cast<int32_t>(members[b].size()),
                  static_cast<int32_t>(bin_tiles.size()), used[b]};
        for (int32_t ch : members[b]) {
            bin_chains.push_back(ch);
            const ChainDesc& cd = chains[ch];
            for (int32_t t = 0; t < cd.tile_count; ++t) bin_tiles.push_back(cd.tile_begin + t);
            if (cd.edge_tile >= 0) bin_tiles.push_back(cd.edge_tile);
        }
        bins.push_back(d);
    }
}

rsv_status build_tiles(rsv_ctx* c, const rsv_leapfrog* lf) {
    for (int s = 0; s < c->pb.n_series; ++s) {
        if (lf[s].n_steps < 1 || lf[s].n_steps > c->pb.max_steps)
            return fail(RSV_EINVAL, "series %d: n_steps %d outside [1, max_steps = %d]", s,
                        lf[s].n_steps, c->pb.max_steps);
        if (!(lf[s].dtau > 0.0) || !std::isfinite(lf[s].dtau))
            return fail(RSV_EINVAL, "series %d: dtau must be finite and > 0", s);
    }
    std::vector<ChainDesc> chains(c->n_chains);
    std::vector<std::vector<TileDesc>> body_of(c->n_chains), edge_of(c->n_chains);
    int64_t n_total = 0;
    for (int s = 0; s < c->pb.n_series; ++s) {
        const int32_t T = static_cast<int32_t>(c->offsets[s + 1] - c->offsets[s]);
        for (int j = 0; j < c->C; ++j) {
            const int32_t ch = s * c->C + j;
            ChainDesc& d = chains[ch];
            d.h_off = c->C * c->offsets[s] + static_cast<int64_t>(j) * T;
            d.d_off = c->offsets[s];
            d.T = T;
            d.series = s;
            if (!tile_chain(ch, T, c->S, c->NW, kicks_for(c->pb.flags, lf[s].n_steps), body_of[ch],
                            edge_of[ch]))
                return fail(RSV_EINVAL, "series %d: n_steps %d too large for a tile", s,
                            lf[s].n_steps);
            d.n_steps = lf[s].n_steps;
            d.dtau = lf[s].dtau;
            n_total += static_cast<int64_t>(body_of[ch].size() + edge_of[ch].size());
        }
    }
    if (n_total > c->lay.max_tiles) return fail(RSV_ENOMEM, "tile count exceeds the workspace");
    // two groups of about half the tiles each when there is a side stream and
    // more than one chain; otherwise one
    c->split = c->n_chains;
    if (c->side && c->n_chains >= 2) {
        int64_t run = 0;
        int32_t ch = 0;
        while (ch < c->n_chains - 1 && 2 * run < n_total) {
            run += static_cast<int64_t>(body_of[ch].size() + edge_of[ch].size());
            ++ch;
        }
        c->split = std::max<int32_t>(1, ch);
    }
    // tile list: per group, its edge tiles (slower per site, so they start
    // in the first round) and then its body tiles, chain by chain
    std::vector<TileDesc> tiles;
    tiles.reserve(static_cast<size_t>(n_total));
    c->n_body = c->n_edge = 0;
    for (int g = 0; g < 2; ++g) {
        const int32_t lo = g == 0 ? 0 : c->split, hi = g == 0 ? c->split : c->n_chains;
        c->group_tile_first[g] = static_cast<int32_t>(tiles.size());
        for (int32_t ch = lo; ch < hi; ++ch) {
            chains[ch].edge_tile = edge_of[ch].empty() ? -1 : static_cast<int32_t>(tiles.size());
            for (const TileDesc& t : edge_of[ch]) tiles.push_back(t);
            c->n_edge += static_cast<int32_t>(edge_of[ch].size());
        }
        for (int32_t ch = lo; ch < hi; ++ch) {
            chains[ch].tile_begin = static_cast<int32_t>(tiles.size());
            chains[ch].tile_count = static_cast<int32_t>(body_of[ch].size());
            for (const TileDesc& t : body_of[ch]) tiles.push_back(t);
            c->n_body += static_cast<int32_t>(body_of[ch].size());
        }
        c->group_tiles[g] = static_cast<int32_t>(tiles.size()) - c->group_tile_first[g];
    }
    c->max_tiles_per_chain = 0;
    for (const ChainDesc& d : chains)
        c->max_tiles_per_chain = std::max(c->max_tiles_per_chain, d.tile_count + 1);
    c->n_bins = 0;
    std::vector<BinDesc> bins;
    std::vector<int32_t> bin_chains, bin_tiles;
    if (c->max_tiles_per_chain - 1 <= kBinMaxChainTiles &&
        bin_shape_available(c->pb.precision, c->S, c->NW))
        pack_bins(chains, c->NW == 1 ? 4 : 1, bins, bin_chains, bin_tiles);
    c->h_tiles = std::move(tiles);
    c->h_chains = chains;
    RSV_HIP(hipMemcpyAsync(c->tiles, c->h_tiles.data(), c->h_tiles.size() * sizeof(TileDesc),
                           hipMemcpyHostToDevice, c->stream));
    RSV_HIP(hipMemcpyAsync(c->chains, c->h_chains.data(), c->h_chains.size() * sizeof(ChainDesc),
                           hipMemcpyHostToDevice, c->stream));
    if (!bins.empty()) {
        RSV_HIP(hipMemcpyAsync(c->bins, bins.data(), bins.size() * sizeof(BinDesc),
                               hipMemcpyHostToDevice, c->stream));
        RSV_HIP(hipMemcpyAsync(c->bin_chains, bin_chains.data(),
                               bin_chains.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                               c->stream));
        RSV_HIP(hipMemcpyAsync(c->bin_tiles, bin_tiles.data(), bin_tiles.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, c->stream));
    }
    RSV_HIP(hipStreamSynchronize(c->stream));
    c->n_bins = static_cast<int32_t>(bins.size());
    c->lf.assign(lf, lf + c->pb.n_series);
    return RSV_OK;
}

rsv_status ensure_tiles(rsv_ctx* c, const rsv_leapfrog* lf) {
    if (!lf) return fail(RSV_EINVAL, "leapfrog parameters are NULL");
    bool same = c->lf.size() == static_cast<size_t>(c->pb.n_series);
    for (int s = 0; same && s < c->pb.n_series; ++s)
        same = c->lf[s].n_steps == lf[s].n_steps && c->lf[s].dtau == lf[s].dtau;
    return same ? RSV_OK : build_tiles(c, lf);
}

template <typename R>
TrajArgs<R> traj_args(rsv_ctx* c, uint64_t sweep, const double* p0) {
    TrajArgs<R> a;
    a.tiles = c->tiles;
    a.tile_first = 0;
    a.n_list = 0;
    a.chains = c->chains;
    a.theta = c->theta;
    a.h_a = static_cast<const R*>(c->h);
    a.h_b = static_cast<R*>(c->h_prop);
    a.state_sel = c->accept;
    if constexpr (sizeof(R) == sizeof(double)) {
        a.y2 = reinterpret_cast<const R*>(c->y2_d);
        a.lrv = reinterpret_cast<const R*>(c->pb.log_rv);
    } else {
        a.y2 = reinterpret_cast<const R*>(c->y2_f);
        a.lrv = reinterpret_cast<const R*>(c->lrv_f);
    }
    a.y2_d = c->y2_d;
    a.lrv_d = c->pb.log_rv;
    a.mass_sqrt = c->log_mass ? static_cast<const R*>(c->mass_sqrt) : nullptr;
    a.p0 = p0;
    a.seed = c->pb.seed;
    a.sweep = sweep;
    a.partials = c->partials;
    a.chain_edge = c->edge;
    a.jitter = c->pb.dtau_jitter;
    a.shift = level_moves(c) ? c->shift : nullptr;
    a.acc_sum = nullptr;
    a.acc_sq = nullptr;
    a.h_prev_out = nullptr;
    a.terms = c->pb.terms;
    a.integrator = (c->pb.flags & RSV_FLAG_OMELYAN)       ? kIntOmelyan
                   : (c->pb.flags & RSV_FLAG_FOREST_RUTH) ? kIntForestRuth
                                                          : kIntLeapfrog;
    a.counters = c->counters;
    return a;
}

// A non-finite state or theta found by the kernels of earlier calls: waits
// for the work already on the stream and reads the flag (4 bytes), so the
// call after the one whose kernels found it always reports it.
rsv_status nonfinite_reported(rsv_ctx* c) {
    uint32_t flag = 0;
    RSV_HIP(hipMemcpyAsync(&flag, c->counters + kCntNonfiniteState, sizeof flag,
                           hipMemcpyDeviceToHost, c->stream));
    RSV_HIP(hipStreamSynchronize(c->stream));
    if (flag)
        return fail(RSV_ENONFINITE, "a non-finite value was found in the state or theta; the "
                                    "chains stay at their last accepted state (rsv_hmc_check "
                                    "clears this once the state is finite)");
    return RSV_OK;
}

// Trajectory kernel over tiles [first, first + count) of the list, on `st`.
template <typename R>
rsv_status launch_traj_tiles(rsv_ctx* c, hipStream_t st, int32_t first, int32_t count,
                             uint64_t sweep, const double* p0, float* acc_sum, float* acc_sq,
                             void* h_prev_out) {
    TrajArgs<R> a = traj_args<R>(c, sweep, p0);
    a.acc_sum = acc_sum;
    a.acc_sq = acc_sq;
    a.h_prev_out = static_cast<R*>(h_prev_out);
    const bool mass = c->log_mass != nullptr;
    const bool timed = c->ev_used < c->ev_start.size();
    if (timed) RSV_HIP(hipEventRecord(c->ev_start[c->ev_used], st));
    a.tile_first = first;
    a.n_list = count;
    RSV_HIP(launch_traj(st, c->pb.precision, c->S, c->NW, mass, &a));
    if (timed) {
        RSV_HIP(hipEventRecord(c->ev_stop[c->ev_used], st));
        c->ev_trajectories[c->ev_used++] = 1;
    }
    return RSV_OK;
}

template <typename R>
rsv_status launch_traj_all(rsv_ctx* c, uint64_t sweep, const double* p0, float* acc_sum,
                           float* acc_sq, void* h_prev_out) {
    return launch_traj_tiles<R>(c, c->stream, 0, c->n_body + c->n_edge, sweep, p0, acc_sum,
                                acc_sq, h_prev_out);
}

FinalizeArgs finalize_args(rsv_ctx* c, uint64_t sweep, int do_metropolis, int do_theta) {
    FinalizeArgs f;
    f.chains = c->chains;
    f.chain_first = 0;
    f.n_chains = c->n_chains;
    f.partials = c->partials;
    f.chain_edge = c->edge;
    f.theta = c->theta;
    f.prior = c->pb.prior;
    f.seed = c->pb.seed;
    f.sweep = sweep;
    f.terms = c->pb.terms;
    f.do_metropolis = do_metropolis;
    f.do_theta = do_theta;
    f.log_u = nullptr;
    f.state_sel = c->accept;
    f.delta_h_out = nullptr;
    f.accepted_out = nullptr;
    f.theta_trace = nullptr;
    f.stats_out = nullptr;
    f.counters = c->counters;
    f.level_move = level_moves(c) ? 1 : 0;
    f.shift = level_moves(c) ? c->shift : nullptr;
    f.slices = c->slices;
    f.arrive = c->arrive;
    return f;
}

// acc_sum / acc_sq (or nullptr): accumulators that receive the state this
// trajectory starts from, i.e. the result of the previous sweep.
// h_prev_out (or nullptr): receives the state this trajectory starts from
// (the previous sweep's trace row); h_trace (or nullptr): receives the state
// after this sweep, by a separate gather.
rsv_status run_trajectory(rsv_ctx* c, uint64_t sweep, const double* p0, const double* log_u,
                          double* delta_h, int32_t* accepted, int do_theta, rsv_theta* theta_trace,
                          void* h_trace, double* stats_out, float* acc_sum = nullptr,
                          float* acc_sq = nullptr, void* h_prev_out = nullptr) {
    const rsv_status st =
        c->pb.precision == RSV_F64
            ? launch_traj_all<double>(c, sweep, p0, acc_sum, acc_sq, h_prev_out)
            : launch_traj_all<float>(c, sweep, p0, acc_sum, acc_sq, h_prev_out);
    if (st != RSV_OK) return st;
    FinalizeArgs f = finalize_args(c, sweep, 1, do_theta);
    f.log_u = log_u;
    f.delta_h_out = delta_h;
    f.accepted_out = accepted;
    f.theta_trace = theta_trace;
    f.stats_out = stats_out;
    RSV_HIP(launch_finalize(c->stream, f, c->max_tiles_per_chain));
    if (h_trace)
        RSV_HIP(launch_gather_state(c->stream, c->chains, c->n_chains, c->max_T, c->accept, c->h,
                                    c->h_prop, level_moves(c) ? c->shift : nullptr, h_trace,
                                    c->pb.precision));
    return RSV_OK;
}

// Every sweep of the call in one launch of the resident kernel.
template <typename R>
rsv_status run_bin(rsv_ctx* c, uint64_t first_sweep, int32_t n_sweeps, int update_theta,
                   const rsv_trace* trace) {
    BinArgs<R> ba;
    ba.traj = traj_args<R>(c, first_sweep, nullptr);
    ba.fin = finalize_args(c, first_sweep, 1, update_theta);
    ba.bins = c->bins;
    ba.bin_chains = c->bin_chains;
    ba.bin_tiles = c->bin_tiles;
    ba.n_bins = c->n_bins;
    ba.n_sweeps = n_sweeps;
    ba.reserved = 0;
    ba.first_sweep = first_sweep;
    ba.n_state = c->n_state;
    ba.dh_trace = trace ? trace->delta_h : nullptr;
    ba.acc_trace = trace ? trace->accepted : nullptr;
    ba.theta_trace = trace ? trace->theta : nullptr;
    ba.h_trace = trace ? static_cast<R*>(trace->h) : nullptr;
    const bool acc = trace && (trace->h_batch_sum || trace->h_sq_sum);
    // batch sums as on the per-kernel path: the states of a batch summed in
    // FP32 and added to the caller's FP64 arrays at the end of the batch
    // (squares alone: every 64 sweeps)
    ba.batch_len = (trace && trace->h_batch_sum) ? trace->batch_len : 64;
    ba.acc_sum = acc ? c->acc_f : nullptr;
    ba.acc_sq = acc ? c->acc_f + c->n_state : nullptr;
    ba.batch_sum = trace ? trace->h_batch_sum : nullptr;
    ba.sq_sum = trace ? trace->h_sq_sum : nullptr;
    if (acc) RSV_HIP(launch_flush(c->stream, c->n_state, ba.acc_sum, ba.acc_sq, nullptr, nullptr));
    const bool timed = c->ev_used < c->ev_start.size();
    if (timed) RSV_HIP(hipEventRecord(c->ev_start[c->ev_used], c->stream));
    RSV_HIP(launch_bin(c->stream, c->pb.precision, c->S, c->NW, c->log_mass != nullptr, &ba));
    if (timed) {
        RSV_HIP(hipEventRecord(c->ev_stop[c->ev_used], c->stream));
        c->ev_trajectories[c->ev_used++] = n_sweeps;
    }
    return RSV_OK;
}

// Leave every chain's current state in the caller's buffer.
rsv_status settle(rsv_ctx* c) {
    RSV_HIP(launch_settle(c->stream, c->chains, c->n_chains, c->max_T, c->accept, c->h, c->h_prop,
                          level_moves(c) ? c->shift : nullptr, c->pb.precision));
    return RSV_OK;
}

}  // namespace

extern "C" {

const char* rsv_last_error(void) { return g_last_error.c_str(); }

int64_t rsv_hmc_state_size(const rsv_problem* pb) {
    int64_t n_data = 0, n_state = 0;
    if (check_problem(pb, &n_data, &n_state) != RSV_OK) return 0;
    return n_state;
}

size_t rsv_hmc_workspace_bytes(const rsv_problem* pb) {
    Layout L;
    if (make_layout(pb, &L) != RSV_OK) return 0;
    return L.total;
}

static rsv_status init_impl(rsv_ctx** out, const rsv_problem* pb, void* h, rsv_theta* theta,
                            const float* log_mass, void* workspace, size_t ws_bytes,
                            void* hip_stream, bool two_streams) {
    if (!out) return fail(RSV_EINVAL, "out is NULL");
    *out = nullptr;
    Layout L;
    rsv_status st = make_layout(pb, &L);
    if (st != RSV_OK) return st;
    if (!pb->y || !pb->log_rv || !h || !theta || !workspace)
        return fail(RSV_EINVAL, "y, log_rv, h, theta and workspace must be non-NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
        return fail(RSV_EINVAL, "workspace must be %zu-byte aligned", kAlign);
    if (ws_bytes < L.total)
        return fail(RSV_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);

    rsv_ctx* c = new rsv_ctx();
    c->pb = *pb;
    c->offsets.assign(pb->offsets, pb->offsets + pb->n_series + 1);
    c->pb.offsets = c->offsets.data();
    c->C = pb->chains_per_series;
    c->n_chains = pb->n_series * pb->chains_per_series;
    tile_shape(pb, &c->S, &c->NW);
    c->n_data = c->offsets[pb->n_series];
    c->n_state = c->n_data * c->C;
    for (int s = 0; s < pb->n_series; ++s)
        c->max_T = std::max<int32_t>(c->max_T, static_cast<int32_t>(c->offsets[s + 1] - c->offsets[s]));
    c->h = h;
    c->theta = theta;
    c->log_mass = log_mass;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ws = static_cast<char*>(workspace);
    c->lay = L;
    c->y2_d = reinterpret_cast<double*>(c->ws + L.y2_d);
    if (pb->precision == RSV_F32_MIXED) {
        c->y2_f = reinterpret_cast<float*>(c->ws + L.y2_f);
        c->lrv_f = reinterpret_cast<float*>(c->ws + L.lrv_f);
    }
    c->h_prop = c->ws + L.h_prop;
    c->tiles = reinterpret_cast<TileDesc*>(c->ws + L.tiles);
    c->chains = reinterpret_cast<ChainDesc*>(c->ws + L.chains);
    c->partials = reinterpret_cast<double*>(c->ws + L.partials);
    c->edge = reinterpret_cast<double*>(c->ws + L.edge);
    c->accept = reinterpret_cast<int32_t*>(c->ws + L.accept);
    c->shift = reinterpret_cast<double*>(c->ws + L.shift);
    c->mass_sqrt = c->ws + L.mass_sqrt;
    c->acc_f = reinterpret_cast<float*>(c->ws + L.acc);
    c->counters = reinterpret_cast<uint32_t*>(c->ws + L.counters);
    c->bins = reinterpret_cast<BinDesc*>(c->ws + L.bins);
    c->bin_chains = reinterpret_cast<int32_t*>(c->ws + L.bin_chains);
    c->bin_tiles = reinterpret_cast<int32_t*>(c->ws + L.bin_tiles);
    c->slices = reinterpret_cast<double*>(c->ws + L.slices);
    c->arrive = reinterpret_cast<uint32_t*>(c->ws + L.arrive);

    auto bail = [&](rsv_status s) {
        delete c;
        return s;
    };
#define RSV_HIP_INIT(call)                                                               \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return bail(fail(RSV_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)));      \
    } while (0)

    RSV_HIP_INIT(hipMemsetAsync(c->counters, 0, kNumCounters * sizeof(uint32_t), c->stream));
    RSV_HIP_INIT(hipMemsetAsync(c->arrive, 0, c->n_chains * sizeof(uint32_t), c->stream));
    RSV_HIP_INIT(hipMemsetAsync(c->edge, 0, c->n_chains * kEdge * sizeof(double), c->stream));
    RSV_HIP_INIT(hipMemsetAsync(c->accept, 0, c->n_chains * sizeof(int32_t), c->stream));
    RSV_HIP_INIT(hipMemsetAsync(c->shift, 0, c->n_chains * sizeof(double), c->stream));
    RSV_HIP_INIT(launch_prepare(c->stream, pb->y, pb->log_rv, c->n_data, c->y2_d, c->y2_f,
                                c->lrv_f));
    if (log_mass)
        RSV_HIP_INIT(launch_mass_table(c->stream, log_mass, c->n_data, c->mass_sqrt,
                                       pb->precision));
    RSV_HIP_INIT(launch_validate(c->stream, pb->y, pb->log_rv, c->n_data, h, c->n_state,
                                 pb->precision, c->counters));
    std::vector<rsv_theta> th(c->n_chains);
    RSV_HIP_INIT(hipMemcpyAsync(th.data(), theta, th.size() * sizeof(rsv_theta),
                                hipMemcpyDeviceToHost, c->stream));
    uint32_t cnt[kNumCounters];
    RSV_HIP_INIT(hipMemcpyAsync(cnt, c->counters, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
    RSV_HIP_INIT(hipStreamSynchronize(c->stream));
    if (cnt[kCntNonfiniteData])
        return bail(fail(RSV_EINVAL, "%u non-finite values in y / log_rv", cnt[kCntNonfiniteData]));
    if (cnt[kCntNonfiniteState])
        return bail(fail(RSV_EINVAL, "%u non-finite values in h", cnt[kCntNonfiniteState]));
    for (int32_t i = 0; i < c->n_chains; ++i) {
        const rsv_theta& t = th[i];
        if (!(std::fabs(t.phi) < 1.0) || !(t.sig2_eta > 0.0) || !(t.sig2_u > 0.0) ||
            !std::isfinite(t.mu) || !std::isfinite(t.xi) || !std::isfinite(t.sig2_eta) ||
            !std::isfinite(t.sig2_u))
            return bail(fail(RSV_EINVAL, "chain %d: theta needs |phi| < 1, finite mu, xi and "
                                         "variances > 0", i));
    }
    if (two_streams && c->n_chains >= 2) {
        RSV_HIP_INIT(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        RSV_HIP_INIT(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        RSV_HIP_INIT(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    }
    // an initial decomposition so that the theta update works before any trajectory
    std::vector<rsv_leapfrog> lf0(pb->n_series, rsv_leapfrog{pb->max_steps, 0, 1.0});
    st = build_tiles(c, lf0.data());
    if (st != RSV_OK) return bail(st);
#undef RSV_HIP_INIT
    *out = c;
    return RSV_OK;
}

rsv_status rsv_hmc_init(rsv_ctx** out, const rsv_problem* pb, void* h, rsv_theta* theta,
                        const float* log_mass, void* workspace, size_t ws_bytes,
                        void* hip_stream) {
    return init_impl(out, pb, h, theta, log_mass, workspace, ws_bytes, hip_stream, true);
}

rsv_status rsv_hmc_init_static(rsv_ctx** out, const rsv_problem* pb, void* h, rsv_theta* theta,
                               const float* log_mass, void* hip_stream) {
    if (!out) return fail(RSV_EINVAL, "out is NULL");
    *out = nullptr;
    Layout L;
    rsv_status st = make_layout(pb, &L);
    if (st != RSV_OK) return st;
    if (L.total > RSV_STATIC_WORKSPACE_BYTES)
        return fail(RSV_ENOMEM, "the problem needs %zu bytes of workspace; the static workspace "
                                "holds %zu (use rsv_hmc_init with a caller workspace)",
                    L.total, static_cast<size_t>(RSV_STATIC_WORKSPACE_BYTES));
    int dev = 0;
    RSV_HIP(hipGetDevice(&dev));
    void* ws = nullptr;
    uint64_t gen = 0;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (static_cast<size_t>(dev) >= g_static_ptr.size()) {
            g_static_ptr.resize(dev + 1, nullptr);
            g_static_gen.resize(dev + 1, 0);
        }
        if (!g_static_ptr[dev]) {
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return fail(RSV_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                            hipGetErrorString(e));
            g_static_ptr[dev] = p;
        }
        ws = g_static_ptr[dev];
        // from here on the array is this context's; an older static context
        // on the device is refused even if this initialisation fails
        gen = ++g_static_gen[dev];
    }
    st = init_impl(out, pb, h, theta, log_mass, ws, RSV_STATIC_WORKSPACE_BYTES, hip_stream, false);
    if (st != RSV_OK) return st;
    (*out)->static_dev = dev;
    (*out)->static_gen = gen;
    return RSV_OK;
}

rsv_status rsv_hmc_momenta(rsv_ctx* c, uint64_t sweep, double* p_out) {
    if (rsv_status u = usable(c); u != RSV_OK) return u;
    if (rsv_status nf = nonfinite_reported(c); nf != RSV_OK) return nf;
    if (!p_out) return fail(RSV_EINVAL, "p_out is NULL");
    RSV_HIP(launch_momenta(c->stream, c->chains, c->n_chains, c->max_T,
                           c->log_mass ? c->mass_sqrt : nullptr, c->pb.precision, c->pb.seed,
                           sweep, p_out));
    return RSV_OK;
}

rsv_status rsv_hmc_trajectory(rsv_ctx* c, uint64_t sweep, const rsv_leapfrog* lf,
                              const double* p0, const double* log_u, double* delta_h,
                              int32_t* accepted) {
    if (rsv_status u = usable(c); u != RSV_OK) return u;
    rsv_status st = nonfinite_reported(c);
    if (st != RSV_OK) return st;
    st = ensure_tiles(c, lf);
    if (st != RSV_OK) return st;
    st = run_trajectory(c, sweep, p0, log_u, delta_h, accepted, 0, nullptr, nullptr, nullptr);
    return st != RSV_OK ? st : settle(c);
}

rsv_status rsv_theta_update(rsv_ctx* c, uint64_t sweep, double* suff_stats) {
    if (rsv_status u = usable(c); u != RSV_OK) return u;
    if (rsv_status nf = nonfinite_reported(c); nf != RSV_OK) return nf;
    RSV_HIP(launch_stats(c->stream, c->tiles, c->n_body + c->n_edge, c->chains, c->theta, c->h,
                         c->h_prop, c->accept, level_moves(c) ? c->shift : nullptr, c->y2_d,
                         c->pb.log_rv, c->partials, c->edge, c->pb.precision));
    FinalizeArgs f = finalize_args(c, sweep, 0, 1);
    f.stats_out = suff_stats;
    RSV_HIP(launch_finalize(c->stream, f, c->max_tiles_per_chain));
    return level_moves(c) ? settle(c) : RSV_OK;
}

rsv_status rsv_hmc_sweep(rsv_ctx* c, uint64_t first_sweep, int32_t n_sweeps,
                         const rsv_leapfrog* lf, int32_t update_theta, const rsv_trace* trace) {
    if (rsv_status u = usable(c); u != RSV_OK) return u;
    if (n_sweeps < 0) return fail(RSV_EINVAL, "n_sweeps must be >= 0");
    if (trace && trace->h_batch_sum && trace->batch_len < 1)
        return fail(RSV_EINVAL, "batch_len must be >= 1 with h_batch_sum");
    rsv_status st = nonfinite_reported(c);
    if (st != RSV_OK) return st;
    st = ensure_tiles(c, lf);
    if (st != RSV_OK) return st;
    if (n_sweeps > 0 && c->n_bins > 0 && (c->pb.flags & RSV_FLAG_RESIDENT)) {
        st = c->pb.precision == RSV_F64
                 ? run_bin<double>(c, first_sweep, n_sweeps, update_theta ? 1 : 0, trace)
                 : run_bin<float>(c, first_sweep, n_sweeps, update_theta ? 1 : 0, trace);
        return st != RSV_OK ? st : settle(c);
    }
    const size_t elem = c->pb.precision == RSV_F64 ? sizeof(double) : sizeof(float);
    const bool acc = trace && (trace->h_batch_sum || trace->h_sq_sum);
    // The states of one batch are summed in FP32 buffers of the workspace
    // (half the read-modify-write traffic of FP64 sums, which at tens of
    // millions of states costs more than the trajectory) and added to the
    // caller's FP64 arrays at the end of each batch.
    float* acc_sum_f = c->acc_f;
    float* acc_sq_f = c->acc_f + c->n_state;
    // without batch sums, the squares are flushed every 64 sweeps
    const int32_t bl = (trace && trace->h_batch_sum) ? trace->batch_len : 64;
    // chain groups: two (on the context's stream and the side stream) unless
    // there is one chain, a static context, or kernel timing records are on
    // (each trajectory launch is then timed alone on the context's stream)
    const int n_groups = (c->split < c->n_chains && c->ev_start.empty()) ? 2 : 1;
    int32_t chain_lo[2] = {0, c->split}, chain_hi[2] = {c->split, c->n_chains};
    int32_t tile_lo[2] = {c->group_tile_first[0], c->group_tile_first[1]};
    int32_t tile_n[2] = {c->group_tiles[0], c->group_tiles[1]};
    int64_t state_lo[2] = {0, 0}, state_n[2] = {c->n_state, 0};
    if (n_groups == 2) {
        state_lo[1] = c->h_chains[c->split].h_off;
        state_n[0] = state_lo[1];
        state_n[1] = c->n_state - state_lo[1];
    } else {
        chain_hi[0] = c->n_chains;
        tile_lo[0] = 0;
        tile_n[0] = c->n_body + c->n_edge;
    }
    hipStream_t gst[2] = {c->stream, c->side};
    auto batch_row = [&](int32_t i) -> double* {  // batch-sum row of the state after sweep i
        return trace->h_batch_sum
                   ? trace->h_batch_sum + static_cast<int64_t>(i / trace->batch_len) * c->n_state
                   : nullptr;
    };
    // end of the batch holding sweep i, for group g's states (or zeroing
    // the FP32 buffers, without a row)
    auto flush = [&](int g, double* row, double* sq) -> hipError_t {
        return launch_flush(gst[g], state_n[g], acc_sum_f + state_lo[g], acc_sq_f + state_lo[g],
                            row ? row + state_lo[g] : nullptr, sq ? sq + state_lo[g] : nullptr);
    };
    if (n_groups == 2) {
        RSV_HIP(hipEventRecord(c->ev_fork, c->stream));
        RSV_HIP(hipStreamWaitEvent(c->side, c->ev_fork, 0));
    }
    // the side stream's work is joined back into the context's stream on
    // every way out, so that later calls see it finished
    auto join = [&]() -> hipError_t {
        if (n_groups < 2) return hipSuccess;
        const hipError_t e = hipEventRecord(c->ev_join, c->side);
        if (e != hipSuccess) return e;
        return hipStreamWaitEvent(c->stream, c->ev_join, 0);
    };
    auto body = [&]() -> rsv_status {
        for (int g = 0; acc && n_sweeps > 0 && g < n_groups; ++g)
            RSV_HIP(flush(g, nullptr, nullptr));
        for (int32_t i = 0; i < n_sweeps; ++i) {
            const uint64_t sweep = first_sweep + static_cast<uint64_t>(i);
            const int64_t ofs = static_cast<int64_t>(i) * c->n_chains;
            double* dh = (trace && trace->delta_h) ? trace->delta_h + ofs : nullptr;
            int32_t* ac = (trace && trace->accepted) ? trace->accepted + ofs : nullptr;
            rsv_theta* tt = (trace && trace->theta) ? trace->theta + ofs : nullptr;
            // the trajectory of sweep i accumulates the state after sweep i - 1
            // and writes it to that sweep's trace row; the last row is gathered
            const bool add = acc && i > 0;
            void* prev_row = (trace && trace->h && i > 0)
                                 ? static_cast<char*>(trace->h) +
                                       static_cast<size_t>(i - 1) * c->n_state * elem
                                 : nullptr;
            for (int g = 0; g < n_groups; ++g) {
                const rsv_status st_g =
                    c->pb.precision == RSV_F64
                        ? launch_traj_tiles<double>(c, gst[g], tile_lo[g], tile_n[g], sweep,
                                                    nullptr, add ? acc_sum_f : nullptr,
                                                    add ? acc_sq_f : nullptr, prev_row)
                        : launch_traj_tiles<float>(c, gst[g], tile_lo[g], tile_n[g], sweep,
                                                   nullptr, add ? acc_sum_f : nullptr,
                                                   add ? acc_sq_f : nullptr, prev_row);
                if (st_g != RSV_OK) return st_g;
                FinalizeArgs f = finalize_args(c, sweep, 1, update_theta ? 1 : 0);
                f.chain_first = chain_lo[g];
                f.n_chains = chain_hi[g] - chain_lo[g];
                f.delta_h_out = dh;
                f.accepted_out = ac;
                f.theta_trace = tt;
                RSV_HIP(launch_finalize(gst[g], f, c->max_tiles_per_chain));
                if (add && (i - 1) % bl == bl - 1)
                    RSV_HIP(flush(g, batch_row(i - 1), trace->h_sq_sum));
            }
        }
        return RSV_OK;
    };
    const rsv_status st_body = body();
    const hipError_t e_join = join();
    if (st_body != RSV_OK) return st_body;
    if (e_join != hipSuccess)
        return fail(RSV_EDEVICE, "joining the side stream: %s", hipGetErrorString(e_join));
    if (trace && trace->h && n_sweeps > 0)  // the state after the last sweep
        RSV_HIP(launch_gather_state(c->stream, c->chains, c->n_chains, c->max_T, c->accept, c->h,
                                    c->h_prop, level_moves(c) ? c->shift : nullptr,
                                    static_cast<char*>(trace->h) +
                                        static_cast<size_t>(n_sweeps - 1) * c->n_state * elem,
                                    c->pb.precision));
    if (acc && n_sweeps > 0) {  // the state after the last sweep, and its batch
        RSV_HIP(launch_accumulate(c->stream, c->chains, c->n_chains, c->max_T, c->accept, c->h,
                                  c->h_prop, level_moves(c) ? c->shift : nullptr, acc_sum_f,
                                  acc_sq_f, c->pb.precision));
        RSV_HIP(launch_flush(c->stream, c->n_state, acc_sum_f, acc_sq_f, batch_row(n_sweeps - 1),
                             trace->h_sq_sum));
    }
    return settle(c);
}

rsv_status rsv_hmc_check(rsv_ctx* c, int64_t* n_nonfinite) {
    if (rsv_status u = usable(c); u != RSV_OK) return u;
    RSV_HIP(hipMemsetAsync(c->counters + kCntNonfiniteState, 0, sizeof(uint32_t), c->stream));
    RSV_HIP(launch_count_nonfinite(c->stream, c->h, c->n_state, c->pb.precision,
                                   c->counters + kCntNonfiniteState));
    uint32_t cnt[kNumCounters];
    RSV_HIP(hipMemcpyAsync(cnt, c->counters, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
    RSV_HIP(hipStreamSynchronize(c->stream));
    RSV_HIP(hipMemsetAsync(c->counters + kCntNonfiniteDH, 0, sizeof(uint32_t), c->stream));
    if (n_nonfinite) *n_nonfinite = cnt[kCntNonfiniteDH];
    if (cnt[kCntNonfiniteState])
        return fail(RSV_ENONFINITE, "%u non-finite values in the state", cnt[kCntNonfiniteState]);
    return RSV_OK;
}

rsv_status rsv_hmc_profile(rsv_ctx* c, int32_t max_records) {
    if (rsv_status u = usable(c); u != RSV_OK) return u;
    if (max_records < 0) return fail(RSV_EINVAL, "max_records must be >= 0");
    for (hipEvent_t e : c->ev_start) RSV_HIP(hipEventDestroy(e));
    for (hipEvent_t e : c->ev_stop) RSV_HIP(hipEventDestroy(e));
    c->ev_start.clear();
    c->ev_stop.clear();
    c->ev_used = 0;
    for (int32_t i = 0; i < max_records; ++i) {
        hipEvent_t a, b;
        RSV_HIP(hipEventCreate(&a));
        RSV_HIP(hipEventCreate(&b));
        c->ev_start.push_back(a);
        c->ev_stop.push_back(b);
    }
    c->ev_trajectories.assign(max_records, 0);
    return RSV_OK;
}

rsv_status rsv_hmc_kernel_time(rsv_ctx* c, double* total_ms, int64_t* n_records) {
    if (rsv_status u = usable(c); u != RSV_OK) return u;
    double sum = 0.0;
    int64_t n = 0;
    if (c->ev_used > 0) RSV_HIP(hipEventSynchronize(c->ev_stop[c->ev_used - 1]));
    for (size_t i = 0; i < c->ev_used; ++i) {
        float ms = 0.f;
        RSV_HIP(hipEventElapsedTime(&ms, c->ev_start[i], c->ev_stop[i]));
        sum += ms;
        n += c->ev_trajectories[i];
    }
    if (total_ms) *total_ms = sum;
    if (n_records) *n_records = n;
    c->ev_used = 0;
    return RSV_OK;
}

rsv_status rsv_hmc_destroy(rsv_ctx* c) {
    delete c;
    return RSV_OK;
}

}  // extern "C"
