// batch.hip -- batch entry points of the C-ABI in include/lbmx.h: many
// cavities of uneven size, Rayleigh number and wall type advanced together by
// one kernel launch per time step (k_step_batch), replayed from a captured
// hipGraph, with converged cavities retired from the work list and the launch
// shape chosen by a timing autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "batch.hpp"
#include "host.hpp"

using namespace lbmx;
using namespace lbmx::host;

namespace {

enum : int32_t { ST_ACTIVE = 0, ST_CONVERGED = 1, ST_MAXSTEPS = 2, ST_UNSTABLE = 3 };

}  // namespace

struct lbmx_batch {
    int count = 0;
    int32_t storage = LBMX_F32;
    int32_t force_model = LBMX_FORCE_EQ15;  // shared by all cavities
    std::vector<lbmx_params> p;
    std::vector<Derived> d;
    std::vector<Layout> L;
    std::vector<size_t> off;       // byte offset of cavity k's first lattice
    std::vector<size_t> scr;       // byte offset of cavity k's Nu scratch (4 n + 8 doubles)
    std::vector<int> cur;          // lattice holding cavity k's current state
    std::vector<int32_t> state;    // ST_*
    std::vector<int64_t> t;
    std::vector<lbmx_nu> last;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    void *d_cavs = nullptr;
    Tile *d_tiles = nullptr;
    size_t tiles_cap = 0;
    uint32_t ntiles = 0;
    int parity = 0;                // lattice index of every active cavity
    uint32_t *d_t = nullptr;       // per-cavity step counters, 2 x count (k_step_batch)
    int block = 256;               // threads per block = nodes per tile
    int grid = 0;                  // blocks; 0 = one per tile
    int graph_steps = 64;          // steps per captured graph; 0 = direct launches
    hipGraphExec_t gexec = nullptr;
    int gparity = -1;              // parity the graph was captured from
    int gsteps = 0;
    uint32_t gtiles = 0;
    int cus = 256;
};

namespace {

// Cavity k's current lattice; the other one is spare between launches (the
// next step of an active cavity overwrites it; a retired cavity's is idle).
View view_of(lbmx_batch *b, int k)
{
    const lbmx_params &p = b->p[k];
    char *base = b->ws + b->off[k];
    const size_t lat = b->L[k].lattice;
    return make_view(base + (size_t)b->cur[k] * lat, base + (size_t)(1 - b->cur[k]) * lat, lat, p,
                     b->d[k], true, b->stream);
}

double *scratch_of(lbmx_batch *b, int k) { return reinterpret_cast<double *>(b->ws + b->scr[k]); }

void drop_graph(lbmx_batch *b)
{
    if (b->gexec)
        (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->gparity = -1;
}

// Cavity table for the kernels (depends on the arithmetic type only).
template <class St>
lbmx_status upload_cavs(lbmx_batch *b)
{
    using T = typename St::T;
    std::vector<BatchCav<T>> h(b->count);
    for (int k = 0; k < b->count; ++k) {
        BatchCav<T> &c = h[k];
        c.lat[0] = b->ws + b->off[k];
        c.lat[1] = b->ws + b->off[k] + b->L[k].lattice;
        c.geo = geometry<St>(make_view(c.lat[0], c.lat[1], b->L[k].lattice, b->p[k], b->d[k], true,
                                       b->stream));
        c.rates = make_rates<T>(&b->p[k], b->d[k]);
        c.cells = uint32_t(b->p[k].n) * b->p[k].n * b->p[k].n;
        c.inv_n = 1.0f / float(b->p[k].n);
    }
    if (b->d_cavs)
        (void)hipFree(b->d_cavs);
    b->d_cavs = nullptr;
    HIP_TRY(hipMalloc(&b->d_cavs, sizeof(BatchCav<T>) * b->count));
    HIP_TRY(hipMemcpy(b->d_cavs, h.data(), sizeof(BatchCav<T>) * b->count, hipMemcpyHostToDevice));
    return LBMX_OK;
}

// Work list of the active cavities, tiles of b->block nodes.
lbmx_status build_tiles(lbmx_batch *b)
{
    std::vector<Tile> tiles;
    for (int k = 0; k < b->count; ++k) {
        if (b->state[k] != ST_ACTIVE)
            continue;
        const uint32_t cells = uint32_t(b->p[k].n) * b->p[k].n * b->p[k].n;
        for (uint32_t s = 0; s < cells; s += uint32_t(b->block))
            tiles.push_back(Tile{uint32_t(k), s});
    }
    drop_graph(b);
    b->ntiles = uint32_t(tiles.size());
    if (tiles.empty())
        return LBMX_OK;
    if (tiles.size() > b->tiles_cap) {
        if (b->d_tiles)
            (void)hipFree(b->d_tiles);
        b->d_tiles = nullptr;
        b->tiles_cap = 0;
        HIP_TRY(hipMalloc(&b->d_tiles, sizeof(Tile) * tiles.size()));
        b->tiles_cap = tiles.size();
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    HIP_TRY(hipMemcpy(b->d_tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice));
    return LBMX_OK;
}

unsigned grid_blocks(const lbmx_batch *b)
{
    if (b->grid <= 0 || uint32_t(b->grid) > b->ntiles)
        return b->ntiles;
    return unsigned(b->grid);
}

template <class St>
lbmx_status launch_direct(lbmx_batch *b, int64_t nsteps)
{
    using T = typename St::T;
    const auto *cavs = reinterpret_cast<const BatchCav<T> *>(b->d_cavs);
    for (int64_t s = 0; s < nsteps; ++s) {
        const uint32_t *t_in = b->d_t + (size_t)b->parity * b->count;
        uint32_t *t_out = b->d_t + (size_t)(b->parity ^ 1) * b->count;
        switch (b->force_model) {
        case LBMX_FORCE_EQ15_RHO:
            hipLaunchKernelGGL((k_step_batch<St, LBMX_FORCE_EQ15_RHO>), dim3(grid_blocks(b)),
                               dim3(b->block), 0, b->stream, cavs, b->d_tiles, b->ntiles, b->parity,
                               t_in, t_out);
            break;
        case LBMX_FORCE_GUO:
            hipLaunchKernelGGL((k_step_batch<St, LBMX_FORCE_GUO>), dim3(grid_blocks(b)),
                               dim3(b->block), 0, b->stream, cavs, b->d_tiles, b->ntiles, b->parity,
                               t_in, t_out);
            break;
        default:
            hipLaunchKernelGGL((k_step_batch<St, LBMX_FORCE_EQ15>), dim3(grid_blocks(b)),
                               dim3(b->block), 0, b->stream, cavs, b->d_tiles, b->ntiles, b->parity,
                               t_in, t_out);
        }
        b->parity ^= 1;
    }
    HIP_TRY(hipGetLastError());
    return LBMX_OK;
}

// Cavity k restarts at step 0: its device step counter read by the next
// launch (the batch's current parity) is cleared.
lbmx_status reset_step(lbmx_batch *b, int k)
{
    static const uint32_t kZero = 0;
    HIP_TRY(hipMemcpyAsync(b->d_t + (size_t)b->parity * b->count + k, &kZero, sizeof kZero,
                           hipMemcpyHostToDevice, b->stream));
    return LBMX_OK;
}

// Capture graph_steps launches (an even number, so a replay ends on the
// parity it started from) into an executable graph.
template <class St>
lbmx_status capture(lbmx_batch *b)
{
    drop_graph(b);
    const int p0 = b->parity;
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    lbmx_status s = launch_direct<St>(b, b->graph_steps);
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    b->parity = p0;
    if (s != LBMX_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess)
        return fail(LBMX_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->gexec = nullptr;
        return fail(LBMX_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    b->gparity = p0;
    b->gsteps = b->graph_steps;
    b->gtiles = b->ntiles;
    return LBMX_OK;
}

template <class St>
lbmx_status advance(lbmx_batch *b, int64_t nsteps)
{
    if (b->ntiles == 0 || nsteps == 0)
        return LBMX_OK;
    int64_t done = 0;
    if (b->graph_steps > 0) {
        while (nsteps - done >= b->graph_steps) {
            if (!b->gexec || b->gparity != b->parity || b->gsteps != b->graph_steps ||
                b->gtiles != b->ntiles) {
                lbmx_status s = capture<St>(b);
                if (s != LBMX_OK)
                    return s;
            }
            HIP_TRY(hipGraphLaunch(b->gexec, b->stream));
            done += b->graph_steps;
        }
    }
    lbmx_status s = launch_direct<St>(b, nsteps - done);
    if (s != LBMX_OK)
        return s;
    for (int k = 0; k < b->count; ++k)
        if (b->state[k] == ST_ACTIVE) {
            b->t[k] += nsteps;
            b->cur[k] = b->parity;
        }
    return LBMX_OK;
}

lbmx_status check(const lbmx_batch *b, int k)
{
    if (!b)
        return fail(LBMX_EINVAL, "batch handle is NULL");
    if (k < 0 || k >= b->count)
        return fail(LBMX_EINVAL, "cavity index %d outside [0, %d)", k, b->count);
    return LBMX_OK;
}

// Launch the Nu reduction of every cavity in `ks`, then copy all results
// with one synchronisation.
lbmx_status nusselt_many(lbmx_batch *b, const std::vector<int> &ks, std::vector<lbmx_nu> &out)
{
    out.assign(ks.size(), lbmx_nu{});
    std::vector<double> res(4 * ks.size());
    for (size_t i = 0; i < ks.size(); ++i) {
        const int k = ks[i];
        lbmx_status s = LBMX_DISPATCH(b->storage, launch_nu, view_of(b, k), scratch_of(b, k), nullptr);
        if (s != LBMX_OK)
            return s;
        HIP_TRY(hipMemcpyAsync(&res[4 * i], scratch_of(b, k) + 4 * (size_t)b->p[k].n,
                               4 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (size_t i = 0; i < ks.size(); ++i) {
        out[i].nu3d = res[4 * i];
        out[i].nu2d = res[4 * i + 1];
        out[i].numax = res[4 * i + 2];
        out[i].nonfinite = int32_t(res[4 * i + 3]);
        out[i].step = b->t[ks[i]];
    }
    return LBMX_OK;
}

template <class St>
lbmx_status batch_step_t(lbmx_batch *b, int64_t n)
{
    return advance<St>(b, n);
}

template <class St>
lbmx_status batch_upload_t(lbmx_batch *b)
{
    return upload_cavs<St>(b);
}

std::string tune_key(const lbmx_batch *b)
{
    hipDeviceProp_t prop;
    int dev = 0;
    std::string name = "gpu";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        name = prop.gcnArchName;
    size_t cells = 0;
    for (int k = 0; k < b->count; ++k)
        if (b->state[k] == ST_ACTIVE)
            cells += size_t(b->p[k].n) * b->p[k].n * b->p[k].n;
    std::ostringstream os;
    os << name << "|storage" << b->storage << "|cavities" << b->count << "|cells" << cells;
    return os.str();
}

// Cache file: a JSON object, one entry per line:
//   "key": {"block": B, "grid": G, "us_per_step": X},
std::map<std::string, std::vector<double>> read_cache(const char *path)
{
    std::map<std::string, std::vector<double>> m;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        const size_t q0 = line.find('"');
        if (q0 == std::string::npos)
            continue;
        const size_t q1 = line.find('"', q0 + 1);
        if (q1 == std::string::npos)
            continue;
        double bl = 0, gr = 0, us = 0;
        if (std::sscanf(line.c_str() + q1 + 1, ": {\"block\": %lf, \"grid\": %lf, \"us_per_step\": %lf",
                        &bl, &gr, &us) == 3)
            m[line.substr(q0 + 1, q1 - q0 - 1)] = {bl, gr, us};
    }
    return m;
}

void write_cache(const char *path, const std::map<std::string, std::vector<double>> &m)
{
    std::ofstream out(path);
    out << "{\n";
    size_t i = 0;
    for (const auto &kv : m) {
        char buf[160];
        std::snprintf(buf, sizeof(buf), "{\"block\": %d, \"grid\": %d, \"us_per_step\": %.3f}",
                      int(kv.second[0]), int(kv.second[1]), kv.second[2]);
        out << "\"" << kv.first << "\": " << buf << (++i < m.size() ? ",\n" : "\n");
    }
    out << "}\n";
}

}  // namespace

extern "C" {

lbmx_status lbmx_batch_create(const lbmx_params *p, int32_t count, void *stream, lbmx_batch **out)
{
    if (!out)
        return fail(LBMX_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p || count < 1 || count > 65536)
        return fail(LBMX_EINVAL, "need 1 <= count <= 65536 parameter sets");
    lbmx_batch *b = new (std::nothrow) lbmx_batch();
    if (!b)
        return fail(LBMX_ENOMEM, "host allocation failed");
    b->count = count;
    b->storage = p[0].storage;
    b->force_model = p[0].force_model;
    size_t total = 0;
    for (int k = 0; k < count; ++k) {
        Derived d;
        lbmx_status s = derive(&p[k], &d);
        if (s != LBMX_OK) {
            delete b;
            return s;
        }
        if (p[k].storage != b->storage) {
            delete b;
            return fail(LBMX_EINVAL, "cavity %d: all cavities of a batch share one storage", k);
        }
        if (p[k].force_model != b->force_model) {
            delete b;
            return fail(LBMX_EINVAL, "cavity %d: all cavities of a batch share one force model", k);
        }
        if (p[k].n > 255) {
            delete b;
            return fail(LBMX_EINVAL, "cavity %d: batch cavities need n <= 255", k);
        }
        b->p.push_back(p[k]);
        b->d.push_back(d);
        // n <= 255 keeps every lattice under 4 GiB (FP64: 255^3 x 208 B),
        // as the 32-bit byte offsets of k_step_batch require.
        Layout L = layout_of(&p[k]);
        b->L.push_back(L);
        b->off.push_back(total);
        total += 2 * L.lattice;
        b->scr.push_back(total);
        total += align_up(sizeof(double) * (4 * (size_t)p[k].n + 8), 256);
    }
    b->cur.assign(count, 0);
    b->state.assign(count, ST_ACTIVE);
    b->t.assign(count, 0);
    b->last.assign(count, lbmx_nu{});
    b->ws_bytes = total;
    hipError_t e;
    if (stream) {
        b->stream = reinterpret_cast<hipStream_t>(stream);
    } else {
        e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete b;
            return fail(LBMX_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
        }
        b->own_stream = true;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        b->cus = prop.multiProcessorCount;
    void *m = nullptr;
    e = hipMalloc(&m, total);
    if (e != hipSuccess) {
        lbmx_batch_destroy(b);
        return fail(e == hipErrorOutOfMemory ? LBMX_ENOMEM : LBMX_EDEVICE, "hipMalloc(%zu) failed: %s",
                    total, hipGetErrorString(e));
    }
    b->ws = reinterpret_cast<char *>(m);
    e = hipMalloc(&b->d_t, 2 * sizeof(uint32_t) * count);
    if (e == hipSuccess)
        e = hipMemset(b->d_t, 0, 2 * sizeof(uint32_t) * count);
    if (e != hipSuccess) {
        lbmx_batch_destroy(b);
        return fail(LBMX_EDEVICE, "step counters: %s", hipGetErrorString(e));
    }
    lbmx_status s = LBMX_DISPATCH(b->storage, batch_upload_t, b);
    if (s == LBMX_OK)
        s = build_tiles(b);
    for (int k = 0; s == LBMX_OK && k < count; ++k)
        s = LBMX_DISPATCH(b->storage, unstream_rest, view_of(b, k), nullptr);
    if (s == LBMX_OK) {
        e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess)
            s = fail(LBMX_EDEVICE, "init failed: %s", hipGetErrorString(e));
    }
    if (s != LBMX_OK) {
        lbmx_batch_destroy(b);
        return s;
    }
    *out = b;
    return LBMX_OK;
}

void lbmx_batch_destroy(lbmx_batch *b)
{
    if (!b)
        return;
    if (b->stream)
        (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->d_tiles)
        (void)hipFree(b->d_tiles);
    if (b->d_cavs)
        (void)hipFree(b->d_cavs);
    if (b->d_t)
        (void)hipFree(b->d_t);
    if (b->ws)
        (void)hipFree(b->ws);
    if (b->own_stream)
        (void)hipStreamDestroy(b->stream);
    delete b;
}

lbmx_status lbmx_batch_init_rest(lbmx_batch *b, int32_t k, const double *theta0_host)
{
    lbmx_status s = check(b, k);
    if (s != LBMX_OK)
        return s;
    // A re-initialised cavity rejoins the lockstep at the batch's parity.
    b->cur[k] = b->parity;
    s = reset_step(b, k);
    if (s != LBMX_OK)
        return s;
    s = LBMX_DISPATCH(b->storage, rest_from_host, view_of(b, k), theta0_host);
    if (s != LBMX_OK)
        return s;
    b->t[k] = 0;
    b->last[k] = lbmx_nu{};
    if (b->state[k] != ST_ACTIVE) {
        b->state[k] = ST_ACTIVE;
        return build_tiles(b);
    }
    return LBMX_OK;
}

lbmx_status lbmx_batch_step(lbmx_batch *b, int64_t nsteps)
{
    if (!b)
        return fail(LBMX_EINVAL, "batch handle is NULL");
    if (nsteps < 0)
        return fail(LBMX_EINVAL, "nsteps must be >= 0");
    return LBMX_DISPATCH(b->storage, batch_step_t, b, nsteps);
}

lbmx_status lbmx_batch_run_to_steady(lbmx_batch *b, double tol, int64_t every, int64_t max_steps,
                                     int32_t *n_converged)
{
    if (!b)
        return fail(LBMX_EINVAL, "batch handle is NULL");
    if (!(tol > 0) || every < 1 || max_steps < 0)
        return fail(LBMX_EINVAL, "need tol > 0, every >= 1, max_steps >= 0");
    std::vector<int> act;
    for (int k = 0; k < b->count; ++k)
        if (b->state[k] == ST_ACTIVE)
            act.push_back(k);
    std::vector<lbmx_nu> nu;
    lbmx_status s = nusselt_many(b, act, nu);
    if (s != LBMX_OK)
        return s;
    for (size_t i = 0; i < act.size(); ++i)
        b->last[act[i]] = nu[i];
    const std::vector<int64_t> t0 = b->t;
    while (!act.empty()) {
        s = LBMX_DISPATCH(b->storage, batch_step_t, b, every);
        if (s != LBMX_OK)
            return s;
        s = nusselt_many(b, act, nu);
        if (s != LBMX_OK)
            return s;
        bool retired = false;
        std::vector<int> still;
        for (size_t i = 0; i < act.size(); ++i) {
            const int k = act[i];
            const double prev = b->last[k].nu3d;
            b->last[k] = nu[i];
            int32_t st = ST_ACTIVE;
            if (nu[i].nonfinite > 0 || !std::isfinite(nu[i].nu3d))
                st = ST_UNSTABLE;
            else if (std::fabs(nu[i].nu3d - prev) < tol)
                st = ST_CONVERGED;
            else if (b->t[k] - t0[k] >= max_steps)
                st = ST_MAXSTEPS;
            b->state[k] = st;
            if (st == ST_ACTIVE)
                still.push_back(k);
            else
                retired = true;
        }
        act.swap(still);
        if (retired) {
            s = build_tiles(b);
            if (s != LBMX_OK)
                return s;
        }
    }
    int32_t conv = 0;
    bool unstable = false, maxed = false;
    for (int k = 0; k < b->count; ++k) {
        conv += b->state[k] == ST_CONVERGED;
        unstable |= b->state[k] == ST_UNSTABLE;
        maxed |= b->state[k] == ST_MAXSTEPS;
    }
    if (n_converged)
        *n_converged = conv;
    if (unstable)
        return fail(LBMX_EUNSTABLE, "a cavity of the batch diverged");
    if (maxed)
        return fail(LBMX_ENOTCONVERGED, "%d of %d cavities converged", conv, b->count);
    return LBMX_OK;
}

lbmx_status lbmx_batch_info(const lbmx_batch *b, int32_t k, int32_t *state, int64_t *t,
                            lbmx_nu *last)
{
    lbmx_status s = check(b, k);
    if (s != LBMX_OK)
        return s;
    if (state) *state = b->state[k];
    if (t) *t = b->t[k];
    if (last) *last = b->last[k];
    return LBMX_OK;
}

lbmx_status lbmx_batch_nusselt(lbmx_batch *b, int32_t k, lbmx_nu *out)
{
    lbmx_status s = check(b, k);
    if (s != LBMX_OK)
        return s;
    if (!out)
        return fail(LBMX_EINVAL, "out is NULL");
    std::vector<lbmx_nu> nu;
    s = nusselt_many(b, {k}, nu);
    if (s != LBMX_OK)
        return s;
    *out = nu[0];
    if (out->nonfinite > 0 || !std::isfinite(out->nu3d))
        return fail(LBMX_EUNSTABLE, "cavity %d: non-finite Nu", k);
    return LBMX_OK;
}

lbmx_status lbmx_batch_init_from(lbmx_batch *b, int32_t k, lbmx_batch *src, int32_t ks)
{
    lbmx_status s = check(b, k);
    if (s != LBMX_OK)
        return s;
    s = check(src, ks);
    if (s != LBMX_OK)
        return s;
    if (src == b && ks == k)
        return fail(LBMX_EINVAL, "source and destination are the same cavity");
    s = check_same_device(src->ws, b->ws, "batches");
    if (s != LBMX_OK)
        return s;
    // as lbmx_batch_init_rest: the cavity rejoins the lockstep at the batch's parity
    b->cur[k] = b->parity;
    s = reset_step(b, k);
    if (s != LBMX_OK)
        return s;
    s = init_from_state(view_of(b, k), b->storage, view_of(src, ks), src->storage,
                        b->d[k].u_c / src->d[ks].u_c);
    if (s != LBMX_OK)
        return s;
    b->t[k] = 0;
    b->last[k] = lbmx_nu{};
    if (b->state[k] != ST_ACTIVE) {
        b->state[k] = ST_ACTIVE;
        return build_tiles(b);
    }
    return LBMX_OK;
}

lbmx_status lbmx_batch_read_macro(lbmx_batch *b, int32_t k, double *rho, double *ux, double *uy,
                                  double *uz, double *theta)
{
    lbmx_status s = check(b, k);
    if (s != LBMX_OK)
        return s;
    return LBMX_DISPATCH(b->storage, macro_to_host, view_of(b, k), rho, ux, uy, uz, theta);
}

lbmx_status lbmx_batch_resample(lbmx_batch *b, int32_t k, int32_t out_n, float *host_uvwt)
{
    lbmx_status s = check(b, k);
    if (s != LBMX_OK)
        return s;
    if (!host_uvwt || out_n < 1 || out_n > 1024)
        return fail(LBMX_EINVAL, "need host_uvwt != NULL and 1 <= out_n <= 1024");
    const int n = b->p[k].n;
    const size_t cells = size_t(n) * n * n, mc = size_t(out_n) * out_n * out_n;
    DevBuf fields, outb;
    HIP_TRY(hipMalloc(&fields.p, 4 * cells * sizeof(double)));
    HIP_TRY(hipMalloc(&outb.p, 4 * mc * sizeof(float)));
    double *fd = reinterpret_cast<double *>(fields.p);
    s = LBMX_DISPATCH(b->storage, launch_macro, view_of(b, k), nullptr, fd, fd + cells, fd + 2 * cells,
                      fd + 3 * cells);
    if (s != LBMX_OK)
        return s;
    hipLaunchKernelGGL(k_resample, dim3(unsigned((mc + 255) / 256)), dim3(256), 0, b->stream, fd, n, 4,
                       reinterpret_cast<float *>(outb.p), out_n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(host_uvwt, outb.p, 4 * mc * sizeof(float), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return LBMX_OK;
}

lbmx_status lbmx_batch_set_launch(lbmx_batch *b, int32_t block, int32_t grid, int32_t graph_steps)
{
    if (!b)
        return fail(LBMX_EINVAL, "batch handle is NULL");
    if (block < 64 || block > 1024 || block % 64 != 0)
        return fail(LBMX_EINVAL, "block = %d: need a multiple of 64 in [64, 1024]", block);
    if (grid < 0 || graph_steps < 0 || graph_steps % 2 != 0)
        return fail(LBMX_EINVAL, "need grid >= 0 and an even graph_steps >= 0");
    const bool retile = block != b->block;
    b->block = block;
    b->grid = grid;
    b->graph_steps = graph_steps;
    drop_graph(b);
    return retile ? build_tiles(b) : LBMX_OK;
}

lbmx_status lbmx_batch_get_launch(const lbmx_batch *b, int32_t *block, int32_t *grid,
                                  int32_t *graph_steps)
{
    if (!b)
        return fail(LBMX_EINVAL, "batch handle is NULL");
    if (block) *block = b->block;
    if (grid) *grid = b->grid;
    if (graph_steps) *graph_steps = b->graph_steps;
    return LBMX_OK;
}

lbmx_status lbmx_batch_autotune(lbmx_batch *b, const char *cache_path, double *us_per_step)
{
    if (!b)
        return fail(LBMX_EINVAL, "batch handle is NULL");
    const std::string key = tune_key(b);
    std::map<std::string, std::vector<double>> cache;
    if (cache_path) {
        cache = read_cache(cache_path);
        auto it = cache.find(key);
        if (it != cache.end()) {
            if (us_per_step) *us_per_step = it->second[2];
            return lbmx_batch_set_launch(b, int(it->second[0]), int(it->second[1]), b->graph_steps);
        }
    }
    const int keep_graph = b->graph_steps;
    const int blocks[] = {128, 256, 512, 1024};
    const int grids[] = {0, 2 * b->cus, 4 * b->cus, 8 * b->cus, 16 * b->cus};
    double best = 1e300;
    int bb = b->block, bg = b->grid;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    lbmx_status s = LBMX_OK;
    for (int bl : blocks) {
        for (int gr : grids) {
            s = lbmx_batch_set_launch(b, bl, gr, 0);
            if (s == LBMX_OK)
                s = LBMX_DISPATCH(b->storage, batch_step_t, b, 4);
            if (s != LBMX_OK)
                break;
            hipError_t e = hipEventRecord(e0, b->stream);
            if (e == hipSuccess)
                s = LBMX_DISPATCH(b->storage, batch_step_t, b, 20);
            if (e == hipSuccess)
                e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess)
                e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess)
                e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess)
                s = fail(LBMX_EDEVICE, "autotune timing failed: %s", hipGetErrorString(e));
            if (s != LBMX_OK)
                break;
            const double us = 1e3 * ms / 20.0;
            if (us < best) {
                best = us;
                bb = bl;
                bg = gr;
            }
        }
        if (s != LBMX_OK)
            break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != LBMX_OK)
        return s;
    // The timing steps advanced the cavities: put every cavity back at rest.
    for (int k = 0; k < b->count; ++k) {
        b->cur[k] = b->parity;
        s = reset_step(b, k);
        if (s != LBMX_OK)
            return s;
        s = LBMX_DISPATCH(b->storage, unstream_rest, view_of(b, k), nullptr);
        if (s != LBMX_OK)
            return s;
        b->t[k] = 0;
        b->last[k] = lbmx_nu{};
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    s = lbmx_batch_set_launch(b, bb, bg, keep_graph);
    if (s != LBMX_OK)
        return s;
    if (cache_path) {
        cache[key] = {double(bb), double(bg), best};
        write_cache(cache_path, cache);
    }
    if (us_per_step)
        *us_per_step = best;
    return LBMX_OK;
}

}  // extern "C"
