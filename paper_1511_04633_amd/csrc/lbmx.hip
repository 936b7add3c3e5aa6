// lbmx.hip -- single-cavity entry points of the C-ABI in include/lbmx.h.
//
// Li, Yang & Zhang (arXiv:1511.04633): parameters in lattice units from
// Sec. 4 (Eq. 38), relaxation rates of Eq. (26) and Sec. 3.2 (Eqs. 35-36),
// cavity types of Sec. 2 (Eqs. 6-10).  All arithmetic of the time step runs
// in the kernels of kernels.hpp; this file validates, allocates, launches
// and copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "host.hpp"

using namespace lbmx;
using namespace lbmx::host;

// Reduction scratch of lbmx_nusselt_noalloc: the 4 per-row partial sums of
// the hot-wall Nu reduction for up to kNoAllocMaxN rows, then the 4 results
// (32.8 KB).  Every GPU the library runs on holds its own copy for the life
// of the process.  In host code this name is not a device address: kernels
// and copies get the address hipGetSymbolAddress returns for the current
// device.
constexpr int kNoAllocMaxN = 1024;
constexpr size_t kScratchDoubles = 4 * size_t(kNoAllocMaxN) + 8;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
thread_local std::string g_last_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

}

namespace lbmx {
namespace host {
lbmx_status fail(lbmx_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}
}  // namespace host
}  // namespace lbmx

struct lbmx_cavity {
    lbmx_params p;
    Derived d;
    Layout L;
    hipStream_t stream;
    bool own_stream;
    char *ws;
    bool own_ws;
    int cur;
    int64_t t;
    int bx, by;
    bool off32;  // a lattice spans < 4 GiB: kernels use 32-bit byte offsets
    // The state is unusable: a Nu evaluation found non-finite values, or a
    // device call failed while the state was being changed.  Stepping,
    // saving and using the cavity as a source return LBMX_ESTATE until an
    // initialisation succeeds.
    bool failed;
};

namespace {

char *lattice(lbmx_cavity *h, int k) { return h->ws + (size_t)k * h->L.lattice; }

double *nu_scratch(lbmx_cavity *h) { return reinterpret_cast<double *>(h->ws + h->L.scratch_off); }

View view(lbmx_cavity *h)
{
    return make_view(lattice(h, h->cur), lattice(h, 1 - h->cur), h->L.lattice, h->p, h->d, h->off32,
                     h->stream);
}

// One row of up to 256 nodes along x per block row; up to 256 threads per
// block (at 256^3, 256 x 1 blocks measured 1% faster than 256 x 2 and 5%
// faster than half-row 128 x 2 blocks).
void default_launch(int n, int *bx, int *by)
{
    *bx = n < 256 ? n : 256;
    int b = 256 / *bx;
    if (b < 1) b = 1;
    if (b > n) b = n;
    *by = b;
}

template <class St, int kForce>
void launch_step_kernels(lbmx_cavity *h, int64_t nsteps)
{
    using T = typename St::T;
    const Geometry<T> geo = geometry<St>(view(h));
    const Rates<T> rates = make_rates<T>(&h->p, h->d);
    const int n = h->p.n;
    dim3 block(h->bx, h->by, 1);
    dim3 grid((n + h->bx - 1) / h->bx, (n + h->by - 1) / h->by, n);
    Geometry<T> g = geo;
    for (int64_t s = 0; s < nsteps; ++s) {
        g.step = uint32_t(h->t);
        if (h->off32)
            hipLaunchKernelGGL((k_step<St, true, kForce>), grid, block, 0, h->stream,
                               lattice(h, h->cur), lattice(h, 1 - h->cur), g, rates);
        else
            hipLaunchKernelGGL((k_step<St, false, kForce>), grid, block, 0, h->stream,
                               lattice(h, h->cur), lattice(h, 1 - h->cur), g, rates);
        h->cur = 1 - h->cur;
        h->t += 1;
    }
}

template <class St>
lbmx_status launch_steps(lbmx_cavity *h, int64_t nsteps)
{
    switch (h->p.force_model) {
    case LBMX_FORCE_EQ15_RHO: launch_step_kernels<St, LBMX_FORCE_EQ15_RHO>(h, nsteps); break;
    case LBMX_FORCE_GUO: launch_step_kernels<St, LBMX_FORCE_GUO>(h, nsteps); break;
    default: launch_step_kernels<St, LBMX_FORCE_EQ15>(h, nsteps);
    }
    HIP_TRY(hipGetLastError());
    return LBMX_OK;
}

lbmx_status check_handle(const lbmx_cavity *h)
{
    if (!h)
        return fail(LBMX_EINVAL, "cavity handle is NULL");
    return LBMX_OK;
}

// As check_handle, and ESTATE for a failed cavity (calls that need a
// usable state: stepping, saving, serving as a source).
lbmx_status check_usable(const lbmx_cavity *h)
{
    lbmx_status s = check_handle(h);
    if (s != LBMX_OK)
        return s;
    if (h->failed)
        return fail(LBMX_ESTATE, "the cavity's state is unusable (diverged or a device call failed); "
                    "initialise it again");
    return LBMX_OK;
}

// Run an initialisation that rewrites the state: the cavity is failed while
// it runs and stays failed if it does not succeed.
template <class Fn>
lbmx_status reinit(lbmx_cavity *h, Fn fn)
{
    h->failed = true;
    lbmx_status s = fn();
    if (s == LBMX_OK)
        h->failed = false;
    return s;
}

// Checkpoint file header (no padding: 8 + 4 + 4 + 336 + 3 x 8 bytes).
constexpr char kCkptMagic[8] = {'L', 'B', 'M', 'X', 'C', 'K', 'P', 'T'};
constexpr uint32_t kCkptVersion = 2;  // 2: fixed-point energy in units of 2^-15 Theta
constexpr size_t kCkptChunk = size_t(64) << 20;  // staging buffer bytes
struct CkptHeader {
    char magic[8];
    uint32_t version;
    uint32_t params_bytes;
    lbmx_params p;
    int64_t t;
    uint64_t lattice_bytes;
    uint64_t slab_nodes;
};
static_assert(sizeof(lbmx_params) == 336, "lbmx_params is expected to have no padding");
static_assert(sizeof(CkptHeader) == 376, "checkpoint header layout");

// The parameter set as it matters to the state: custom rates only if used;
// the Nu stencil only reads the state.
lbmx_params canonical(const lbmx_params &p)
{
    lbmx_params q = p;
    q.nu_stencil = 0;
    if (!q.custom_rates) {
        std::memset(q.s, 0, sizeof q.s);
        std::memset(q.tau, 0, sizeof q.tau);
    }
    return q;
}

struct File {
    FILE *f;
    explicit File(FILE *x) : f(x) {}
    File(const File &) = delete;
    File &operator=(const File &) = delete;
    ~File()
    {
        if (f)
            std::fclose(f);
    }
    FILE *release()
    {
        FILE *x = f;
        f = nullptr;
        return x;
    }
};

struct HostBuf {
    void *p = nullptr;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf()
    {
        if (p)
            (void)hipHostFree(p);
    }
};

}  // namespace

extern "C" {

lbmx_status lbmx_params_default(lbmx_params *p)
{
    if (!p)
        return fail(LBMX_EINVAL, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->n = 16;
    p->wall_type = 1;
    p->ra = 1e3;
    p->pr = 0.71;
    p->ma = 0.1;
    p->theta_hot = 0.5;
    p->theta_cold = -0.5;
    p->theta_ref = 0.0;
    p->buoyancy_scale = 1.0;
    p->storage = LBMX_F32;
    p->custom_rates = 0;
    return LBMX_OK;
}

lbmx_status lbmx_derive(const lbmx_params *p, double *out)
{
    if (!out)
        return fail(LBMX_EINVAL, "out is NULL");
    Derived d;
    lbmx_status s = derive(p, &d);
    if (s != LBMX_OK)
        return s;
    out[0] = d.u_c;
    out[1] = d.gbeta;
    out[2] = d.nu;
    out[3] = d.alpha;
    out[4] = d.s_nu;
    out[5] = d.tau_t;
    return LBMX_OK;
}

lbmx_status lbmx_workspace_bytes(const lbmx_params *p, size_t *bytes)
{
    if (!bytes)
        return fail(LBMX_EINVAL, "bytes is NULL");
    Derived d;
    lbmx_status s = derive(p, &d);
    if (s != LBMX_OK)
        return s;
    *bytes = layout_of(p).total;
    return LBMX_OK;
}

lbmx_status lbmx_bytes_per_cell(int32_t storage, double *bytes)
{
    if (!bytes)
        return fail(LBMX_EINVAL, "bytes is NULL");
    const size_t bf = flow_size(storage), bg = energy_size(storage);
    if (!bf)
        return fail(LBMX_EINVAL, "storage = %d not a lbmx_storage", storage);
    *bytes = 2.0 * double(19 * bf + 7 * bg);
    return LBMX_OK;
}

lbmx_status lbmx_create(const lbmx_params *p, void *dev_workspace, size_t ws_bytes, void *stream,
                        lbmx_cavity **out)
{
    if (!out)
        return fail(LBMX_EINVAL, "out is NULL");
    *out = nullptr;
    Derived d;
    lbmx_status s = derive(p, &d);
    if (s != LBMX_OK)
        return s;
    const Layout L = layout_of(p);
    if (dev_workspace) {
        if (ws_bytes < L.total)
            return fail(LBMX_EINVAL, "workspace of %zu bytes, need %zu", ws_bytes, L.total);
        if (reinterpret_cast<uintptr_t>(dev_workspace) % 256)
            return fail(LBMX_EINVAL, "workspace not 256-byte aligned");
    }
    lbmx_cavity *h = new (std::nothrow) lbmx_cavity();
    if (!h)
        return fail(LBMX_ENOMEM, "host allocation failed");
    h->p = *p;
    h->d = d;
    h->L = L;
    h->cur = 0;
    h->t = 0;
    h->failed = false;
    h->off32 = double(L.lattice) <= 4294967295.0;
    default_launch(p->n, &h->bx, &h->by);
    if (stream) {
        h->stream = reinterpret_cast<hipStream_t>(stream);
        h->own_stream = false;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete h;
            return fail(LBMX_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
        }
        h->own_stream = true;
    }
    if (dev_workspace) {
        h->ws = reinterpret_cast<char *>(dev_workspace);
        h->own_ws = false;
    } else {
        void *m = nullptr;
        hipError_t e = hipMalloc(&m, L.total);
        if (e != hipSuccess) {
            if (h->own_stream)
                (void)hipStreamDestroy(h->stream);
            delete h;
            return fail(e == hipErrorOutOfMemory ? LBMX_ENOMEM : LBMX_EDEVICE,
                        "hipMalloc(%zu) failed: %s", L.total, hipGetErrorString(e));
        }
        h->ws = reinterpret_cast<char *>(m);
        h->own_ws = true;
    }
    s = lbmx_init_rest(h, nullptr);
    if (s != LBMX_OK) {
        lbmx_destroy(h);
        return s;
    }
    *out = h;
    return LBMX_OK;
}

void lbmx_destroy(lbmx_cavity *h)
{
    if (!h)
        return;
    (void)hipStreamSynchronize(h->stream);
    if (h->own_ws)
        (void)hipFree(h->ws);
    if (h->own_stream)
        (void)hipStreamDestroy(h->stream);
    delete h;
}

lbmx_status lbmx_init_rest(lbmx_cavity *h, const double *theta0_host)
{
    lbmx_status s = check_handle(h);
    if (s != LBMX_OK)
        return s;
    return reinit(h, [&]() -> lbmx_status {
        h->cur = 0;
        lbmx_status r = LBMX_DISPATCH(h->p.storage, rest_from_host, view(h), theta0_host);
        if (r == LBMX_OK)
            h->t = 0;
        return r;
    });
}

lbmx_status lbmx_set_populations(lbmx_cavity *h, const double *f_host, const double *g_host,
                                 int64_t t)
{
    lbmx_status s = check_handle(h);
    if (s != LBMX_OK)
        return s;
    if (!f_host || !g_host)
        return fail(LBMX_EINVAL, "population arrays must not be NULL");
    if (t < 0)
        return fail(LBMX_EINVAL, "t must be >= 0");
    return reinit(h, [&]() -> lbmx_status {
        lbmx_status r = LBMX_DISPATCH(h->p.storage, pops_from_host, view(h), f_host, g_host);
        if (r == LBMX_OK)
            h->t = t;
        return r;
    });
}

lbmx_status lbmx_get_populations(lbmx_cavity *h, double *f_host, double *g_host)
{
    lbmx_status s = check_handle(h);
    if (s != LBMX_OK)
        return s;
    return LBMX_DISPATCH(h->p.storage, pops_to_host, view(h), f_host, g_host);
}

lbmx_status lbmx_save(lbmx_cavity *h, const char *path)
{
    lbmx_status s = check_usable(h);
    if (s != LBMX_OK)
        return s;
    if (!path)
        return fail(LBMX_EINVAL, "path is NULL");
    CkptHeader hd;
    std::memset(&hd, 0, sizeof hd);
    std::memcpy(hd.magic, kCkptMagic, sizeof hd.magic);
    hd.version = kCkptVersion;
    hd.params_bytes = sizeof(lbmx_params);
    hd.p = canonical(h->p);
    hd.t = h->t;
    hd.lattice_bytes = h->L.lattice;
    hd.slab_nodes = h->L.slab_nodes;
    File f(std::fopen(path, "wb"));
    if (!f.f)
        return fail(LBMX_EIO, "cannot open %s for writing: %s", path, std::strerror(errno));
    if (std::fwrite(&hd, sizeof hd, 1, f.f) != 1)
        return fail(LBMX_EIO, "writing the header of %s failed", path);
    HostBuf stage;
    const size_t chunk = std::min<size_t>(h->L.lattice, kCkptChunk);
    HIP_TRY(hipHostMalloc(&stage.p, chunk, hipHostMallocDefault));
    const char *lat = lattice(h, h->cur);
    for (size_t off = 0; off < h->L.lattice; off += chunk) {
        const size_t len = std::min(chunk, h->L.lattice - off);
        HIP_TRY(hipMemcpyAsync(stage.p, lat + off, len, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        if (std::fwrite(stage.p, 1, len, f.f) != len)
            return fail(LBMX_EIO, "writing %s failed at byte %zu", path, sizeof hd + off);
    }
    if (std::fclose(f.release()) != 0)
        return fail(LBMX_EIO, "closing %s failed: %s", path, std::strerror(errno));
    return LBMX_OK;
}

lbmx_status lbmx_load(lbmx_cavity *h, const char *path)
{
    lbmx_status s = check_handle(h);
    if (s != LBMX_OK)
        return s;
    if (!path)
        return fail(LBMX_EINVAL, "path is NULL");
    File f(std::fopen(path, "rb"));
    if (!f.f)
        return fail(LBMX_EIO, "cannot open %s: %s", path, std::strerror(errno));
    CkptHeader hd;
    if (std::fread(&hd, sizeof hd, 1, f.f) != 1)
        return fail(LBMX_EIO, "%s is shorter than a checkpoint header", path);
    if (std::memcmp(hd.magic, kCkptMagic, sizeof hd.magic) != 0)
        return fail(LBMX_EINVAL, "%s is not a checkpoint", path);
    if (hd.version != kCkptVersion || hd.params_bytes != sizeof(lbmx_params))
        return fail(LBMX_EINVAL, "%s: checkpoint version %u / parameter size %u, need %u / %zu", path,
                    hd.version, hd.params_bytes, kCkptVersion, sizeof(lbmx_params));
    const lbmx_params mine = canonical(h->p);
    if (std::memcmp(&hd.p, &mine, sizeof mine) != 0)
        return fail(LBMX_EINVAL, "%s was written for another parameter set", path);
    if (hd.lattice_bytes != h->L.lattice || hd.slab_nodes != h->L.slab_nodes || hd.t < 0)
        return fail(LBMX_EINVAL, "%s: lattice of %llu bytes in slabs of %llu nodes at t = %lld, "
                    "need %zu bytes in slabs of %zu", path, (unsigned long long)hd.lattice_bytes,
                    (unsigned long long)hd.slab_nodes, (long long)hd.t, h->L.lattice, h->L.slab_nodes);
    if (std::fseek(f.f, 0, SEEK_END) != 0)
        return fail(LBMX_EIO, "cannot seek in %s", path);
    const long end = std::ftell(f.f);
    if (end < 0 || (unsigned long)end != sizeof hd + h->L.lattice)
        return fail(LBMX_EIO, "%s holds %ld bytes, a checkpoint of this cavity %zu", path, end,
                    sizeof hd + h->L.lattice);
    if (std::fseek(f.f, (long)sizeof hd, SEEK_SET) != 0)
        return fail(LBMX_EIO, "cannot seek in %s", path);
    // Read into the spare lattice and switch to it only once every byte has
    // arrived: a failed read leaves the current state as it was.
    HostBuf stage;
    const size_t chunk = std::min<size_t>(h->L.lattice, kCkptChunk);
    HIP_TRY(hipHostMalloc(&stage.p, chunk, hipHostMallocDefault));
    char *lat = lattice(h, 1 - h->cur);
    for (size_t off = 0; off < h->L.lattice; off += chunk) {
        const size_t len = std::min(chunk, h->L.lattice - off);
        if (std::fread(stage.p, 1, len, f.f) != len)
            return fail(LBMX_EIO, "reading %s failed at byte %zu", path, sizeof hd + off);
        HIP_TRY(hipMemcpyAsync(lat + off, stage.p, len, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    h->cur = 1 - h->cur;
    h->t = hd.t;
    h->failed = false;
    return LBMX_OK;
}

lbmx_status lbmx_init_fields(lbmx_cavity *h, const float *dev_u, const float *dev_v,
                             const float *dev_w, const float *dev_theta, int32_t src_n)
{
    lbmx_status s = check_handle(h);
    if (s != LBMX_OK)
        return s;
    if (!dev_u || !dev_v || !dev_w || !dev_theta)
        return fail(LBMX_EINVAL, "field pointers must not be NULL");
    if (src_n < 1 || src_n > 4096)
        return fail(LBMX_EINVAL, "src_n = %d outside [1, 4096]", src_n);
    return reinit(h, [&]() -> lbmx_status {
        h->cur = 0;
        lbmx_status r = LBMX_DISPATCH(h->p.storage, unstream_fields, view(h), dev_u, dev_v, dev_w,
                                      dev_theta, src_n, 1.0, (const float *)nullptr);
        if (r != LBMX_OK)
            return r;
        HIP_TRY(hipStreamSynchronize(h->stream));
        h->t = 0;
        return LBMX_OK;
    });
}

lbmx_status lbmx_init_from_cavity(lbmx_cavity *dst, lbmx_cavity *src)
{
    lbmx_status s = check_handle(dst);
    if (s != LBMX_OK)
        return s;
    s = check_usable(src);
    if (s != LBMX_OK)
        return s;
    if (src == dst)
        return fail(LBMX_EINVAL, "source and destination are the same cavity");
    s = check_same_device(src->ws, dst->ws, "cavities");
    if (s != LBMX_OK)
        return s;
    return reinit(dst, [&]() -> lbmx_status {
        dst->cur = 0;
        lbmx_status r = init_from_state(view(dst), dst->p.storage, view(src), src->p.storage,
                                        dst->d.u_c / src->d.u_c);
        if (r == LBMX_OK)
            dst->t = 0;
        return r;
    });
}

lbmx_status lbmx_init_from_cavities(lbmx_cavity *dst, lbmx_cavity *a, double wa, lbmx_cavity *b,
                                    double wb)
{
    lbmx_status s = check_handle(dst);
    if (s != LBMX_OK)
        return s;
    if ((s = check_usable(a)) != LBMX_OK || (s = check_usable(b)) != LBMX_OK)
        return s;
    if (a == dst || b == dst || a == b)
        return fail(LBMX_EINVAL, "the two sources and the destination must be three cavities");
    if (!std::isfinite(wa) || !std::isfinite(wb))
        return fail(LBMX_EINVAL, "weights must be finite");
    if ((s = check_same_device(a->ws, dst->ws, "cavities")) != LBMX_OK ||
        (s = check_same_device(b->ws, dst->ws, "cavities")) != LBMX_OK)
        return s;
    return reinit(dst, [&]() -> lbmx_status {
        dst->cur = 0;
        lbmx_status r = init_from_two_states(view(dst), dst->p.storage, view(a), a->p.storage, wa,
                                             dst->d.u_c / a->d.u_c, view(b), b->p.storage, wb,
                                             dst->d.u_c / b->d.u_c);
        if (r == LBMX_OK)
            dst->t = 0;
        return r;
    });
}

lbmx_status lbmx_step(lbmx_cavity *h, int64_t nsteps)
{
    lbmx_status s = check_usable(h);
    if (s != LBMX_OK)
        return s;
    if (nsteps < 0)
        return fail(LBMX_EINVAL, "nsteps must be >= 0");
    s = LBMX_DISPATCH(h->p.storage, launch_steps, h, nsteps);
    if (s != LBMX_OK)
        h->failed = true;
    return s;
}

lbmx_status lbmx_step_timed(lbmx_cavity *h, int64_t nsteps, double *ms)
{
    lbmx_status s = check_usable(h);
    if (s != LBMX_OK)
        return s;
    if (!ms || nsteps < 0)
        return fail(LBMX_EINVAL, "ms is NULL or nsteps < 0");
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    hipError_t e = hipEventRecord(a, h->stream);
    if (e == hipSuccess) {
        s = LBMX_DISPATCH(h->p.storage, launch_steps, h, nsteps);
        e = hipEventRecord(b, h->stream);
    }
    if (e == hipSuccess)
        e = hipEventSynchronize(b);
    float msf = 0.0f;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&msf, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (s != LBMX_OK) {
        h->failed = true;
        return s;
    }
    if (e != hipSuccess)
        return fail(LBMX_EDEVICE, "event timing failed: %s", hipGetErrorString(e));
    *ms = msf;
    return LBMX_OK;
}

lbmx_status lbmx_time(const lbmx_cavity *h, int64_t *t)
{
    lbmx_status s = check_handle(h);
    if (s != LBMX_OK)
        return s;
    if (!t)
        return fail(LBMX_EINVAL, "t is NULL");
    *t = h->t;
    return LBMX_OK;
}

lbmx_status lbmx_read_macro(lbmx_cavity *h, double *rho, double *ux, double *uy, double *uz,
                            double *theta)
{
    lbmx_status s = check_handle(h);
    if (s != LBMX_OK)
        return s;
    return LBMX_DISPATCH(h->p.storage, macro_to_host, view(h), rho, ux, uy, uz, theta);
}

lbmx_status lbmx_nusselt(lbmx_cavity *h, lbmx_nu *out, double *map_host)
{
    lbmx_status s = check_handle(h);
    if (s != LBMX_OK)
        return s;
    if (!out)
        return fail(LBMX_EINVAL, "out is NULL");
    const int n = h->p.n;
    const View v = view(h);
    // the map is staged in the spare lattice (n^2 doubles)
    double *map_dev = map_host ? reinterpret_cast<double *>(v.spare) : nullptr;
    s = LBMX_DISPATCH(h->p.storage, launch_nu, v, nu_scratch(h), map_dev);
    if (s != LBMX_OK)
        return s;
    double res[4];
    HIP_TRY(hipMemcpyAsync(res, nu_scratch(h) + 4 * (size_t)n, sizeof(res), hipMemcpyDeviceToHost,
                           h->stream));
    if (map_host)
        HIP_TRY(hipMemcpyAsync(map_host, map_dev, (size_t)n * n * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    out->nu3d = res[0];
    out->nu2d = res[1];
    out->numax = res[2];
    out->step = h->t;
    out->nonfinite = (int32_t)res[3];
    if (out->nonfinite > 0 || !std::isfinite(res[0])) {
        h->failed = true;
        return fail(LBMX_EUNSTABLE, "%d non-finite local Nu values at t = %lld", out->nonfinite,
                    (long long)h->t);
    }
    return LBMX_OK;
}

lbmx_status lbmx_run_to_steady(lbmx_cavity *h, double tol, int64_t every, int64_t max_steps,
                               lbmx_nu *out)
{
    lbmx_status s = check_usable(h);
    if (s != LBMX_OK)
        return s;
    if (!out || !(tol > 0) || every < 1 || max_steps < 0)
        return fail(LBMX_EINVAL, "need out != NULL, tol > 0, every >= 1, max_steps >= 0");
    const int64_t t0 = h->t;
    s = lbmx_nusselt(h, out, nullptr);
    if (s != LBMX_OK)
        return s;
    double prev = out->nu3d;
    while (h->t - t0 < max_steps) {
        int64_t k = every;
        if (h->t - t0 + k > max_steps)
            k = max_steps - (h->t - t0);
        s = lbmx_step(h, k);
        if (s != LBMX_OK)
            return s;
        s = lbmx_nusselt(h, out, nullptr);
        if (s != LBMX_OK)
            return s;
        if (k == every && std::fabs(out->nu3d - prev) < tol)
            return LBMX_OK;
        prev = out->nu3d;
    }
    return fail(LBMX_ENOTCONVERGED, "no steady Nu within %lld steps", (long long)max_steps);
}

lbmx_status lbmx_set_launch(lbmx_cavity *h, int32_t bx, int32_t by)
{
    lbmx_status s = check_handle(h);
    if (s != LBMX_OK)
        return s;
    if (bx == 0 && by == 0) {
        default_launch(h->p.n, &h->bx, &h->by);
        return LBMX_OK;
    }
    if (bx < 1 || by < 1 || (long)bx * by > 1024)
        return fail(LBMX_EINVAL, "launch (%d, %d) needs bx, by >= 1 and bx*by <= 1024", bx, by);
    h->bx = bx;
    h->by = by;
    return LBMX_OK;
}

lbmx_status lbmx_get_launch(const lbmx_cavity *h, int32_t *bx, int32_t *by)
{
    lbmx_status s = check_handle(h);
    if (s != LBMX_OK)
        return s;
    if (!bx || !by)
        return fail(LBMX_EINVAL, "NULL output");
    *bx = h->bx;
    *by = h->by;
    return LBMX_OK;
}

lbmx_status lbmx_nusselt_noalloc(lbmx_cavity *h, lbmx_nu *out, double *map_host)
{
    lbmx_status s = check_handle(h);
    if (s != LBMX_OK)
        return s;
    if (!out)
        return fail(LBMX_EINVAL, "out is NULL");
    const int n = h->p.n;
    if (n > kNoAllocMaxN)
        return fail(LBMX_EINVAL, "n = %d above the %d rows the static scratch holds", n, kNoAllocMaxN);
    s = check_same_device(h->ws, h->ws, "cavity");
    if (s != LBMX_OK)
        return s;
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(LBMX_EDEVICE, "device %d beyond the %d the library tracks", dev, kMaxDevices);
    double *scr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (!g_scratch_ptr[dev]) {
            void *ptr = nullptr;
            HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            g_scratch_ptr[dev] = reinterpret_cast<double *>(ptr);
        }
        scr = g_scratch_ptr[dev];
    }
    const View v = view(h);
    double *map_dev = map_host ? reinterpret_cast<double *>(v.spare) : nullptr;
    s = LBMX_DISPATCH(h->p.storage, launch_nu, v, scr, map_dev);
    if (s != LBMX_OK)
        return s;
    double res[4];
    HIP_TRY(hipMemcpyAsync(res, scr + 4 * (size_t)n, sizeof(res), hipMemcpyDeviceToHost, h->stream));
    if (map_host)
        HIP_TRY(hipMemcpyAsync(map_host, map_dev, (size_t)n * n * sizeof(double),
                               hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    out->nu3d = res[0];
    out->nu2d = res[1];
    out->numax = res[2];
    out->step = h->t;
    out->nonfinite = (int32_t)res[3];
    if (out->nonfinite > 0 || !std::isfinite(res[0])) {
        h->failed = true;
        return fail(LBMX_EUNSTABLE, "%d non-finite local Nu values at t = %lld", out->nonfinite,
                    (long long)h->t);
    }
    return LBMX_OK;
}

const char *lbmx_strerror(lbmx_status s)
{
    switch (s) {
    case LBMX_OK: return "ok";
    case LBMX_EINVAL: return "invalid argument";
    case LBMX_ENOMEM: return "out of memory";
    case LBMX_EDEVICE: return "HIP runtime error";
    case LBMX_EUNSTABLE: return "non-finite values (run diverged)";
    case LBMX_ENOTCONVERGED: return "not converged within max_steps";
    case LBMX_ESTATE: return "invalid state for this call";
    case LBMX_EIO: return "checkpoint file I/O error";
    default: return "unknown status";
    }
}

const char *lbmx_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
