// sw_noalloc.hip -- the sweep without any device allocation.
//
// sw_sweep_noalloc runs the same phase kernels as sw_sweep (Lin & Zheng,
// Sec. I steps 1-3: bonds and tile labels, border merge, border-root
// resolution, cluster flip) on a caller's spin array, with every buffer of
// the method that is neither an input nor an output -- tile labels, the
// union-find parents, crossing bits, border and flip bitmaps, face labels and
// the replica descriptor -- taken from one static device array.  It is for
// callers that cannot allocate: code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc.
//
// The array lives for the whole process on every device the library runs on.
// Its device address comes from hipGetSymbolAddress, looked up once per
// device with that device current; host code never passes the array's name
// itself to a kernel or a copy (on the host that name is not a device
// address).  Every call on a device shares that device's array, so calls
// that overlap on one device race; each call rewrites everything it reads.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "../../include/sw_api.h"
#include "sw_device.hpp"
#include "sw_internal.hpp"
#include "sw_runtime.hpp"

namespace sw {

// 28 MiB: room for every lattice of up to 2^21 sites (1448^2 in 2D, 128^3 in
// 3D) in the default tile shapes, final labels, ragged tiles and alignment
// included (128^3 with labels takes about 24 MB)
constexpr size_t kScratchBytes = 28u << 20;
constexpr uint64_t kNoallocMaxSites = 1ull << 21;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];   // device address of `scratch`, per device

// the device address of this device's copy of the array (looked up once per
// device, with that device current)
static int scratch_of(int dev, unsigned char** out)
{
    if (dev < 0 || dev >= 64) return fail(SW_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress of the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return SW_OK;
}

__global__ void kput_desc_kernel(SwRep* dst, SwRep v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v;
}

__global__ void kzero_i64_kernel(int64_t* p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

static size_t align256(size_t b) { return (b + 255u) & ~(size_t)255u; }

// carve the descriptor and the per-sweep buffers of h out of base; returns the
// bytes used (the buffers are placed only when base is not null).  The
// border roots' cluster roots (par) are needed only when labels are written.
static size_t carve(SwRep& h, unsigned char* base, SwRep** desc, bool labels)
{
    const size_t n = h.N, nt = (size_t)h.ntiles;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    unsigned char* d = take(sizeof(SwRep));
    h.lab16 = reinterpret_cast<uint16_t*>(take(2 * ((n + 3) & ~(size_t)3)));   // whole groups of 4 sites
    h.par = labels ? reinterpret_cast<int32_t*>(take(4 * n)) : nullptr;
    h.nslots = (uint32_t)(nt * 2 * (size_t)h.ft);
    h.dpar = reinterpret_cast<uint64_t*>(take((size_t)h.nslots * 8));
    h.xbits = reinterpret_cast<uint32_t*>(take(nt * (size_t)h.xwords * 4));
    h.fbits = reinterpret_cast<uint32_t*>(take(nt * (size_t)h.fbw * 4));
    h.bflip = reinterpret_cast<uint32_t*>(take(nt * (size_t)h.fbw * 4));
    h.face = reinterpret_cast<uint16_t*>(take(nt * 2 * (size_t)h.ft * 2));
    if (desc) *desc = reinterpret_cast<SwRep*>(d);
    return off;
}

}  // namespace sw

using namespace sw;

extern "C" int sw_sweep_noalloc(const sw_params* params, int8_t* dev_spins, uint32_t sweep0, int32_t n_sweeps,
                                int64_t* dev_series, int32_t* dev_labels, int32_t* dev_err, void* hip_stream)
{
    int rc = validate_params(params);
    if (rc) return rc;
    if (params->flags & (SW_PCC | SW_PCC_WIND)) return fail(SW_EINVAL, "the allocation-free sweep has no PCC feedback");
    if (params->flags & SW_BITPACK) return fail(SW_EINVAL, "the allocation-free sweep takes int8 spins");
    if (!dev_spins) return fail(SW_EINVAL, "null spin array");
    if (reinterpret_cast<uintptr_t>(dev_spins) & 15u) return fail(SW_EINVAL, "the spin array must be 16-byte aligned");
    if (n_sweeps < 0) return fail(SW_EINVAL, "negative sweep count");
    if ((uint64_t)sweep0 + (uint64_t)n_sweeps > 0xFFFFFFF0ull) return fail(SW_EINVAL, "sweep index overflow");
    const uint64_t nsites = nsites_of(params);
    if (nsites > kNoallocMaxSites)
        return fail(SW_EINVAL, "the allocation-free sweep takes at most 2^21 sites (got %llu)",
                    (unsigned long long)nsites);
    SwRep h;
    std::memset(&h, 0, sizeof(h));
    h.dim = params->dim;
    h.L = params->L;
    h.N = (uint32_t)nsites;
    fill_geometry(h, default_shape(h.dim));
    if (carve(h, nullptr, nullptr, dev_labels != nullptr) > kScratchBytes)
        return fail(SW_EINVAL, "lattice needs more than the %zu scratch bytes", kScratchBytes);
    if (n_sweeps == 0) return SW_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    unsigned char* base = nullptr;
    rc = scratch_of(dev, &base);
    if (rc) return rc;
    SwRep* d = nullptr;
    carve(h, base, &d, dev_labels != nullptr);
    h.spins = dev_spins;
    h.lab32 = dev_labels;
    h.err = dev_err;
    h.flags = (dev_labels ? FLAG_KEEP : 0u) | ((params->flags & SW_OPEN) ? FLAG_OPEN : 0u);
    h.seed = params->seed;
    h.p = (params->p_bond < 0.0) ? -std::expm1(-2.0 * params->J / params->T) : params->p_bond;
    h.thr = threshold_from_p(h.p);
    h.sweep = sweep0;
    h.limit = 0xFFFFFFFFu;
    h.active = 1;
    hipStream_t stream = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(kput_desc_kernel, dim3(1), dim3(64), 0, stream, d, h);
    if (dev_series) {
        const int64_t cnt = 2 * (int64_t)n_sweeps;
        hipLaunchKernelGGL(kzero_i64_kernel, dim3((unsigned)std::min<int64_t>((cnt + 255) / 256, 1024)), dim3(256), 0,
                           stream, dev_series, cnt);
    }
    if (hipGetLastError() != hipSuccess) return fail(SW_EHIP, "set-up kernel launch failed");
    for (int32_t k = 0; k < n_sweeps; ++k) {
        const uint32_t s = sweep0 + (uint32_t)k;
        // E, M of the configuration after sweep s - 1 are summed by K1 of sweep s
        int64_t* em = (dev_series && k > 0) ? dev_series + 2 * (size_t)(k - 1) : nullptr;
        if (launch_k1(h, d, s, em, stream, 0) || launch_k2(h, d, stream, 0) || launch_k3a(h, d, s, stream) ||
            launch_k3(h, d, s, stream, 0))
            return fail(SW_EHIP, "kernel launch failed (sweep %u)", s);
    }
    if (dev_series && launch_measure(h, d, dev_series + 2 * (size_t)(n_sweeps - 1), stream))
        return fail(SW_EHIP, "measurement launch failed");
    return SW_OK;
}
