// c4m_noalloc.hip -- the stepping call for callers that cannot allocate
// device memory: the problem's workspace (padded fields, G_E, temporaries,
// band table, Pade tables, counters) lives in one file-scope device array
// instead of caller memory; the caller passes only its field arrays.
#include <mutex>

#include "c4m_internal.h"

namespace c4m {

// Static scratch: one copy per device the library runs on, held until the
// process ends.  Host code never uses its name as an address (on the host
// the symbol is a stand-in): the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

c4m_status set_error(c4m_status s, const char* msg);   // c4m_host.hip
void problem_set_direct(c4m_problem* p);                // c4m_host.hip

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu[MAX_DEVICES];
void* g_scratch[MAX_DEVICES] = {};

}  // namespace
}  // namespace c4m

using namespace c4m;

extern "C" c4m_status c4m_step_fields_noalloc(const c4m_config* cfg, double* const* fields, int64_t nsteps,
                                              void* hip_stream)
{
    if (!cfg || !fields || nsteps < 0) return set_error(C4M_EINVAL, "null config or fields, or negative step count");
    if (cfg->flags & C4M_FLAG_PROFILE) return set_error(C4M_EINVAL, "profiling creates HIP events: not in the no-allocation call");
    size_t need = 0;
    c4m_status s = c4m_workspace_bytes(cfg, &need);
    if (s != C4M_OK) return s;
    if (need > NOALLOC_SCRATCH_BYTES)
        return set_error(C4M_ENOMEM, "configuration needs more than the 64 MiB static scratch of the no-allocation call");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return set_error(C4M_EDEVICE, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_mu[dev]);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return set_error(C4M_EDEVICE, "hipGetSymbolAddress of the static scratch");
        g_scratch[dev] = ptr;
    }
    // the fields the configuration carries, in c4m_field order
    int ids[9], nf = 0;
    for (int f = 0; f < 9; ++f) {
        const bool lap = f >= C4M_LX;
        if (lap && cfg->lap_mode != C4M_LAP_TRACKED) continue;
        const int comp = lap ? f - C4M_LX : f;
        if (cfg->dim == 2 && comp != C4M_EZ && comp != C4M_HX && comp != C4M_HY) continue;
        ids[nf++] = f;
    }
    for (int i = 0; i < nf; ++i)
        if (!fields[ids[i]]) return set_error(C4M_EINVAL, "a field of the configuration has a null pointer");
    c4m_problem* p = nullptr;
    s = c4m_create(cfg, g_scratch[dev], NOALLOC_SCRATCH_BYTES, hip_stream, &p);
    if (s != C4M_OK) return s;
    problem_set_direct(p);
    for (int i = 0; i < nf && s == C4M_OK; ++i) s = c4m_set_field(p, (c4m_field)ids[i], fields[ids[i]], 1);
    if (s == C4M_OK) s = c4m_step(p, nsteps);
    for (int i = 0; i < nf && s == C4M_OK; ++i) s = c4m_get_field(p, (c4m_field)ids[i], fields[ids[i]], 1);
    if (s == C4M_OK && hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess)
        s = set_error(C4M_EDEVICE, "hipStreamSynchronize");
    c4m_status d = c4m_destroy(p);
    return s != C4M_OK ? s : d;
}
