// Allocation-free scorer training: tpc_mlp_train_noalloc.
//
// Some callers cannot allocate device memory at call time (work under HIP graph
// capture, tight training or serving loops, harnesses that forbid it).  This entry
// point runs the same kernels as tpc_mlp_train, but its two scratch buffers -- the
// packed BF16 weight fragments and the per-block partial gradients -- live in one
// fixed file-scope device array instead of the context's growable scratch.
//
// The array's name is a host-side stand-in in host code; its device address is
// looked up once per device (hipGetSymbolAddress, with that device current) when
// the first context on that device is created, and only that address reaches the
// kernels.  Each device holds its own copy for the life of the process.  Every
// call on one device shares it and leaves the last call's contents behind: the
// packed weights are rewritten at the start of every call and every partial
// gradient is written in full by its block before it is read, so nothing has to
// start at zero.  Calls on one device whose work overlaps (other streams, other
// contexts or threads) race on the array.
#include <mutex>

#include "tpc_internal.h"

namespace tpc {

namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kPartOff = (kMlpQBytes + 255) / 256 * 256;
constexpr size_t kPartBytes =
    (size_t)((kMlpMaxBatch + kMlpTrainChunk - 1) / kMlpTrainChunk) * (TPC_MLP_N_PARAMS + 1) * sizeof(float);
constexpr size_t kScratchBytes = kPartOff + kPartBytes;
static_assert(kScratchBytes == TPC_MLP_NOALLOC_SCRATCH_BYTES && kMlpMaxBatch == TPC_MLP_NOALLOC_MAX_BATCH,
              "sizes stated in the header");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
bool g_looked_up[kMaxDevices];
void* g_addr[kMaxDevices];
hipError_t g_err[kMaxDevices];

}  // namespace

void noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_looked_up[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_err[device] = e;
    g_addr[device] = e == hipSuccess ? p : nullptr;
    g_looked_up[device] = true;
}

void* noalloc_scratch(int device, hipError_t* err) {
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_looked_up[device]) {
        *err = hipErrorNotInitialized;
        return nullptr;
    }
    *err = g_err[device];
    return g_addr[device];
}

size_t noalloc_scratch_bytes() { return kScratchBytes; }

}  // namespace tpc

using namespace tpc;

extern "C" int tpc_mlp_train_noalloc(tpc_ctx_t* c, const float* feats, const uint8_t* labels, const int32_t* order,
                                     const tpc_train_cfg_t* cfg, float* mlp, float* m, float* v, float* loss,
                                     void* stream) {
    if (!c) return TPC_ERR_ARG;
    c->err.clear();
    if (!cfg || cfg->batch < 1 || cfg->n_steps < 0 || cfg->step0 < 0 || !feats || !labels || !order || !mlp ||
        !m || !v || !loss || !(cfg->lr > 0.f) || !(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) ||
        !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) || !(cfg->eps > 0.f))
        return fail(c, TPC_ERR_ARG, "bad training arguments");
    if (cfg->batch > kMlpMaxBatch)
        return fail(c, TPC_ERR_ARG,
                    "batch " + std::to_string(cfg->batch) + " exceeds the allocation-free maximum of " +
                        std::to_string(kMlpMaxBatch) + " rows (its fixed scratch holds " +
                        std::to_string(kScratchBytes) + " bytes)");
    TPC_HIP(c, hipSetDevice(c->device));
    hipError_t e = hipSuccess;
    unsigned char* base = (unsigned char*)noalloc_scratch(c->device, &e);
    if (!base)
        return fail(c, TPC_ERR_HIP, std::string("device address of the fixed scratch: ") + hipGetErrorString(e));
    float* q = (float*)base;
    float* part = (float*)(base + kPartOff);
    hipStream_t st = (hipStream_t)stream;
    mlp_quantize(mlp, q, st);
    for (int k = 0; k < cfg->n_steps; ++k) {
        mlp_grad_step(q, feats, labels, order + (size_t)k * cfg->batch, cfg->batch, part, st);
        mlp_reduce(part, cfg->batch, nullptr, loss + k, mlp, m, v, cfg->step0 + k + 1, cfg->lr, cfg->beta1, cfg->beta2,
                   cfg->eps, st);
        mlp_quantize(mlp, q, st);
    }
    TPC_HIP(c, hipGetLastError());
    return TPC_OK;
}
