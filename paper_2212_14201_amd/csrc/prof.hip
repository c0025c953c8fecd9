// Per-launch kernel timing with HIP events recorded on the state's stream.
// Off by default; when on, every launch the library makes for a state is
// bracketed by two events, and qvm_profile_end aggregates the durations and
// the algorithmic bytes and flops per kernel class.
#include <hip/hip_runtime.h>

#include <cstring>

#include "internal.hpp"

namespace qvm {

static const char* kProfNames[PK_COUNT] = {"dense1", "dense2", "dense3", "diag", "phase",
                                           "swappair", "tile", "basis", "rdm1"};

int prof_begin(qvm_sv* sv) {
    if (!sv->prof.on) return -1;
    Prof& P = sv->prof;
    const size_t need = 2 * (P.recs.size() + 1);
    while (P.events.size() < need) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        P.events.push_back(e);
    }
    const int ev = (int)(2 * P.recs.size());
    if (hipEventRecord(P.events[ev], sv->stream) != hipSuccess) return -1;
    return ev;
}

void prof_end(qvm_sv* sv, int token, int kind, double bytes, double flops) {
    if (token < 0) return;
    Prof& P = sv->prof;
    if (hipEventRecord(P.events[token + 1], sv->stream) != hipSuccess) return;
    P.recs.push_back(ProfRec{kind, token, bytes, flops});
}

}  // namespace qvm

using namespace qvm;

extern "C" {

qvm_status qvm_profile_begin(qvm_sv* sv) {
    if (!sv) return fail(QVM_EARG, "NULL state handle");
    sv->prof.recs.clear();
    sv->prof.on = true;
    return QVM_OK;
}

qvm_status qvm_profile_end(qvm_sv* sv, qvm_kernel_stat* out, int32_t max, int32_t* count) {
    if (!sv) return fail(QVM_EARG, "NULL state handle");
    Prof& P = sv->prof;
    P.on = false;
    QVM_HIP(sv, hipStreamSynchronize(sv->stream));
    qvm_kernel_stat agg[PK_COUNT];
    memset(agg, 0, sizeof(agg));
    for (int k = 0; k < PK_COUNT; ++k) strncpy(agg[k].name, kProfNames[k], sizeof(agg[k].name) - 1);
    P.last_ms.clear();
    P.last_kind.clear();
    for (const ProfRec& r : P.recs) {
        float ms = 0;
        QVM_HIP(sv, hipEventElapsedTime(&ms, P.events[r.ev], P.events[r.ev + 1]));
        P.last_ms.push_back(ms);
        P.last_kind.push_back(r.kind);
        qvm_kernel_stat& a = agg[r.kind];
        a.launches += 1;
        a.total_ms += ms;
        a.bytes += r.bytes;
        a.flops += r.flops;
    }
    P.recs.clear();
    int32_t n = 0;
    for (int k = 0; k < PK_COUNT; ++k)
        if (agg[k].launches) {
            if (out && n < max) out[n] = agg[k];
            ++n;
        }
    if (count) *count = n;
    return QVM_OK;
}

qvm_status qvm_profile_launches(const qvm_sv* sv, double* ms, int32_t* kind, int32_t max,
                                int32_t* count) {
    if (!sv) return fail(QVM_EARG, "NULL state handle");
    const Prof& P = sv->prof;
    const int32_t n = (int32_t)P.last_ms.size();
    if (count) *count = n;
    for (int32_t i = 0; i < n && i < max; ++i) {
        if (ms) ms[i] = P.last_ms[i];
        if (kind) kind[i] = P.last_kind[i];
    }
    return QVM_OK;
}

}  // extern "C"
