// Host-side helpers shared by the engine's drivers: status macros, the
// workspace carver, device workspace / descriptor arena / pinned buffers.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "engine.hpp"
#include "sdc_aux.hpp"
#include "sdc.h"

namespace sdc {

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return SDC_ERR_DEVICE; \
    } while (0)
#define CHK(x)                 \
    do {                       \
        int r_ = (x);          \
        if (r_ < 0) return r_; \
    } while (0)

static constexpr double kRhoOneSide = 1e-3;  // see rank_from_rho

// ---------------------------------------------------------------------------
// Workspace and staging
// ---------------------------------------------------------------------------
// Bump allocator over the handle's workspace.  A sizing pass (base null)
// measures; the carving pass must stay within cap, else `overflow` is set and
// the caller refuses to launch anything.
struct Carver {
    char* base;
    size_t cap;
    size_t off = 0;
    bool overflow = false;
    explicit Carver(char* b, size_t c = 0) : base(b), cap(c) {}
    template <class T> T* take(size_t n) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += n * sizeof(T);
        if (base && off > cap) overflow = true;
        return p;
    }
};

inline int ensure_ws(Handle& h, size_t bytes) {
    if (h.budget && bytes > h.budget) return SDC_ERR_NOMEM;
    if (bytes <= h.ws_size) return SDC_OK;
    if (h.no_alloc) return SDC_ERR_NOMEM;
    if (h.ws) {
        HIPCHK(hipStreamSynchronize(h.stream));
        HIPCHK(hipFree(h.ws));
        h.ws = nullptr;
        h.ws_size = 0;
    }
    size_t sz = bytes + bytes / 8 + (1 << 20);
    if (h.budget && sz > h.budget) sz = bytes;
    if (hipMalloc(&h.ws, sz) != hipSuccess) {
        h.ws = nullptr;
        (void)hipGetLastError();
        return SDC_ERR_NOMEM;
    }
    h.ws_size = sz;
    return SDC_OK;
}

inline int ensure_desc(Handle& h, size_t bytes) {
    if (bytes <= h.desc_size) return SDC_OK;
    if (h.no_alloc) return SDC_ERR_NOMEM;
    if (h.desc_d) {
        HIPCHK(hipStreamSynchronize(h.stream));
        HIPCHK(hipFree(h.desc_d));
        HIPCHK(hipHostFree(h.desc_h));
        h.desc_d = h.desc_h = nullptr;
    }
    if (hipMalloc(&h.desc_d, bytes) != hipSuccess) return SDC_ERR_NOMEM;
    if (hipHostMalloc(&h.desc_h, bytes, hipHostMallocDefault) != hipSuccess) return SDC_ERR_NOMEM;
    h.desc_size = bytes;
    h.desc_off = 0;
    h.desc_dirty = 0;
    return SDC_OK;
}

inline int ensure_streams(Handle& h) {
    if (h.qs.crit) return SDC_OK;
    if (h.no_alloc) return SDC_ERR_DEVICE;
    if (hipStreamCreateWithFlags(&h.qs.crit, hipStreamNonBlocking) != hipSuccess) return SDC_ERR_DEVICE;
    if (hipStreamCreateWithFlags(&h.qs.rest, hipStreamNonBlocking) != hipSuccess) return SDC_ERR_DEVICE;
    hipEvent_t* ev[4] = {&h.qs.evP, &h.qs.evR, &h.qs.evE, &h.qs.evD};
    for (hipEvent_t* e : ev)
        if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) return SDC_ERR_DEVICE;
    return SDC_OK;
}
// Stream and events of the graph replay.
inline int ensure_graph_stream(Handle& h) {
    if (h.gstream) return SDC_OK;
    if (h.no_alloc) return SDC_ERR_DEVICE;
    if (hipStreamCreateWithFlags(&h.gstream, hipStreamNonBlocking) != hipSuccess) return SDC_ERR_DEVICE;
    for (hipEvent_t& e : h.gev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return SDC_ERR_DEVICE;
    return SDC_OK;
}
inline void release_graph_stream(Handle& h) {
    if (h.gstream) (void)hipStreamSynchronize(h.gstream);
    for (hipEvent_t& e : h.gev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    if (h.gstream) (void)hipStreamDestroy(h.gstream);
    h.gstream = nullptr;
}
inline void release_streams(Handle& h) {
    if (h.qs.crit) (void)hipStreamSynchronize(h.qs.crit);
    if (h.qs.rest) (void)hipStreamSynchronize(h.qs.rest);
    hipEvent_t ev[4] = {h.qs.evP, h.qs.evR, h.qs.evE, h.qs.evD};
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    if (h.qs.crit) (void)hipStreamDestroy(h.qs.crit);
    if (h.qs.rest) (void)hipStreamDestroy(h.qs.rest);
    h.qs = QrStreams{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
}

inline int ensure_dnorm(Handle& h, size_t elems) {
    if (elems <= h.dnorm_cap) return SDC_OK;
    if (h.no_alloc) return SDC_ERR_NOMEM;
    if (h.dnorm) {
        HIPCHK(hipStreamSynchronize(h.stream));
        HIPCHK(hipFree(h.dnorm));
        h.dnorm = nullptr;
        h.dnorm_cap = 0;
    }
    const size_t cap = elems < 1024 ? 1024 : elems;
    if (hipMalloc(reinterpret_cast<void**>(&h.dnorm), cap * sizeof(double)) != hipSuccess) return SDC_ERR_NOMEM;
    h.dnorm_cap = cap;
    return SDC_OK;
}

// Wait for the handle's stream by polling an event: at the per-iteration
// decision points (convergence norms, ranks, split points) the host must act
// as soon as the data is there, and a blocking synchronization can put the
// thread to sleep for tens of microseconds.
inline int sync_spin(Handle& h) {
    if (!h.ev_sync && h.no_alloc) return SDC_ERR_DEVICE;
    if (!h.ev_sync) HIPCHK(hipEventCreateWithFlags(&h.ev_sync, hipEventDisableTiming));
    HIPCHK(hipEventRecord(h.ev_sync, h.stream));
    hipError_t e;
    while ((e = hipEventQuery(h.ev_sync)) == hipErrorNotReady) {
    }
    HIPCHK(e);
    h.desc_dirty = 0;  // every copy issued so far has run
    return SDC_OK;
}

inline int ensure_dstage(Handle& h, size_t elems) {
    if (elems <= h.dstage_cap) return SDC_OK;
    if (h.no_alloc) return SDC_ERR_NOMEM;
    if (h.dstage) {
        HIPCHK(hipStreamSynchronize(h.stream));
        HIPCHK(hipFree(h.dstage));
        h.dstage = nullptr;
        h.dstage_cap = 0;
    }
    const size_t cap = elems < 4096 ? 4096 : elems;
    if (hipMalloc(reinterpret_cast<void**>(&h.dstage), cap * sizeof(double)) != hipSuccess) return SDC_ERR_NOMEM;
    h.dstage_cap = cap;
    return SDC_OK;
}

inline int ensure_host(Handle& h, size_t bytes) {
    if (bytes <= h.host_size) return SDC_OK;
    if (h.no_alloc) return SDC_ERR_NOMEM;
    if (h.host) {
        HIPCHK(hipStreamSynchronize(h.stream));
        HIPCHK(hipHostFree(h.host));
        h.host = nullptr;
    }
    if (hipHostMalloc(&h.host, bytes, hipHostMallocDefault) != hipSuccess) return SDC_ERR_NOMEM;
    h.host_size = bytes;
    return SDC_OK;
}

// Copy a host array of descriptors to the device arena through its pinned
// mirror.  The copy is asynchronous and reads the mirror when it runs, so the
// arena may be rewound (desc_off lowered) at any time, but a mirror byte that
// an earlier copy still has to read is not overwritten: writing below
// desc_dirty first waits for the most recent copy (copies on the stream
// complete in order, so every earlier one has then read its bytes).
template <class T> inline const T* upload(Handle& h, const std::vector<T>& v) {
    const size_t bytes = v.size() * sizeof(T);
    size_t off = (h.desc_off + 255) & ~size_t(255);
    if (off + bytes > h.desc_size) return nullptr;
    if (!h.ev_desc && (h.no_alloc || hipEventCreateWithFlags(&h.ev_desc, hipEventDisableTiming) != hipSuccess)) {
        h.ev_desc = nullptr;
        return nullptr;
    }
    if (off < h.desc_dirty) {
        if (hipEventSynchronize(h.ev_desc) != hipSuccess) return nullptr;
        h.desc_dirty = 0;
    }
    std::memcpy(h.desc_h + off, v.data(), bytes);
    if (hipMemcpyAsync(h.desc_d + off, h.desc_h + off, bytes, hipMemcpyHostToDevice, h.stream) != hipSuccess)
        return nullptr;
    if (hipEventRecord(h.ev_desc, h.stream) != hipSuccess) return nullptr;
    h.desc_dirty = std::max(h.desc_dirty, off + bytes);
    h.desc_off = off + bytes;
    return reinterpret_cast<const T*>(h.desc_d + off);
}
#define UPLOAD(ptr, vec)                                   \
    auto ptr = upload(h, vec);                             \
    if (!ptr) return SDC_ERR_DEVICE;

// Small device results of several problems to the host with one copy:
// gathered on the device into h.dstage, copied to h.host, synchronized.
// `out` points at the segments, back to back in the order given.
inline int read_back(Handle& h, const std::vector<GatherDesc>& g, double*& out) {
    size_t total = 0;
    for (const GatherDesc& d : g) total = std::max(total, (size_t)d.off + (size_t)d.n);
    if (int st = ensure_dstage(h, total + 1)) return st;
    if (int st = ensure_host(h, (total + 1) * sizeof(double) + 64)) return st;
    const size_t mark = h.desc_off;
    UPLOAD(dg, g);
    gather_batch(dg, (int)g.size(), h.dstage, h.stream);
    HIPCHK(hipMemcpyAsync(h.host, h.dstage, total * sizeof(double), hipMemcpyDeviceToHost, h.stream));
    if (int st = sync_spin(h)) return st;
    h.desc_off = mark;
    out = reinterpret_cast<double*>(h.host);
    return SDC_OK;
}


}  // namespace sdc
