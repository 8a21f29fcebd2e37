// Host-side helpers of libba: error text, status plumbing, device arenas.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "ba.h"

namespace ba {

void set_error(const char *fmt, ...);

#define BA_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t _e = (call);                                                                        \
        if (_e != hipSuccess) {                                                                        \
            ::ba::set_error("%s: %s (%s:%d)", #call, hipGetErrorString(_e), __FILE__, __LINE__);       \
            return BA_E_HIP;                                                                           \
        }                                                                                              \
    } while (0)

#define BA_TRY(expr)                                                                                   \
    do {                                                                                               \
        ba_status _s = (expr);                                                                         \
        if (_s != BA_OK) return _s;                                                                    \
    } while (0)

// Optional per-kernel timing with HIP events (ba_profile_enable).
void prof_begin(const char *name, hipStream_t s);
void prof_end(hipStream_t s);
struct ProfScope {
    hipStream_t s;
    ProfScope(const char *name, hipStream_t st) : s(st) { prof_begin(name, st); }
    ~ProfScope() { prof_end(s); }
};

// A slot-owned block of device memory that allocations of the calling thread
// are carved from (bump allocation, 256-byte aligned) while it is installed in
// tl_slot_arena; the owner resets `off` when the work that used it is done.
// Allocations that do not fit fall through to hipMalloc.
struct SlotArena {
    char *base = nullptr;
    size_t cap = 0;
    size_t off = 0;
};
extern thread_local SlotArena *tl_slot_arena;

// A set of device allocations released together (memory carved from an
// installed slot arena is returned by the arena's owner, not here).
struct DevArena {
    std::vector<void *> ptrs;
    size_t bytes = 0;
    DevArena() = default;
    DevArena(const DevArena &) = delete;
    DevArena &operator=(const DevArena &) = delete;
    ~DevArena() { release(); }
    void release() {
        for (void *p : ptrs) (void)hipFree(p);
        ptrs.clear();
        bytes = 0;
    }
    template <class T>
    ba_status alloc(T **p, int64_t count) {
        size_t nb = sizeof(T) * (size_t)(count > 0 ? count : 1);
        if (SlotArena *a = tl_slot_arena) {
            const size_t nba = (nb + 255) / 256 * 256;
            if (a->off + nba <= a->cap) {
                *p = (T *)(a->base + a->off);
                a->off += nba;
                bytes += nb;
                return BA_OK;
            }
        }
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, nb);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("device allocation of %zu bytes failed: %s", nb, hipGetErrorString(e));
            return BA_E_NOMEM;
        }
        ptrs.push_back(q);
        bytes += nb;
        *p = (T *)q;
        return BA_OK;
    }
};

}  // namespace ba
