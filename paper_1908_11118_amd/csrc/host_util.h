// host_util.h -- error reporting and small helpers for the host side of libregc_hip.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>

#include "../../include/regc.h"

namespace regc {

// thread-local message of the last failure (regc_last_error)
void set_error(const char *fmt, ...);

#define REGC_HIP(call)                                                                     \
    do {                                                                                   \
        hipError_t _e = (call);                                                            \
        if (_e != hipSuccess) {                                                            \
            ::regc::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(_e), __FILE__, \
                              __LINE__);                                                   \
            return REGC_EHIP;                                                              \
        }                                                                                  \
    } while (0)

#define REGC_CHECK(cond, code, ...)          \
    do {                                     \
        if (!(cond)) {                       \
            ::regc::set_error(__VA_ARGS__);  \
            return (code);                   \
        }                                    \
    } while (0)

// device buffer owned by a context
template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    int alloc(size_t count)
    {
        release();
        if (count == 0) count = 1;
        hipError_t e = hipMalloc((void **)&p, count * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            set_error("hipMalloc(%zu bytes) failed: %s", count * sizeof(T), hipGetErrorString(e));
            return REGC_ENOMEM;
        }
        n = count;
        return REGC_OK;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    ~DevBuf() { release(); }
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

// A HIP event destroyed with its scope (also on early error returns).
struct ScopedEvent {
    hipEvent_t e = nullptr;
    hipError_t create() { return hipEventCreate(&e); }
    ~ScopedEvent()
    {
        if (e) (void)hipEventDestroy(e);
    }
    ScopedEvent() = default;
    ScopedEvent(const ScopedEvent &) = delete;
    ScopedEvent &operator=(const ScopedEvent &) = delete;
};

}  // namespace regc
