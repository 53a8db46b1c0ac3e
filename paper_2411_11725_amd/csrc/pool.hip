// Device memory for meshes: plain hipMalloc / hipFree, or a pool.
//
// hipFree waits for the whole device, so a process that creates and destroys
// meshes while other meshes are stepping (the solve server) would stall every
// stream at each retirement.  A pool takes device memory in large chunks once
// and hands out and takes back sub-ranges (first fit, neighbours coalesced on
// release) without calling the runtime; chunks go back to the runtime only
// when the pool is destroyed.  A thread installs a pool with
// set_thread_pool(); allocations made by that thread (mesh buffers, demag
// tensor set-up temporaries) then come from it, and a mesh remembers the pool
// its buffers came from.  Pinned host blocks for the step-controller mirror
// are recycled the same way.
#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "nm_internal.h"

namespace nm {

struct DevPool {
    struct Chunk {
        char *base = nullptr;
        size_t size = 0;
        std::map<size_t, size_t> free;   // offset -> length
    };
    std::mutex mu;
    std::vector<Chunk> chunks;
    std::map<char *, std::pair<size_t, size_t>> live;   // pointer -> (chunk, length)
    std::vector<void *> host_free;                      // recycled pinned blocks
    std::vector<void *> host_all;
    size_t chunk_bytes = size_t(512) << 20;
    nm_allocator user{};   // caller's hooks: every block comes from user.alloc
};

static thread_local DevPool *t_pool = nullptr;

DevPool *pool_create() { return new DevPool(); }

DevPool *pool_create_user(const nm_allocator &a) {
    DevPool *P = new DevPool();
    P->user = a;
    return P;
}

void pool_destroy(DevPool *P) {
    if (!P) return;
    for (auto &c : P->chunks) (void)hipFree(c.base);
    for (void *h : P->host_all) (void)hipHostFree(h);
    delete P;
}

void set_thread_pool(DevPool *P) { t_pool = P; }
DevPool *thread_pool() { return t_pool; }

static constexpr size_t kAlign = 256;

hipError_t dev_alloc(void **p, size_t bytes, DevPool *P) {
    bytes = (bytes + kAlign - 1) / kAlign * kAlign;
    if (bytes == 0) bytes = kAlign;
    if (!P) return hipMalloc(p, bytes);
    if (P->user.alloc) {   // the caller's allocator, block by block
        void *q = P->user.alloc(bytes, P->user.ctx);
        if (!q || (reinterpret_cast<uintptr_t>(q) % kAlign) != 0) {
            if (q) P->user.free(q, P->user.ctx);
            return hipErrorOutOfMemory;
        }
        *p = q;
        return hipSuccess;
    }
    std::lock_guard<std::mutex> lk(P->mu);
    for (size_t ci = 0; ci < P->chunks.size(); ++ci) {
        auto &fr = P->chunks[ci].free;
        for (auto it = fr.begin(); it != fr.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            fr.erase(it);
            if (len > bytes) fr[off + bytes] = len - bytes;
            char *q = P->chunks[ci].base + off;
            P->live[q] = {ci, bytes};
            *p = q;
            return hipSuccess;
        }
    }
    DevPool::Chunk c;
    c.size = bytes > P->chunk_bytes ? bytes : P->chunk_bytes;
    hipError_t e = hipMalloc((void **)&c.base, c.size);
    if (e != hipSuccess) return e;
    if (c.size > bytes) c.free[bytes] = c.size - bytes;
    P->chunks.push_back(c);
    P->live[c.base] = {P->chunks.size() - 1, bytes};
    *p = c.base;
    return hipSuccess;
}

void dev_free(void *p, DevPool *P) {
    if (!p) return;
    if (!P) {
        (void)hipFree(p);
        return;
    }
    if (P->user.alloc) {
        P->user.free(p, P->user.ctx);
        return;
    }
    std::lock_guard<std::mutex> lk(P->mu);
    auto it = P->live.find((char *)p);
    if (it == P->live.end()) return;
    const size_t ci = it->second.first;
    size_t off = (size_t)((char *)p - P->chunks[ci].base), len = it->second.second;
    P->live.erase(it);
    auto &fr = P->chunks[ci].free;
    auto nx = fr.lower_bound(off);
    if (nx != fr.end() && nx->first == off + len) {   // merge with the following range
        len += nx->second;
        nx = fr.erase(nx);
    }
    if (nx != fr.begin()) {                             // and with the preceding one
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
            pv->second += len;
            return;
        }
    }
    fr[off] = len;
}

hipError_t host_alloc(void **p, size_t bytes, DevPool *P) {
    if (!P || P->user.alloc) return hipHostMalloc(p, bytes, hipHostMallocDefault);
    if (bytes > kPoolHostBlock) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lk(P->mu);
    if (!P->host_free.empty()) {
        *p = P->host_free.back();
        P->host_free.pop_back();
        return hipSuccess;
    }
    hipError_t e = hipHostMalloc(p, kPoolHostBlock, hipHostMallocDefault);
    if (e == hipSuccess) P->host_all.push_back(*p);
    return e;
}

void host_free(void *p, DevPool *P) {
    if (!p) return;
    if (!P || P->user.alloc) {
        (void)hipHostFree(p);
        return;
    }
    std::lock_guard<std::mutex> lk(P->mu);
    P->host_free.push_back(p);
}

}  // namespace nm
