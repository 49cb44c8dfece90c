// Host-side lifetime of a context and of the device blocks it lends to the
// problems and chain sets made on it. The code is written against a small device
// interface, so the library (HIP memory, ordered by the context's stream) and a
// host-only check program (malloc, built with the address and undefined-behaviour
// sanitizers) run the same logic. This header includes no HIP header.
//
// The device interface `Dev` provides
//   bool alloc(void** p, size_t bytes)  a new block, false when the device is full
//   void release(void* p)               free a block no queued work uses any more
//   void drain()                        wait until no queued work uses any block
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>

namespace goac {

// Released blocks of one context, by size. All work of a context runs on its one
// stream, so a block handed back here is reused only by work queued after
// everything that used it; no wait is needed on either side. At most max_bytes
// are kept; a block beyond that is freed once the stream has passed its users.
template <class Dev>
struct BlockCache {
    static constexpr size_t kGranule = (size_t)1 << 16;
    size_t max_bytes;
    std::multimap<size_t, void*> blocks;
    size_t bytes = 0;

    explicit BlockCache(size_t max) : max_bytes(max) {}

    // A block of at least *want bytes: the smallest cached block no larger than
    // twice the request rounded up to kGranule, else a new one (dropping the cache
    // and trying once more when the device is full). *want becomes the block's
    // size. Returns false when no block can be had.
    bool get(Dev& dev, size_t* want, void** out) {
        const size_t w = (*want + kGranule - 1) / kGranule * kGranule;
        auto it = blocks.lower_bound(w);
        if (it != blocks.end() && it->first <= 2 * w) {
            *out = it->second;
            *want = it->first;
            bytes -= it->first;
            blocks.erase(it);
            return true;
        }
        if (!dev.alloc(out, w)) {
            dev.drain();
            clear(dev);
            if (!dev.alloc(out, w)) {
                *out = nullptr;
                return false;
            }
        }
        *want = w;
        return true;
    }

    // Hand a block back (p may be null). Past the cap the stream is drained first,
    // since work queued earlier may still use the block.
    void put(Dev& dev, void* p, size_t size) {
        if (!p) return;
        if (bytes + size > max_bytes) {
            dev.drain();
            dev.release(p);
            return;
        }
        blocks.emplace(size, p);
        bytes += size;
    }

    // Free every cached block (the caller has drained the stream).
    void clear(Dev& dev) {
        for (auto& b : blocks) dev.release(b.second);
        blocks.clear();
        bytes = 0;
    }
};

// What keeps a context alive: the caller's handle until goac_ctx_destroy, and
// every problem or chain set made on it until that one is destroyed (each returns
// its blocks to the context's cache as it goes). The context is freed when the
// last of them lets go, in whichever order that happens.
struct Holders {
    int64_t live = 0;       // problems and chain sets not yet destroyed
    bool released = false;  // the caller has released its handle

    void attach() { ++live; }
    // A dependent is gone; true when the context must be freed now.
    bool detach() { return --live == 0 && released; }
    // The caller lets go; true when the context must be freed now. A second
    // release of a context that is still held changes nothing.
    bool release() {
        if (released) return false;
        released = true;
        return live == 0;
    }
};

// End of a problem or chain set: its blocks return to the context's cache while
// the context is certainly alive, the object is deleted, and only then may the
// context go.
template <class Ctx, class Obj, class FreeBlocks, class FreeCtx>
void destroy_dependent(Ctx* ctx, Obj* obj, FreeBlocks free_blocks, FreeCtx free_ctx) {
    free_blocks(obj);
    delete obj;
    if (ctx->holders.detach()) free_ctx(ctx);
}

// The caller's release of a context.
template <class Ctx, class FreeCtx>
void release_context(Ctx* ctx, FreeCtx free_ctx) {
    if (ctx && ctx->holders.release()) free_ctx(ctx);
}

}  // namespace goac
