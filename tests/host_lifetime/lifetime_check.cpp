// Host-only check of the context lifetime and block cache (lifetime.h), built
// with g++ and the address and undefined-behaviour sanitizers. The library's own
// header is included unchanged; device memory is replaced by malloc through a
// stub device that counts every block, so a block freed twice, used after being
// freed, or never freed makes this program fail.
//
//   lifetime_check            every destroy order, cache reuse, the cap, running
//                             out of memory, repeated releases, random orders
//   lifetime_check early-free the context is freed when the caller releases it
//                             although a problem still holds it, as a context
//                             without the holder count would be: the problem's
//                             destroy then writes into the freed context
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "../../paper_2409_08808_amd/csrc/lifetime.h"

static long g_blocks = 0;      // blocks the stub device has handed out and not freed
static long g_contexts = 0;    // contexts not yet freed
static long g_fail = 0;

#define CHECK(cond)                                                          \
    do {                                                                     \
        if (!(cond)) {                                                       \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++g_fail;                                                        \
        }                                                                    \
    } while (0)

struct StubDev {
    size_t capacity = (size_t)1 << 40;
    size_t used = 0;
    int drains = 0;
    std::map<void*, size_t> live;
    bool alloc(void** p, size_t bytes) {
        if (used + bytes > capacity) return false;
        *p = std::malloc(bytes);
        if (!*p) return false;
        std::memset(*p, 0xA5, std::min<size_t>(bytes, 4096));
        live[*p] = bytes;
        used += bytes;
        ++g_blocks;
        return true;
    }
    void release(void* p) {
        auto it = live.find(p);
        CHECK(it != live.end());
        if (it == live.end()) return;
        used -= it->second;
        live.erase(it);
        --g_blocks;
        std::free(p);
    }
    void drain() { ++drains; }
};

struct Ctx {
    StubDev dev;
    goac::BlockCache<StubDev> pool;
    goac::Holders holders;
    explicit Ctx(size_t cap) : pool(cap) { ++g_contexts; }
};

// a problem or chain set: one arena from the context's cache
struct Obj {
    Ctx* ctx;
    void* arena = nullptr;
    size_t bytes = 0;
};

static void free_ctx(Ctx* c) {
    c->dev.drain();
    c->pool.clear(c->dev);
    CHECK(c->dev.live.empty());  // every block came back before the context went
    --g_contexts;
    delete c;
}

static void free_blocks(Obj* o) {
    o->ctx->pool.put(o->ctx->dev, o->arena, o->bytes);
    o->arena = nullptr;
}

static Obj* make(Ctx* c, size_t bytes) {
    Obj* o = new Obj{c};
    size_t b = bytes;
    if (!c->pool.get(c->dev, &b, &o->arena)) {
        delete o;
        return nullptr;
    }
    CHECK(b >= bytes && b % goac::BlockCache<StubDev>::kGranule == 0);
    std::memset(o->arena, 0x5A, std::min<size_t>(b, 4096));  // the arena is used
    o->bytes = b;
    c->holders.attach();
    return o;
}

static void destroy(Obj* o) { goac::destroy_dependent(o->ctx, o, free_blocks, free_ctx); }
static void release(Ctx* c) { goac::release_context(c, free_ctx); }

// every order of releasing a context and destroying a problem and a chain set
static void all_orders() {
    int order[3] = {0, 1, 2};
    int n = 0;
    do {
        Ctx* c = new Ctx((size_t)8 << 30);
        Obj* pb = make(c, 3 << 20);
        Obj* ch = make(c, 5 << 20);
        for (int k : order) {
            if (k == 0) release(c);
            if (k == 1) destroy(pb);
            if (k == 2) destroy(ch);
        }
        CHECK(g_contexts == 0 && g_blocks == 0);
        ++n;
    } while (std::next_permutation(order, order + 3));
    CHECK(n == 6);
}

// released blocks are reused for requests up to twice smaller, not for larger ones
static void reuse() {
    Ctx* c = new Ctx((size_t)8 << 30);
    Obj* a = make(c, 4 << 20);
    void* pa = a->arena;
    destroy(a);
    CHECK(c->pool.blocks.size() == 1);
    Obj* b = make(c, 3 << 20);  // 4 MiB <= 2 x 3 MiB: the cached block
    CHECK(b->arena == pa && b->bytes == (4u << 20));
    destroy(b);
    Obj* d = make(c, 1 << 20);  // 4 MiB > 2 x 1 MiB: a new block
    CHECK(d->arena != pa && c->pool.blocks.size() == 1);
    Obj* e = make(c, 5 << 20);  // larger: a new block
    CHECK(e->arena != pa);
    destroy(d);
    destroy(e);
    release(c);
    CHECK(g_contexts == 0 && g_blocks == 0);
}

// beyond the cap a released block is freed at once, after draining the stream
static void cap() {
    Ctx* c = new Ctx((size_t)6 << 20);
    Obj* a = make(c, 4 << 20);
    Obj* b = make(c, 4 << 20);
    destroy(a);
    const int d0 = c->dev.drains;
    destroy(b);  // 8 MiB would exceed the 6 MiB cap
    CHECK(c->dev.drains == d0 + 1 && c->pool.bytes == (4u << 20) && c->dev.live.size() == 1);
    release(c);
    CHECK(g_contexts == 0 && g_blocks == 0);
}

// a full device: the cache is dropped and the allocation tried once more
static void out_of_memory() {
    Ctx* c = new Ctx((size_t)8 << 30);
    c->dev.capacity = 8 << 20;
    Obj* a = make(c, 3 << 20);
    Obj* b = make(c, 3 << 20);
    destroy(a);                 // 3 MiB cached, 3 MiB in use
    Obj* d = make(c, 5 << 20);  // needs the cached block's room
    CHECK(d != nullptr && c->pool.blocks.empty());
    Obj* e = make(c, 1 << 20);  // 8 MiB in use: no room at all
    CHECK(e == nullptr);
    destroy(b);
    destroy(d);
    release(c);
    CHECK(g_contexts == 0 && g_blocks == 0);
}

// the caller's second release of a context that is still held changes nothing
static void repeated_release() {
    Ctx* c = new Ctx((size_t)8 << 30);
    Obj* a = make(c, 1 << 20);
    release(c);
    release(c);
    CHECK(g_contexts == 1);
    destroy(a);
    CHECK(g_contexts == 0 && g_blocks == 0);
}

// many problems and chain sets made and destroyed in random orders
static void random_orders() {
    uint64_t s = 12345;
    auto next = [&s]() {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return (uint32_t)(s >> 33);
    };
    for (int round = 0; round < 300; ++round) {
        Ctx* c = new Ctx((size_t)(next() % 64 + 1) << 20);
        std::vector<Obj*> objs;
        const int n = 1 + next() % 12;
        bool released = false;
        for (int k = 0; k < 3 * n; ++k) {
            const uint32_t r = next() % 4;
            if (r < 2 && (int)objs.size() < n) {
                objs.push_back(make(c, (size_t)(next() % (8 << 20)) + 1));
            } else if (r == 2 && !objs.empty()) {
                const size_t i = next() % objs.size();
                Obj* o = objs[i];
                objs.erase(objs.begin() + (long)i);
                if (released && objs.empty()) {
                    destroy(o);  // the last holder: frees the context
                    c = nullptr;
                    break;
                }
                destroy(o);
            } else if (r == 3 && !released && !objs.empty()) {
                release(c);
                released = true;
            }
        }
        if (c) {
            if (!released) release(c);
            while (!objs.empty()) {
                Obj* o = objs.back();
                objs.pop_back();
                destroy(o);
            }
        }
        CHECK(g_contexts == 0 && g_blocks == 0);
    }
}

// A context freed while a problem still holds it: the problem's destroy returns
// its arena to the freed context's cache.
static void early_free() {
    Ctx* c = new Ctx((size_t)8 << 30);
    Obj* pb = make(c, 1 << 20);
    free_ctx(c);  // no holder count: freed at the caller's release
    destroy(pb);
}

int main(int argc, char** argv) {
    if (argc > 1 && std::strcmp(argv[1], "early-free") == 0) {
        early_free();
        std::printf("early-free: not detected\n");
        return 0;
    }
    all_orders();
    reuse();
    cap();
    out_of_memory();
    repeated_release();
    random_orders();
    if (g_fail) {
        std::printf("lifetime: %ld checks failed\n", g_fail);
        return 1;
    }
    std::printf("lifetime: ok\n");
    return 0;
}
