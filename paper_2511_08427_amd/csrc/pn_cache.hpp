// Bookkeeping of the library's cached device memory -- plans and their work
// buffers -- independent of the device API: the memory policy `Mem` is a
// template parameter (hipMalloc/hipFree in the library, a counting fake in
// the CPU test of these rules).  Not part of the public ABI.
//
// Graph capture.  Kernels captured into a HIP graph keep the device
// addresses they were captured with, so memory a captured call uses must
// outlive the graph:
//   * a plan used by a call under stream capture is pinned: the LRU never
//     evicts it (the cache grows past its limit instead);
//   * a buffer of a pinned plan is never freed or re-purposed: a later call
//     that needs it larger, or laid out for another storage type, retires
//     it (it stays allocated until release) and gets a new one;
//   * under capture nothing is allocated or re-purposed: a captured call
//     must find its plan and buffers ready, i.e. follow an eager call with
//     the same geometry, batch and types.
// Everything is freed by the library's release of its caches, which
// therefore invalidates every graph that captured one of its calls.
#pragma once

#include <cstddef>
#include <cstdint>
#include <list>
#include <memory>
#include <vector>

namespace pn {

// One cached device buffer.
struct DevBuf {
    void *ptr = nullptr;
    size_t cap = 0;    // bytes
    int32_t tag = -1;  // the layout its contents were made for (-1: none yet)
};

enum class Ensure {
    kReady,      // the buffer already fits and holds this layout
    kFresh,      // new memory, or re-purposed for this layout: (re)initialise it
    kNoMem,      // the allocation failed (the buffer is unchanged)
    kCapturing,  // a change is needed but the caller's stream is capturing (nothing done)
};

template <class Mem>
class BufferKeeper {
public:
    BufferKeeper() = default;
    BufferKeeper(const BufferKeeper &) = delete;
    BufferKeeper &operator=(const BufferKeeper &) = delete;
    ~BufferKeeper() { release_retired(); }

    // Makes `b` hold at least `need` bytes laid out for `tag`.  `pinned`:
    // b belongs to a plan a captured graph may use; `capturing`: the
    // calling stream is capturing.
    Ensure ensure(DevBuf &b, size_t need, int32_t tag, bool pinned, bool capturing)
    {
        if (b.ptr && b.cap >= need && b.tag == tag) return Ensure::kReady;
        if (capturing) return Ensure::kCapturing;
        if (b.ptr && b.cap >= need && !pinned) {
            b.tag = tag;
            return Ensure::kFresh;
        }
        void *np = nullptr;
        if (!Mem::alloc(&np, need == 0 ? 1 : need)) return Ensure::kNoMem;
        if (b.ptr) {
            if (pinned) retired_.push_back(b.ptr);
            else Mem::release(b.ptr);
        }
        b.ptr = np;
        b.cap = need;
        b.tag = tag;
        return Ensure::kFresh;
    }

    // Frees a buffer of a plan that is being destroyed.
    void free(DevBuf &b)
    {
        if (b.ptr) Mem::release(b.ptr);
        b = DevBuf{};
    }

    void release_retired()
    {
        for (void *p : retired_) Mem::release(p);
        retired_.clear();
    }

    size_t retired() const { return retired_.size(); }

private:
    std::vector<void *> retired_;
};

// Least-recently-used list of plans.  P needs `bool held() const`: a held
// plan (used under capture, or by a live batch plan) is never evicted.
template <class P>
class PlanLru {
public:
    // The first plan (most recently used first) for which pred holds, moved
    // to the front; nullptr if none.
    template <class Pred>
    P *find(Pred pred)
    {
        for (auto it = plans_.begin(); it != plans_.end(); ++it) {
            if (pred(**it)) {
                if (it != plans_.begin()) plans_.splice(plans_.begin(), plans_, it);
                return plans_.front().get();
            }
        }
        return nullptr;
    }

    // Inserts a plan as the most recently used one, then evicts the least
    // recently used plans that are not held while more than `limit` are
    // kept; the new plan itself is never evicted (when every other plan is
    // held the list grows past the limit).
    P *insert(std::unique_ptr<P> p, size_t limit)
    {
        plans_.push_front(std::move(p));
        P *front = plans_.front().get();
        trim(limit, 1);
        return front;
    }

    // Evicts the least recently used plans that are not held, sparing the
    // `spare` most recently used ones, while more than `limit` are kept.
    void trim(size_t limit, size_t spare = 0)
    {
        auto it = plans_.end();
        size_t left = plans_.size();  // plans at or before `it`
        while (plans_.size() > limit && left > spare) {
            --it;
            --left;
            if ((*it)->held()) continue;
            it = plans_.erase(it);
        }
    }

    void clear() { plans_.clear(); }

    // Destroys every plan for which keep() is false.
    template <class Keep>
    void remove_unless(Keep keep)
    {
        for (auto it = plans_.begin(); it != plans_.end();) {
            if (keep(**it)) ++it;
            else it = plans_.erase(it);
        }
    }
    size_t size() const { return plans_.size(); }

private:
    std::list<std::unique_ptr<P>> plans_;  // most recently used first
};

}  // namespace pn
