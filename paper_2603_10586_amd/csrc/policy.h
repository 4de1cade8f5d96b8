// Admission policy of the solve server (host only, no device calls, so it is testable on
// its own).  Requests carry a device footprint (operator + solver workspaces, estimated
// before anything is allocated) and the key of their geometry.  A request is admitted
// when a slot is free and its footprint fits the HBM budget next to the admitted requests
// and the cached operators; requests are considered in arrival order, but one that does not
// fit yet does not hold back later ones that do (no head-of-line blocking), until it has
// been overtaken by `max_bypass` later admissions (0: no limit): from then on nothing
// behind it is admitted before it, so a large request cannot starve.  Cached
// operators that no admitted request uses are evicted least recently used when a request
// needs their bytes.  A request whose operator is cached needs only its solver bytes and
// pins the cache entry until it finishes.  A request that cannot fit even in an empty
// device is refused at submission.
#pragma once

#include <cstddef>
#include <cstdint>
#include <list>
#include <string>
#include <unordered_map>
#include <vector>

namespace qrvie {
namespace sched {

class Policy {
public:
    Policy(int slots, size_t budget, int op_cache, int max_bypass = 0)
        : slots_(slots), budget_(budget), op_cache_(op_cache), max_bypass_(max_bypass) {}

    // Queue a request; false (refused) when it cannot fit an otherwise empty budget (its
    // operator may be evicted before it starts, so the whole footprint must fit).  The
    // footprint of a request that builds its operator includes op_bytes (what a cached
    // operator keeps) and build_bytes (the build's transient buffers); a cache hit needs
    // neither.
    bool enqueue(uint64_t ticket, const std::string& key, size_t footprint, size_t op_bytes, size_t build_bytes = 0) {
        if (footprint > budget_ || op_bytes + build_bytes > footprint) return false;
        jobs_[ticket] = Job{key, footprint, op_bytes, build_bytes, 0, false, 0};
        queue_.push_back(ticket);
        return true;
    }

    // Admit every queued request that fits now, in arrival order; evicted cache keys are
    // appended to `evicted` (their operators are to be destroyed by the caller).
    void admit(std::vector<uint64_t>* admitted, std::vector<std::string>* evicted) {
        std::vector<Job*> waiting;          // passed over in this admission pass, still queued
        for (auto it = queue_.begin(); it != queue_.end() && running_ < slots_;) {
            Job& j = jobs_.at(*it);
            const bool hit = cached(j.key);
            const std::string* keep = hit ? &j.key : nullptr;   // a hit never evicts its own operator
            const size_t need = hit ? j.footprint - j.op_bytes - j.build_bytes : j.footprint;
            if (in_use_ + need > budget_ + evictable(keep)) {
                waiting.push_back(&j);      // does not fit even after evictions: evict nothing
                ++it;
                continue;
            }
            bool starved = false;           // an earlier request may not be overtaken again
            for (Job* w : waiting) starved = starved || (max_bypass_ > 0 && w->bypassed >= max_bypass_);
            if (starved) break;
            for (Job* w : waiting) ++w->bypassed;
            while (in_use_ + need > budget_ && evict_one(evicted, keep)) {
            }
            in_use_ += need;
            peak_ = in_use_ > peak_ ? in_use_ : peak_;
            j.need = need;
            j.pinned = hit;
            if (hit) {
                Entry& e = cache_.at(j.key);
                ++e.pins;
                lru_.splice(lru_.end(), lru_, e.pos);   // most recently used
                ++hits_;
            }
            ++running_;
            admitted->push_back(*it);
            it = queue_.erase(it);
        }
    }

    // A running request finished.  `built` is true when it built a new operator (not a
    // cache hit); the return value says whether that operator is kept in the cache (else
    // the caller destroys it).  Cache overflow evictions are appended to `evicted`.
    bool finish(uint64_t ticket, bool built, std::vector<std::string>* evicted) {
        Job j = jobs_.at(ticket);
        jobs_.erase(ticket);
        in_use_ -= j.need;
        --running_;
        if (j.pinned) {
            --cache_.at(j.key).pins;
            return false;
        }
        if (!built || op_cache_ <= 0 || cached(j.key)) return false;
        lru_.push_back(j.key);
        cache_[j.key] = Entry{j.op_bytes, 0, std::prev(lru_.end())};
        in_use_ += j.op_bytes;
        peak_ = in_use_ > peak_ ? in_use_ : peak_;
        while ((int)cache_.size() > op_cache_ && evict_one(evicted)) {
        }
        return cached(j.key);
    }

    // Drop every cached operator (server shutdown); keys are appended to `evicted`.
    void clear(std::vector<std::string>* evicted) {
        while (evict_one(evicted)) {
        }
    }

    bool cached(const std::string& key) const { return cache_.count(key) != 0; }
    // Whether an admitted (not yet finished) request holds a pin on its cached operator.
    bool pinned(uint64_t ticket) const {
        auto it = jobs_.find(ticket);
        return it != jobs_.end() && it->second.pinned;
    }
    size_t in_use() const { return in_use_; }
    size_t peak() const { return peak_; }
    int running() const { return running_; }
    size_t queued() const { return queue_.size(); }
    size_t cache_size() const { return cache_.size(); }
    int64_t hits() const { return hits_; }
    int64_t evictions() const { return evictions_; }

private:
    struct Job {
        std::string key;
        size_t footprint, op_bytes, build_bytes, need;
        bool pinned;
        int bypassed;                       // later requests admitted while this one waited
    };
    struct Entry {
        size_t bytes;
        int pins;
        std::list<std::string>::iterator pos;
    };

    // Bytes held by cached operators that no admitted request pins, other than `keep`.
    size_t evictable(const std::string* keep) const {
        size_t b = 0;
        for (const auto& kv : cache_)
            if (kv.second.pins == 0 && !(keep && kv.first == *keep)) b += kv.second.bytes;
        return b;
    }

    // Evict the least recently used unpinned operator other than `keep`; false if none.
    bool evict_one(std::vector<std::string>* evicted, const std::string* keep = nullptr) {
        for (auto it = lru_.begin(); it != lru_.end(); ++it) {
            Entry& e = cache_.at(*it);
            if (e.pins > 0 || (keep && *it == *keep)) continue;
            in_use_ -= e.bytes;
            evicted->push_back(*it);
            cache_.erase(*it);
            lru_.erase(it);
            ++evictions_;
            return true;
        }
        return false;
    }

    int slots_;
    size_t budget_;
    int op_cache_;
    int max_bypass_;
    int running_ = 0;
    size_t in_use_ = 0, peak_ = 0;
    int64_t hits_ = 0, evictions_ = 0;
    std::list<uint64_t> queue_;
    std::unordered_map<uint64_t, Job> jobs_;
    std::list<std::string> lru_;
    std::unordered_map<std::string, Entry> cache_;
};

}  // namespace sched
}  // namespace qrvie
