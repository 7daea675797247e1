// lbvp_graph.h -- host side of LBVP_GRAPH, shared by the D2Q9 and D3Q19 step
// calls: the key of a captured chunk of steps and a small cache of the
// instantiated graphs kept per context or batch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>
#include <vector>

namespace lbvp_host {

// The launches of one chunk of steps, identified by everything that is baked
// into them: chunk length, whether the last step keeps the fields, the lattice
// parity, the AA step parity, the record phase and buffer, and the argument
// generation (bumped whenever kernel arguments or tables change).
struct GraphKey {
    int64_t n = 0, phase = 0;
    int32_t keep = 0, cur = 0, par = 0, rec = 0;
    uint64_t gen = 0;
    bool same(const GraphKey& o) const
    {
        return n == o.n && phase == o.phase && keep == o.keep && cur == o.cur && par == o.par && rec == o.rec &&
               gen == o.gen;
    }
};

// A few instantiated graphs, most recently used last.
class GraphCache {
  public:
    GraphCache() = default;
    GraphCache(const GraphCache&) = delete;
    GraphCache& operator=(const GraphCache&) = delete;
    ~GraphCache() { drop(); }
    hipGraphExec_t find(const GraphKey& k)
    {
        for (size_t i = 0; i < e_.size(); ++i)
            if (e_[i].first.same(k)) {
                auto hit = e_[i];
                e_.erase(e_.begin() + (long)i);
                e_.push_back(hit);
                return hit.second;
            }
        return nullptr;
    }
    // An evicted graph may still run: the stream is drained before it is freed.
    void put(const GraphKey& k, hipGraphExec_t x, hipStream_t s)
    {
        if (e_.size() == CAP) {
            (void)hipStreamSynchronize(s);
            (void)hipGraphExecDestroy(e_.front().second);
            e_.erase(e_.begin());
        }
        e_.emplace_back(k, x);
    }
    void clear(hipStream_t s)
    {
        if (e_.empty()) return;
        (void)hipStreamSynchronize(s);
        drop();
    }
    bool empty() const { return e_.empty(); }

  private:
    void drop()
    {
        for (auto& x : e_) (void)hipGraphExecDestroy(x.second);
        e_.clear();
    }
    static constexpr size_t CAP = 8;
    std::vector<std::pair<GraphKey, hipGraphExec_t>> e_;
};

}  // namespace lbvp_host
