// registry.hpp -- the systems that the slots of a batch refer to.
//
// A batch keeps one device view per distinct system its slots use, indexed
// by a small integer that the kernels read from the slot table.  The
// registry holds a reference on every system it lists (the caller passes
// retain / release), so a system cannot be freed, and its address cannot be
// reused by another system, while an entry names it.  An entry stays listed
// while slots use it; once none does it becomes collectable, and
// collect() -- to be called only when no queued device work can still read
// the entry -- drops it and hands back the references to release.  Plain
// host code (no HIP), so that its logic is checked on the CPU.
#pragma once

#include <vector>

namespace hcn {

template <class Handle>
class SysRegistry {
public:
    explicit SysRegistry(int capacity) : cap_(capacity) {}

    int capacity() const { return cap_; }
    int size() const { return (int)sys_.size(); }
    Handle at(int idx) const { return sys_[idx]; }
    bool live(int idx) const { return sys_[idx] != Handle(); }
    int users(int idx) const { return users_[idx]; }

    // entry of h, or -1
    int find(Handle h) const {
        for (int q = 0; q < (int)sys_.size(); ++q)
            if (sys_[q] == h) return q;
        return -1;
    }

    // an entry for h with one more user: the existing one, else a free one
    // (*fresh = true: the caller retains h and uploads its view), else -1
    // when every entry is in use (collect after a synchronisation may free
    // some)
    int acquire(Handle h, bool *fresh) {
        *fresh = false;
        int idx = find(h);
        if (idx < 0) {
            for (int q = 0; q < (int)sys_.size() && idx < 0; ++q)
                if (!live(q)) idx = q;
            if (idx < 0) {
                if ((int)sys_.size() >= cap_) return -1;
                idx = (int)sys_.size();
                sys_.push_back(Handle());
                users_.push_back(0);
            }
            sys_[idx] = h;
            users_[idx] = 0;
            *fresh = true;
        }
        users_[idx] += 1;
        return idx;
    }

    // one user of entry idx fewer (the entry stays until collected)
    void drop(int idx) {
        if (idx >= 0 && idx < (int)users_.size() && users_[idx] > 0) users_[idx] -= 1;
    }

    // free every listed entry without users; returns their handles, whose
    // references the caller releases
    std::vector<Handle> collect() {
        std::vector<Handle> out;
        for (int q = 0; q < (int)sys_.size(); ++q)
            if (live(q) && users_[q] == 0) {
                out.push_back(sys_[q]);
                sys_[q] = Handle();
            }
        return out;
    }

    // every listed handle (for the final release)
    std::vector<Handle> all() const {
        std::vector<Handle> out;
        for (int q = 0; q < (int)sys_.size(); ++q)
            if (live(q)) out.push_back(sys_[q]);
        return out;
    }

private:
    int cap_;
    std::vector<Handle> sys_;
    std::vector<int> users_;
};

}  // namespace hcn
