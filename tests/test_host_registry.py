"""Host logic of the batch's system registry (csrc/registry.hpp), on the CPU.

The registry lists the systems that a batch's slots use, holding a
reference on each, so that a system freed by its owner (or a new system
loaded at the same address) can never be confused with one still in use.
The checks drive the header with plain handles through the sequences the
batch and the server produce: add, release, free-then-reload, a full
registry, collection after a synchronisation.
"""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1501_06625_amd", "csrc")

DRIVER = r"""
#include <cassert>
#include <cstdio>
#include "registry.hpp"

// a stand-in for hcn_sys: a handle with a reference count
struct Sys { int refs = 1; bool freed = false; };
static void retain(Sys *s) { s->refs += 1; }
static void release(Sys *s) { if (--s->refs == 0) s->freed = true; }

int main() {
    using Reg = hcn::SysRegistry<Sys *>;
    Sys a, b, c;
    {
        // the same system twice shares an entry; a second one gets its own
        Reg r(2);
        bool fresh;
        int ia = r.acquire(&a, &fresh); assert(ia == 0 && fresh); retain(&a);
        int ia2 = r.acquire(&a, &fresh); assert(ia2 == 0 && !fresh);
        int ib = r.acquire(&b, &fresh); assert(ib == 1 && fresh); retain(&b);
        assert(r.users(0) == 2 && r.users(1) == 1);
        // full: a third system finds no entry until entries are collected
        int ic = r.acquire(&c, &fresh); assert(ic == -1);
        // the owner frees a: the registry's reference keeps it alive
        release(&a); assert(!a.freed && a.refs == 1);
        // both slots of a are released; nothing is dropped before collect()
        r.drop(ia); r.drop(ia2); assert(r.live(0));
        assert(r.find(&a) == 0);
        // after the queue has drained, collect drops a (its last reference)
        for (Sys *h : r.collect()) release(h);
        assert(a.freed && !r.live(0) && r.live(1));
        // the freed entry is reused for c
        ic = r.acquire(&c, &fresh); assert(ic == 0 && fresh); retain(&c);
        assert(r.find(&a) == -1 && r.find(&c) == 0);
        // b is still in use: collect keeps it
        assert(r.collect().empty());
        for (Sys *h : r.all()) release(h);
        assert(b.refs == 1 && c.refs == 1);
    }
    {
        // free-then-reload at the same address: the registry still holds the
        // old system, so "the same address" can only mean the same system
        Sys *s = new Sys;
        Reg r(4);
        bool fresh;
        int i0 = r.acquire(s, &fresh); retain(s);
        release(s);                 // the owner frees it: still alive
        assert(!s->freed);
        r.drop(i0);
        for (Sys *h : r.collect()) release(h);
        assert(s->freed);           // now gone, and no longer listed
        assert(r.find(s) == -1);
        delete s;
    }
    {
        // drop of an unknown or empty entry is harmless
        Reg r(1);
        r.drop(-1); r.drop(5);
        bool fresh;
        assert(r.acquire(&a, &fresh) == 0);
        r.drop(0); r.drop(0);
        assert(r.users(0) == 0);
    }
    std::puts("registry ok");
    return 0;
}
"""


def test_registry_logic():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "drv.cpp")
        exe = os.path.join(d, "drv")
        with open(src, "w") as f:
            f.write(DRIVER)
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, src, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
        assert out.returncode == 0, out.stderr
        assert "registry ok" in out.stdout
