"""The Python binding's bookkeeping, on the CPU with a stand-in for the C library.

Only argument marshalling lives in the binding; what it must get right on its own
is keeping the plan and grids of a server ticket alive until the library reports
the ticket done (the server reads them until then).
"""
import ctypes
import gc
import weakref

import pytest

import paper_2506_22035_amd as sp


class _FakeLib:
    """Implements the four server calls the binding makes: tickets finish when told."""

    def __init__(self):
        self.next = 1
        self.done = set()

    def spider_server_create(self, budget, slots, queue, out):
        ctypes.cast(out, ctypes.POINTER(ctypes.c_void_p))[0] = 1234
        return 0

    def spider_submit(self, h, plan, xin, xout, steps, ticket):
        ctypes.cast(ticket, ctypes.POINTER(ctypes.c_uint64))[0] = self.next
        self.next += 1
        return 0

    def spider_poll(self, h, ticket, done, result):
        ctypes.cast(done, ctypes.POINTER(ctypes.c_int))[0] = 1 if ticket.value in self.done else 0
        ctypes.cast(result, ctypes.POINTER(ctypes.c_int))[0] = 0
        return 0

    def spider_server_destroy(self, h):
        return 0

    def spider_last_error(self):
        return b""


class _FakePlan:
    handle = ctypes.c_void_p(5678)

    def check_tensor(self, t):
        pass


class _FakeTensor:
    def data_ptr(self):
        return 4096


def test_server_keeps_ticket_objects_until_done(monkeypatch):
    fake = _FakeLib()
    monkeypatch.setattr(sp, "lib", lambda: fake)
    srv = sp.Server(1 << 20)
    plan, xin, xout = _FakePlan(), _FakeTensor(), _FakeTensor()
    refs = [weakref.ref(o) for o in (plan, xin, xout)]
    t = srv.submit(plan, xin, xout, 3)
    del plan, xin, xout
    gc.collect()
    assert all(r() is not None for r in refs)
    assert srv.poll(t) == (False, 0)
    assert all(r() is not None for r in refs)
    fake.done.add(t)
    assert srv.poll(t) == (True, 0)
    gc.collect()
    assert all(r() is None for r in refs)
    # a ticket reported done keeps answering from the binding
    assert srv.poll(t) == (True, 0)
    srv.close()


def test_server_close_releases_tickets_in_flight(monkeypatch):
    fake = _FakeLib()
    monkeypatch.setattr(sp, "lib", lambda: fake)
    srv = sp.Server(1 << 20)
    plan = _FakePlan()
    ref = weakref.ref(plan)
    srv.submit(plan, _FakeTensor(), _FakeTensor(), 1)
    del plan
    gc.collect()
    assert ref() is not None
    srv.close()
    gc.collect()
    assert ref() is None


def test_library_shares_torchs_hip_runtime():
    # Loaded before torch is imported, the library would bring its own HIP runtime and
    # torch a second one (torch's stream handles would then be foreign to the library,
    # and the runtime initialised second finds no GPU).  The binding imports torch
    # first, so one copy of libamdhip64 is mapped whatever the caller imports first.
    import subprocess
    import sys
    code = ("import paper_2506_22035_amd as sp; sp.lib(); import torch; "
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         cwd=sp.__path__[0] + "/..")
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"
