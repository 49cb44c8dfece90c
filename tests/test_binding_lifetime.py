"""Handle lifetimes in the Python binding, checked without a device: a reference
cycle that holds a Problem (a test frame kept alive by an exception's traceback,
as `pytest.raises(...) as e` leaves behind) keeps its Context alive only through
the cycle, and the cyclic collector finalizes the members of a cycle in no fixed
order, so goac_problem_destroy may follow goac_ctx_destroy. The library frees a
context only after the last problem or chain set made on it is destroyed, so
either order is valid; the binding must destroy each handle exactly once."""
import gc

import paper_2409_08808_amd as G


class _RecordingLib:
    def __init__(self):
        self.calls = []

    def goac_ctx_destroy(self, h):
        self.calls.append(("ctx", h))

    def goac_problem_destroy(self, h):
        self.calls.append(("problem", h))

    def goac_chains_destroy(self, h):
        self.calls.append(("chains", h))


def test_cycle_finalizes_context_and_dependents_once(monkeypatch):
    lib = _RecordingLib()
    monkeypatch.setattr(G, "_lib", lib)
    ctx = object.__new__(G.Context)
    ctx._h = 1
    pb = object.__new__(G.Problem)
    pb._h, pb.ctx = 2, ctx
    ch = object.__new__(G.Chains)
    ch._h, ch.ctx = 3, ctx
    cycle = [ctx, pb, ch]
    cycle.append(cycle)
    del ctx, pb, ch, cycle
    gc.collect()
    assert sorted(lib.calls) == [("chains", 3), ("ctx", 1), ("problem", 2)]
    # the order the collector chose (the context may come first)
    print("finalization order:", [c[0] for c in lib.calls])


def test_explicit_close_is_idempotent(monkeypatch):
    lib = _RecordingLib()
    monkeypatch.setattr(G, "_lib", lib)
    ctx = object.__new__(G.Context)
    ctx._h = 7
    ctx.close()
    ctx.close()
    del ctx
    gc.collect()
    assert lib.calls == [("ctx", 7)]
