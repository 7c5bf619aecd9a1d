"""The Python binding's stream handling, on the CPU: a call given a stream
runs with that stream as torch's current one (so the binding's own
allocations and fills are ordered with the library's kernels there), and
every public call that takes a stream is wrapped that way."""
import inspect

from paper_1712_03439_amd import rsim


def test_a_given_stream_is_current_for_the_whole_call(monkeypatch):
    seen = []

    class Ctx:
        def __init__(self, s):
            self.s = s

        def __enter__(self):
            seen.append(("enter", self.s))

        def __exit__(self, *exc):
            seen.append(("exit", self.s))

    class FakeTorch:
        class cuda:
            stream = Ctx

    monkeypatch.setattr(rsim, "_torch", lambda: FakeTorch)

    @rsim._on_stream
    def call(a, b=1, stream=None):
        seen.append(("body", stream))
        return a + b

    assert call(1) == 2 and seen == [("body", None)]
    seen.clear()
    assert call(1, 2, "s") == 3 and seen == [("enter", "s"), ("body", "s"), ("exit", "s")]
    seen.clear()
    assert call(1, stream="t") == 2 and seen == [("enter", "t"), ("body", "t"), ("exit", "t")]


def test_every_call_taking_a_stream_is_wrapped():
    unwrapped = []
    for name, fn in inspect.getmembers(rsim, inspect.isfunction):
        if name.startswith("_") or fn.__module__ != rsim.__name__ or name == "device_status":
            continue
        if "stream" in inspect.signature(fn).parameters and not hasattr(fn, "__wrapped__"):
            unwrapped.append(name)
    assert not unwrapped, unwrapped
