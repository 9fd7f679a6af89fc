"""Host-side checks of the Python binding's stream bookkeeping, without a
GPU: a call on a stream other than the current one makes that stream wait
for the current one and records every tensor it touches as used there."""
import paper_2108_04791_amd as isp


class FakeStream:
    def __init__(self, name):
        self.name = name
        self.device = 0
        self.waited = []

    def wait_stream(self, other):
        self.waited.append(other.name)

    def __eq__(self, other):
        return isinstance(other, FakeStream) and other.name == self.name

    def __hash__(self):
        return hash(self.name)


class FakeTensor:
    is_cuda = True

    def __init__(self):
        self.recorded = []

    def record_stream(self, s):
        self.recorded.append(s.name)


def test_other_stream_waits_and_records(monkeypatch):
    cur = FakeStream("current")
    monkeypatch.setattr(isp.torch.cuda, "current_stream", lambda device=None: cur)
    side = FakeStream("side")
    a, b = FakeTensor(), FakeTensor()
    isp._on_stream(side, a, b, None)
    assert side.waited == ["current"]
    assert a.recorded == ["side"] and b.recorded == ["side"]


def test_current_or_default_stream_untouched(monkeypatch):
    cur = FakeStream("current")
    monkeypatch.setattr(isp.torch.cuda, "current_stream", lambda device=None: cur)
    a = FakeTensor()
    isp._on_stream(None, a)
    isp._on_stream(FakeStream("current"), a)
    assert a.recorded == [] and cur.waited == []
