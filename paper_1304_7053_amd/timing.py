"""Kernel timing on one GPU, shared by the autotuner and the benchmark.

A call is timed with a pair of HIP events recorded on its launch stream.  For
the events to bracket the kernels alone, the stream must already hold the
call when the first event is reached: a short kernel (6-20 us here) finishes
faster than Python and ctypes marshal the next launch, so an idle stream
would add the host's launch time to the interval.  Every timed series is
therefore queued behind a spin kernel (torch.cuda._sleep) long enough to
cover the host work of enqueueing it.

Between timed calls that must find their operands in HBM rather than in the
256 MB Infinity Cache, the cache is flushed by READING a 512 MB buffer
(clean lines only; a write would leave dirty lines that drain during the next
timed kernel), unless the caller rotates operand sets instead.
"""
import torch

_spin_cycles_per_us = None


def spin_rate():
    """Spin-kernel cycles per microsecond on this device (measured once)."""
    global _spin_cycles_per_us
    if _spin_cycles_per_us is None:
        torch.cuda.synchronize()
        cycles = 2_000_000
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(1000)
        e0.record()
        torch.cuda._sleep(cycles)
        e1.record()
        e1.synchronize()
        us = max(e0.elapsed_time(e1) * 1e3, 1.0)
        _spin_cycles_per_us = cycles / us
    return _spin_cycles_per_us


def spin(us):
    """Queue a kernel that keeps the current stream busy for about `us`."""
    torch.cuda._sleep(max(1, int(spin_rate() * us)))


class Flusher:
    """Evicts the Infinity Cache by reading a buffer twice its size."""

    def __init__(self, nbytes=512 << 20):
        self.buf = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        self.out = torch.empty((), dtype=torch.float32, device="cuda")

    def __call__(self):
        torch.sum(self.buf, dim=0, out=self.out)


def time_series(call, reps, host_us=60.0, flush=None):
    """Per-call durations (seconds) of `reps` calls of call(i), timed with
    event pairs on the current stream, the whole series queued behind a spin
    kernel; with `flush`, the cache is flushed (read) before each call,
    outside its events.  Returns the sorted list."""
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    spin(reps * host_us * (2 if flush is not None else 1) + 100.0)
    for i, (e0, e1) in enumerate(evs):
        if flush is not None:
            flush()
        e0.record(stream)
        call(i)
        e1.record(stream)
    torch.cuda.synchronize()
    return sorted(e0.elapsed_time(e1) / 1e3 for e0, e1 in evs)


def median(ts):
    return ts[len(ts) // 2]
