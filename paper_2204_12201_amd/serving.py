"""Continuous-batching request loop over the library (host side).

Requests of several kinds (a ciphertext product at one ring size, a p = 17
bridge conversion at another, an imputation query: the integer-weighted sums
of resident encrypted genotypes for one target's classes, then the bridge of
that target's class scores to bits and the one-hot argmax over the classes,
...) arrive over time.  The loop keeps each
kind's relinearization key resident, queues arrived requests per kind, and
whenever a kind's stream is idle admits the queued requests of that kind (up to
its batch cap) as one batch, as long as the device bytes of everything in
flight stay within a budget: inputs gathered into one buffer, the library's
workspace for the batch, and the outputs.  Each kind runs on its own HIP
stream (default priority), so batches of different kinds overlap on the
device, and requests that arrive while batches run are admitted as slots and
memory free up.  A batch is retired when its completion event has fired; every
request then records its latency from arrival to completion.

Requests carry their input ciphertexts already on the device; a result is the
request's own slice of its batch's output, the same words a call on that
request alone returns (products and conversions are independent per
ciphertext).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import fhe


@dataclass
class Request:
    rid: int
    kind: str
    arrival: float                 # seconds on the loop's clock
    x: object = None               # device [1][2][k][n] (first operand; unused by weighted sums)
    y: object = None               # device [1][2][k][n] second operand (products)
    w: object = None               # host int32 [rows][nin] weights (weighted sums)
    s: object = None               # device [rows][2][k][n] class scores at p (imputation queries)
    result: object = None          # device tensor once done; for imputation queries the
                                   # pair (weighted sums [rows], one-hot argmax [rows])
    done: float = None             # completion time on the loop's clock
    batch: int = 0                 # size of the batch it ran in

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class Lane:
    """One request kind: its context, resident key, stream and batch cap.
    op: "mul" (out = x * y, relinearized), "bridge" (the p-bit conversion
    of x, nbits bit ciphertexts), "wsum" (rows of integer weights applied to
    the lane's resident ciphertexts `shared`, one output per row) or "impute"
    (the weighted sums of "wsum", then the request's `rows` class scores at
    the bridge modulus of `ctx2` converted to nbits bits each and reduced to
    the one-hot argmax over the rows: the case study's query, its modular
    stage and its bit-level comparison; BFV has no switch between the two
    plaintext moduli, so the scores enter the bit-level stage as their own
    p-ary ciphertexts)."""
    kind: str
    ctx: object
    rlk: object
    op: str
    max_batch: int
    nbits: int = 0
    shared: object = None          # device [nin][2][k][n] resident inputs (wsum, impute)
    rows: int = 0                  # weight rows per request (wsum, impute)
    ctx2: object = None            # context of the bit-level stage (impute)
    rlk2: object = None
    stream: object = None
    queue: collections.deque = field(default_factory=collections.deque)
    inflight: tuple = None         # (requests, event, bytes, buffers)

    def bytes_for(self, count: int) -> int:
        c = self.ctx
        ct = c.ct_words * 8
        if self.op == "mul":
            ws = fhe.lib().fhe_workspace_bytes(c._h, fhe.OP_MUL_RELIN, count)
            return ws + 3 * count * ct
        if self.op in ("wsum", "impute"):
            nin = self.shared.shape[0]
            ws = fhe.lib().fhe_workspace_bytes(c._h, fhe.OP_WEIGHTED_SUM, count * self.rows * nin)
            total = ws + count * self.rows * ct
            if self.op == "impute":
                c2, m = self.ctx2, count * self.rows
                ct2 = c2.ct_words * 8
                total += max(fhe.lib().fhe_workspace_bytes(c2._h, fhe.OP_BRIDGE, m),
                             fhe.lib().fhe_workspace_bytes(c2._h, fhe.OP_ARGMAX, count))
                total += m * ct2 * (1 + 2 * self.nbits + 1)  # scores, bits and their class-major copy, argmax
            return total
        ws = fhe.lib().fhe_workspace_bytes(c._h, fhe.OP_BRIDGE, count)
        return ws + count * ct * (1 + self.nbits)


class Server:
    def __init__(self, lanes, budget_bytes: int):
        import torch
        self.torch = torch
        self.lanes = {ln.kind: ln for ln in lanes}
        for ln in lanes:
            ln.stream = torch.cuda.Stream(device=ln.ctx.device)
        self.budget = int(budget_bytes)
        self.in_flight_bytes = 0
        self.t0 = time.perf_counter()
        self.finished: list[Request] = []
        self.peak_bytes = 0
        self.max_concurrent = 0        # most lanes with a batch in flight at once

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request):
        self.lanes[req.kind].queue.append(req)

    def _launch(self, ln: Lane) -> bool:
        if ln.inflight is not None or not ln.queue:
            return False
        count = min(len(ln.queue), ln.max_batch)
        while count > 0 and self.in_flight_bytes + ln.bytes_for(count) > self.budget:
            count //= 2
        if count == 0:
            return False
        reqs = [ln.queue.popleft() for _ in range(count)]
        nbytes = ln.bytes_for(count)
        torch = self.torch
        with torch.cuda.stream(ln.stream):
            if ln.op == "wsum":
                out = ln.ctx.weighted_sum(ln.shared, np.concatenate([r.w for r in reqs]))
                bufs = (out,)
            elif ln.op == "impute":
                sums = ln.ctx.weighted_sum(ln.shared, np.concatenate([r.w for r in reqs]))
                sc = torch.cat([r.s for r in reqs]) if count > 1 else reqs[0].s  # [count * rows]
                bits = ln.ctx2.bridge_to_bits(ln.rlk2, sc, ln.nbits)
                k2, n2 = ln.ctx2.k, ln.ctx2.n
                cls = bits.view(count, ln.rows, ln.nbits, 2, k2, n2).transpose(0, 1).contiguous()
                hot = ln.ctx2.argmax(ln.rlk2, cls)  # [rows][count]
                out = (sums, hot)
                bufs = (sc, bits, cls, sums, hot)
            elif ln.op == "mul":
                xs = torch.cat([r.x for r in reqs]) if count > 1 else reqs[0].x
                ys = torch.cat([r.y for r in reqs]) if count > 1 else reqs[0].y
                out = ln.ctx.mul_relin(ln.rlk, xs, ys)
                bufs = (xs, ys, out)
            else:
                xs = torch.cat([r.x for r in reqs]) if count > 1 else reqs[0].x
                out = ln.ctx.bridge_to_bits(ln.rlk, xs, ln.nbits)
                bufs = (xs, out)
            ev = torch.cuda.Event()
            ev.record(ln.stream)
        per = ln.rows if ln.op in ("wsum", "impute") else 1
        for j, r in enumerate(reqs):
            if ln.op == "impute":
                r.result = (out[0][j * per:(j + 1) * per], out[1][:, j])
            else:
                r.result = out[j * per:(j + 1) * per]
            r.batch = count
        ln.inflight = (reqs, ev, nbytes, bufs)
        self.in_flight_bytes += nbytes
        self.peak_bytes = max(self.peak_bytes, self.in_flight_bytes)
        self.max_concurrent = max(self.max_concurrent,
                                  sum(lane.inflight is not None for lane in self.lanes.values()))
        return True

    def _retire(self, ln: Lane) -> bool:
        if ln.inflight is None:
            return False
        reqs, ev, nbytes, _ = ln.inflight
        if not ev.query():
            return False
        t = self.now()
        for r in reqs:
            r.done = t
        self.finished.extend(reqs)
        ln.inflight = None
        self.in_flight_bytes -= nbytes
        return True

    def step(self) -> bool:
        """Retire finished batches, then launch on idle lanes; True if anything
        changed."""
        changed = False
        for ln in self.lanes.values():
            changed |= self._retire(ln)
        for ln in self.lanes.values():
            changed |= self._launch(ln)
        return changed

    def busy(self) -> bool:
        return any(ln.inflight is not None or ln.queue for ln in self.lanes.values())

    def run(self, schedule):
        """schedule: requests sorted by arrival (seconds from the start).  Each is
        submitted when the clock reaches its arrival time; returns when all are
        done."""
        self.t0 = time.perf_counter()
        pending = collections.deque(schedule)
        while pending or self.busy():
            t = self.now()
            while pending and pending[0].arrival <= t:
                self.submit(pending.popleft())
            if not self.step():
                time.sleep(0.0002)
        return self.finished


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, -(-p * len(xs) // 100) - 1))
    return xs[int(i)]


def summary(finished, seconds: float) -> dict:
    out = {"completed": len(finished), "throughput_req_per_s": len(finished) / seconds if seconds else None}
    kinds = sorted({r.kind for r in finished})
    for kind in kinds + [None]:
        lat = [r.latency * 1e3 for r in finished if kind is None or r.kind == kind]
        bs = [r.batch for r in finished if kind is None or r.kind == kind]
        key = kind or "all"
        out[key] = {"count": len(lat), "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
                    "mean_batch": sum(bs) / len(bs) if bs else None}
    return out
