"""Continuous-batching server for selected Green's-function solves.

Requests arrive over time (each: block size b, block count n_b, N_E energies on
linspace(-2, 2, N_E), a seed for its random device, and a precision tag).  The
server

  * splits every request into energy chunks (energies are independent,
    Section II-A) and admits chunks in arrival order while their HBM
    footprint -- per-energy inputs and outputs, plus the request's H once --
    fits the budget, so large requests stream through the device (the
    library's workspace is a fixed cap per launch slot, outside the budget);
  * keeps a request's device H (generated on the device from the request's
    seed) resident until its last chunk finishes;
  * launches, whenever a launch slot is free, ONE qtx_rgf_solve over every
    admitted chunk not yet launched (chunks of different requests, block
    sizes and precisions in one call; the library batches per block size and
    runs block sizes concurrently);
  * keeps several launches in flight on separate streams (one library context
    per slot, each with its own workspace), so chunks admitted while others
    run overlap on the device -- continuous batching, not a queue;
  * on completion computes the transmission and contact current per energy
    on the device (qtx_rgf_observables), copies them out, frees the chunk and
    records latency = completion time - arrival time.

All arithmetic runs in the library; this module only schedules and marshals.
The executor is pluggable so the scheduling logic can be driven by a virtual
clock in tests.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional

import numpy as np

PRECISIONS = {
    "fp64": dict(prec="fp64"),
    # INT8 modular products, 10 moduli in the retarded chain and 11 in the lesser
    # chain: the fastest scheme that meets 1e-6 on the realistic workload
    "mixed": dict(prec="int8", n_slices=10, prec_lesser="int8", n_slices_lesser=11),
}


@dataclasses.dataclass
class Request:
    rid: int
    b: int
    n_b: int
    n_e: int
    seed: int
    precision: str = "fp64"
    t_arrive: float = 0.0
    keep_blocks: bool = False        # copy every output block to the host (verification; FPX
                                     # outputs as their bytes)
    # filled by the server
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    chunks_left: int = 0
    T_L: Optional[np.ndarray] = None
    j_L: Optional[np.ndarray] = None
    status: Optional[np.ndarray] = None
    blocks: Optional[Dict[str, np.ndarray]] = None
    rejected: bool = False

    @property
    def energies(self) -> np.ndarray:
        return np.linspace(-2.0, 2.0, self.n_e)

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.t_arrive


@dataclasses.dataclass
class Chunk:
    req: Request
    e0: int
    e1: int
    nbytes: int
    handle: object = None            # executor's device state


def request_stream(rate: float, duration: float, seed: int = 0, b_choices=None, nb_range=(8, 48),
                   ne_range=(16, 128), mixed_fraction: float = 0.5, first_id: int = 0) -> List[Request]:
    """Poisson arrivals at `rate` per second over `duration` seconds.  Per request:
    b uniform on b_choices (default 128, 160, ..., 512), n_b and N_E uniform
    integers in their ranges, precision mixed with probability mixed_fraction,
    seed = 1000 + id."""
    rng = np.random.default_rng(seed)
    if b_choices is None:
        b_choices = list(range(128, 513, 32))
    t = 0.0
    out = []
    rid = first_id
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        out.append(Request(rid=rid, b=int(rng.choice(b_choices)),
                           n_b=int(rng.integers(nb_range[0], nb_range[1] + 1)),
                           n_e=int(rng.integers(ne_range[0], ne_range[1] + 1)), seed=1000 + rid,
                           precision="mixed" if rng.random() < mixed_fraction else "fp64", t_arrive=t))
        rid += 1
    return out


class Server:
    """Scheduling core.  `executor` provides:
         footprint(req, n_energies) -> bytes          (per-chunk device memory)
         request_bytes(req) -> bytes                  (per-request memory, e.g. H)
         start_request(req) / finish_request(req)     (device-resident H)
         make_chunk(chunk)                            (device inputs/outputs)
         launch(slot, chunks)                         (one batched solve)
         poll(slot) -> bool                           (launch finished?)
         collect(chunk)                               (results to host, free)
         n_slots                                      (launches in flight)
    """

    def __init__(self, executor, hbm_budget: int, chunk_energies: int = 8, max_pending: int = 1 << 30,
                 clock: Callable[[], float] = time.perf_counter,
                 on_done: Optional[Callable[[Request], None]] = None, policy: str = "fifo",
                 max_wait: float = 10.0):
        if policy not in ("fifo", "sjf"):
            raise ValueError("policy: 'fifo' or 'sjf'")
        self.ex = executor
        self.on_done = on_done   # called with each request as it completes
        # admission order: "fifo" = arrival order; "sjf" = the pending request with the
        # least work first (flops of its selected solves), except that a request pending
        # for max_wait seconds or more is admitted first (no starvation)
        self.policy = policy
        self.max_wait = float(max_wait)
        self.budget = int(hbm_budget)
        self.chunk_energies = int(chunk_energies)
        self.max_pending = int(max_pending)
        self.clock = clock
        self.used = 0
        self.peak_used = 0
        self.pending: collections.deque = collections.deque()     # chunks waiting for admission
        self.ready: List[Chunk] = []                               # admitted, not launched
        self.inflight: Dict[int, List[Chunk]] = {}                 # slot -> chunks
        self.requests: List[Request] = []
        self.active_requests: Dict[int, Request] = {}
        self.launches = 0
        self.max_chunks_per_launch = 0

    # ---------------------------------------------------------------- intake
    def submit(self, req: Request, now: Optional[float] = None) -> bool:
        """Queue a request (split into energy chunks).  Returns False if rejected
        (too many pending chunks, or a chunk can never fit the budget)."""
        self.requests.append(req)
        chunks = []
        for e0 in range(0, req.n_e, self.chunk_energies):
            e1 = min(req.n_e, e0 + self.chunk_energies)
            chunks.append(Chunk(req, e0, e1, self.ex.footprint(req, e1 - e0)))
        too_big = any(c.nbytes + self.ex.request_bytes(req) > self.budget for c in chunks)
        if len(self.pending) + len(chunks) > self.max_pending or too_big:
            req.rejected = True
            return False
        req.chunks_left = len(chunks)
        self.pending.extend(chunks)
        return True

    # ---------------------------------------------------------------- one scheduling round
    def step(self) -> bool:
        """Admit, launch, collect.  Returns True if anything happened."""
        progress = False
        # collect finished launches
        for slot in list(self.inflight):
            if self.ex.poll(slot):
                for c in self.inflight.pop(slot):
                    self.ex.collect(c)
                    self.used -= c.nbytes
                    r = c.req
                    r.chunks_left -= 1
                    if r.chunks_left == 0:
                        r.t_done = self.clock()
                        self.ex.finish_request(r)
                        self.active_requests.pop(r.rid, None)
                        self.used -= self.ex.request_bytes(r)
                        if self.on_done is not None:
                            self.on_done(r)
                progress = True
        # admit while memory allows, in the policy's order (the chosen chunk must fit:
        # no overtaking past it, so every request eventually runs)
        while self.pending:
            i = self._pick()
            c = self.pending[i]
            r = c.req
            extra = 0 if r.rid in self.active_requests else self.ex.request_bytes(r)
            if self.used + c.nbytes + extra > self.budget:
                break
            del self.pending[i]
            if extra:
                r.t_admit = self.clock()
                self.ex.start_request(r)
                self.active_requests[r.rid] = r
                self.used += extra
            self.ex.make_chunk(c)
            self.used += c.nbytes
            self.peak_used = max(self.peak_used, self.used)
            self.ready.append(c)
            progress = True
        # launch everything admitted on a free slot
        if self.ready:
            free = [s for s in range(self.ex.n_slots) if s not in self.inflight]
            if free:
                slot = free[0]
                batch, self.ready = self.ready, []
                self.ex.launch(slot, batch)
                self.inflight[slot] = batch
                self.launches += 1
                self.max_chunks_per_launch = max(self.max_chunks_per_launch, len(batch))
                progress = True
        return progress

    @staticmethod
    def work(req: Request) -> float:
        """Flops of a request's selected solves: [144 (n_b - 1) + 24] b^3 per energy."""
        return req.n_e * (144.0 * (req.n_b - 1) + 24.0) * float(req.b) ** 3

    def _pick(self) -> int:
        """Index of the pending chunk to admit next."""
        if self.policy == "fifo" or len(self.pending) <= 1:
            return 0
        if self.clock() - self.pending[0].req.t_arrive >= self.max_wait:
            return 0          # the oldest request has waited long enough
        best, best_w = 0, None
        for i, c in enumerate(self.pending):
            w = self.work(c.req)
            if best_w is None or w < best_w:   # strict: the earliest chunk of the lightest request
                best, best_w = i, w
        return best

    def idle(self) -> bool:
        return not (self.pending or self.ready or self.inflight)

    # ---------------------------------------------------------------- drivers
    def run(self, arrivals: List[Request], time_limit: Optional[float] = None, sleep: float = 2e-4):
        """Real-time driver: submit requests when their arrival time has passed
        (arrival times are relative to the start), run until all are done or the
        time limit is reached."""
        t0 = self.clock()
        queue = collections.deque(sorted(arrivals, key=lambda r: r.t_arrive))
        while queue or not self.idle():
            now = self.clock() - t0
            if time_limit is not None and now > time_limit:
                break
            while queue and queue[0].t_arrive <= now:
                r = queue.popleft()
                r.t_arrive += t0
                self.submit(r)
            if not self.step():
                time.sleep(sleep)
        for r in queue:
            r.t_arrive += t0
            self.requests.append(r)
        return self.report(self.clock() - t0)

    def report(self, wall: float) -> dict:
        done = [r for r in self.requests if r.t_done is not None]
        lat = np.array([r.latency for r in done]) if done else np.array([])
        energies = int(sum(r.n_e for r in done))
        return {
            "requests": len(self.requests),
            "completed": len(done),
            "rejected": sum(r.rejected for r in self.requests),
            "unfinished": sum(1 for r in self.requests if r.t_done is None and not r.rejected),
            "energy_points": energies,
            "energy_points_per_s": energies / wall if wall > 0 else None,
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "wall_s": wall,
            "launches": self.launches,
            "max_chunks_per_launch": self.max_chunks_per_launch,
            "peak_hbm_bytes": self.peak_used,
        }


# ---------------------------------------------------------------------------
# GPU executor (the library does every step of the solve)
# ---------------------------------------------------------------------------

class GpuExecutor:
    """Device state and launches for Server on one GPU."""

    def __init__(self, n_slots: int = 3, device: int = 0, workspace_per_slot: int = 0, split: bool = False,
                 sigma_diag: bool = False, out_bits: int = 64):
        import torch
        from . import qtx
        self.torch = torch
        self.qtx = qtx
        self.n_slots = n_slots
        # solve every energy as two half-chains (QTX_SPLIT_CHAIN): about half the
        # sequential steps per launch, the same results to rounding, twice the
        # library workspace per energy
        self.split = split
        # compact storage (more energies fit the budget, same arithmetic):
        # sigma_diag -- the device's self-energies are scalar multiples of I per
        # block, so Sigma^R_ii and Sigma^<_ii travel as b-vectors (QTX_SIGMA_DIAG);
        # out_bits < 64 -- G^R_{i,i+1}, G^R_{i+1,i}, G^<_{i,i+1} are written as FPX
        # bytes of that width (Section V-A); the observables read only the
        # diagonal blocks, which stay complex128.
        self.sigma_diag = bool(sigma_diag)
        self.out_bits = 64 if out_bits in (0, 64) else int(out_bits)
        if self.out_bits != 64 and (self.out_bits % 8 or not 16 <= self.out_bits <= 56):
            raise ValueError("out_bits: 64 (complex128) or an FPX width 16, 24, .., 56")
        if split and self.out_bits != 64:
            raise ValueError("FPX outputs are not available for split chains")
        self.device = device
        self.ctx = [qtx.Context(device, workspace_bytes=workspace_per_slot) for _ in range(n_slots)]
        if workspace_per_slot:
            # claim the library workspaces before torch's caching allocator takes the memory
            for c in self.ctx:
                c.reserve_workspace(workspace_per_slot)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_slots)]
        self.events = [None] * n_slots
        self.H: Dict[int, tuple] = {}
        self.Sigma: Dict[tuple, object] = {}

    # memory model: per-energy inputs (Sigma^R, Sigma^<) and the five output arrays;
    # the request's H is counted once (request_bytes); the library's workspace is a
    # fixed per-slot cap (workspace_per_slot), outside this budget.
    def footprint(self, req: Request, n_energies: int) -> int:
        bb = req.b * req.b * 16
        sigma = 2 * req.n_b * (req.b * 16 if self.sigma_diag else bb)
        off_block = bb if self.out_bits == 64 else req.b * req.b * self.out_bits // 4
        return n_energies * (sigma + 2 * req.n_b * bb + 3 * (req.n_b - 1) * off_block)

    def request_bytes(self, req: Request) -> int:
        return (3 * req.n_b - 2) * req.b * req.b * 16

    def start_request(self, req: Request):
        """Random Hermitian BT H of the request, generated on the device from its seed."""
        torch = self.torch
        g = torch.Generator(device="cuda").manual_seed(req.seed)
        b, n_b = req.b, req.n_b
        kw = dict(device="cuda", dtype=torch.float64, generator=g)
        X = torch.complex(torch.randn(n_b, b, b, **kw), torch.randn(n_b, b, b, **kw)) / math.sqrt(2.0)
        H_d = (X + X.conj().transpose(1, 2)) / math.sqrt(2.0 * b)
        C = torch.complex(torch.randn(max(n_b - 1, 0), b, b, **kw), torch.randn(max(n_b - 1, 0), b, b, **kw))
        H_u = (math.sqrt(0.5 / b) / math.sqrt(2.0)) * C
        H_l = H_u.conj().transpose(1, 2).contiguous()
        self.H[req.rid] = (H_d.contiguous(), H_u.contiguous(), H_l)
        if req.keep_blocks:    # host copy of the inputs for verification
            req.blocks = {"H_d": H_d.cpu().numpy(), "H_u": H_u.cpu().numpy(), "H_l": H_l.cpu().numpy()}

    def finish_request(self, req: Request):
        self.H.pop(req.rid, None)

    def make_chunk(self, c: Chunk):
        from . import inputs
        torch = self.torch
        req = c.req
        E = req.energies[c.e0:c.e1]
        sr, sl = inputs.random_bt_scalars(req.n_b, E)
        H_d, H_u, H_l = self.H[req.rid]
        n_e, n_b, b = E.size, req.n_b, req.b
        kw = dict(dtype=torch.complex128, device="cuda")

        def sigma(scal):
            if not self.sigma_diag:
                return inputs.diag_blocks_device(scal, b)
            d = torch.from_numpy(np.ascontiguousarray(scal)).to("cuda")
            return d[:, :, None].expand(n_e, n_b, b).contiguous()

        def offdiag():
            if self.out_bits == 64:
                return torch.empty((n_e, n_b - 1, b, b), **kw)
            return torch.empty((n_e, n_b - 1, b * b * self.out_bits // 4), dtype=torch.uint8, device="cuda")
        dp = self.qtx.DeviceProblem(
            energies=E, H_d=H_d, H_u=H_u, H_l=H_l, SR_d=sigma(sr), SL_d=sigma(sl),
            GR_d=torch.empty((n_e, n_b, b, b), **kw), GR_u=offdiag(), GR_l=offdiag(),
            GL_d=torch.empty((n_e, n_b, b, b), **kw), GL_u=offdiag(),
            status=torch.full((n_e,), -1, dtype=torch.int32, device="cuda"), split=self.split,
            sigma_diag=self.sigma_diag, out_bits=self.out_bits)
        c.handle = dp

    def launch(self, slot: int, chunks: List[Chunk]):
        from . import inputs
        torch = self.torch
        s = self.streams[slot]
        # inputs were produced on the current stream: order the slot's stream after them
        s.wait_stream(torch.cuda.current_stream())
        dps = [c.handle for c in chunks]
        sch = [PRECISIONS[c.req.precision] for c in chunks]
        with torch.cuda.stream(s):
            self.ctx[slot].solve(dps, prec=[x["prec"] for x in sch], n_slices=[x.get("n_slices", 0) for x in sch],
                                 prec_lesser=[x.get("prec_lesser") for x in sch],
                                 n_slices_lesser=[x.get("n_slices_lesser", -1) for x in sch], stream=s)
            for c in chunks:
                dp = c.handle
                # contact broadening and occupation of the left lead (inputs of the device model)
                gam = 2.0 * 0.5 * np.eye(dp.b)
                fL = inputs.fermi(dp.energies, 0.1, 0.025)
                c.obs = self.ctx[slot].observables(dp, gam, fL, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        self.events[slot] = ev

    def poll(self, slot: int) -> bool:
        ev = self.events[slot]
        return ev is None or ev.query()

    def collect(self, c: Chunk):
        dp = c.handle
        req = c.req
        T, j = c.obs
        n = req.n_e
        if req.T_L is None:
            req.T_L = np.zeros(n)
            req.j_L = np.zeros(n)
            req.status = np.zeros(n, dtype=np.int32)
            if req.keep_blocks and req.blocks is None:
                req.blocks = {}
        req.T_L[c.e0:c.e1] = T.cpu().numpy()
        req.j_L[c.e0:c.e1] = j.cpu().numpy()
        req.status[c.e0:c.e1] = dp.status.cpu().numpy()
        if req.keep_blocks:
            for k in ("GR_d", "GR_u", "GR_l", "GL_d", "GL_u"):
                v = getattr(dp, k).cpu().numpy()
                if k not in req.blocks:
                    req.blocks[k] = np.zeros((n,) + v.shape[1:], dtype=v.dtype)
                req.blocks[k][c.e0:c.e1] = v
        c.handle = None
        c.obs = None

    def close(self):
        for c in self.ctx:
            c.close()
