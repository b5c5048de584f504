"""Serving loop: continuous batching of many fine DNN-MG flows on one GPU.

Requests (a channel mesh size, a step count, a field seed and an arrival
time) are admitted while a slot is free and their device memory fits the HBM
budget; every tick steps all active flows together with one batched,
graph-captured launch (dnnmg_batch_prepare + dnnmg_batch_launch), so requests
that arrive while others run join at the next tick boundary and finished ones
leave.  Each flow keeps its GRU state and corrected velocity resident on the
device between ticks.

The flows' state and workspace live in one device arena made when the server
starts (dnnmg_arena_*): admitting a request carves its block and enqueues its
set-up on the serving stream, retiring it returns the block; neither
allocates, frees or waits for the stream, so the ticks already in flight keep
the GPU busy while the host admits and retires.

The coarse solve is not part of this build: each admitted request gets a ring
of `ring` coarse (v, p) time levels evaluated on the device from its seeded
Fourier field (calibrated on the device too, without a read-back), and step
n reads level n mod ring.

Per-step latency is the time from the moment a flow's step becomes eligible
(its admission, or the completion of its previous step) to the completion of
the tick that carries it.  Ticks are pipelined: while the GPU runs one, the
host admits arrivals and issues the next, and a flow's block is returned only
after the tick with its last step has finished.  The per-tick flow table is
formed from numpy arrays of handles and device pointers, rebuilt only when
the membership changes.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import DnnMG, Arena, Batch, DnnmgError, DNNMG_ENOMEM, make_config, synth


class Scheduler:
    """Admission policy (host logic only): requests wait in arrival order and
    are admitted first come, first served while fewer than max_flows run and
    their bytes fit the remaining budget.  A request larger than the whole
    budget is refused."""

    def __init__(self, budget: int, max_flows: int, cost):
        self.budget, self.max_flows, self.cost = int(budget), int(max_flows), cost
        self.used, self.running, self.queue = 0, 0, []

    def arrive(self, req):
        if self.cost(req) > self.budget:
            raise ValueError("request %s needs %d bytes, more than the whole budget of %d"
                             % (req.get("id"), self.cost(req), self.budget))
        self.queue.append(req)

    def admissible(self, limit=None):
        """Pop and return the requests that can start now (at most `limit`)."""
        out = []
        while (self.queue and self.running < self.max_flows and self.used + self.cost(self.queue[0]) <= self.budget
               and (limit is None or len(out) < limit)):
            r = self.queue.pop(0)
            self.used += self.cost(r)
            self.running += 1
            out.append(r)
        return out

    def requeue(self, req):
        """Undo the admission of req (its memory could not be placed yet):
        it goes back to the head of the queue."""
        self.used -= self.cost(req)
        self.running -= 1
        self.queue.insert(0, req)

    def release(self, req):
        self.used -= self.cost(req)
        self.running -= 1


@dataclass
class Active:
    req: dict
    idx: int                 # the request's row in the server's per-request arrays
    ctx: DnnMG
    vring: object            # (ring, Nc*2) float32 device view (its row stride spans the flow's ring group)
    pring: object            # (ring, Nc) float32 device view (likewise)
    b_out: object            # (Nc*2,) float64 device tensor: restricted rhs of the last step
    admitted: float = 0.0


class Server:
    def __init__(self, K=2, H=64, Hm=64, precision="bf16", weight_seed=1234, nu=1e-3, dt=0.005,
                 hbm_budget=None, max_flows=64, ring=8, use_graph=True, stream=None):
        import torch
        self.K, self.H, self.Hm, self.precision = K, H, Hm, precision
        self.nu, self.dt, self.ring, self.use_graph = nu, dt, ring, use_graph
        self.max_flows = max_flows
        self.stream = stream if stream is not None else torch.cuda.Stream()
        w = synth.xavier_weights(K, H, Hm, weight_seed)
        with torch.cuda.stream(self.stream):
            # a one-patch context that owns the shared weights
            self.model = DnnMG(make_config(1, 1, K, H, Hm, dt, nu, precision, 15),
                               synth.rect_mesh(1, 1), w, stream=self.stream)
        free, total = torch.cuda.mem_get_info()
        self.hbm_budget = int(hbm_budget if hbm_budget is not None else min(0.5 * free, 16 << 30))
        self.arena = Arena(self.hbm_budget)
        self.batch = Batch(max_flows)

    def warmup(self):
        """Before any request is timed: one tick of the model's own one-patch
        context (captures the batch graph, loads the kernels), then one small
        request taken through admission, a tick beside the model's context and
        retirement, so that the first use of every host and device path of a
        request (context creation, the kernels that evaluate its field ring)
        falls outside the measurement.  The shared weights are not changed by
        a step."""
        import torch
        nc = self.model.s["Nc"]
        with torch.cuda.stream(self.stream):
            v = torch.zeros(2 * nc, dtype=torch.float32, device="cuda")
            p = torch.zeros(nc, dtype=torch.float32, device="cuda")
            b = torch.empty(2 * nc, dtype=torch.float64, device="cuda")
            self.batch.prepare([self.model], [v], [p], None, [b], stream=self.stream)
            self.batch.launch(graph=self.use_graph, stream=self.stream)
        self.stream.synchronize()
        a = self.admit(dict(id=-1, nx=4, ny=2, steps=1, field_seed=0), -1, 0.0)
        with torch.cuda.stream(self.stream):
            self.batch.prepare([self.model, a.ctx], [v, a.vring[0]], [p, a.pring[0]], None, [b, a.b_out],
                               stream=self.stream)
            self.batch.launch(graph=self.use_graph, stream=self.stream)
        self.stream.synchronize()
        self.retire(a)

    def config(self, nx, ny):
        return make_config(nx, ny, self.K, self.H, self.Hm, self.dt, self.nu, self.precision, synth.DIR_CHANNEL)

    def flow_bytes(self, nx, ny):
        """Arena bytes of one request's flow (state and workspace)."""
        return Arena.block_bytes(self.config(nx, ny))

    # nodes of one group evaluation of the field rings (its FP64 temporaries
    # take about 0.5 KB per node)
    RING_GROUP_NODES = 1 << 18

    def admit_group(self, reqs, now):
        """Contexts in the arena for reqs, in order, and their field rings,
        all enqueued on the serving stream.  Returns (admitted Active list,
        the requests from the first one the arena has no block for yet)."""
        import torch
        made = []
        with torch.cuda.stream(self.stream):
            for i, r in enumerate(reqs):
                cxy = synth.rect_mesh(r["nx"], r["ny"], synth.CHANNEL_LX, synth.CHANNEL_LY)
                try:
                    ctx = DnnMG(self.config(r["nx"], r["ny"]), cxy, share=self.model, stream=self.stream,
                                arena=self.arena)
                except DnnmgError as e:
                    if e.code == DNNMG_ENOMEM:
                        return self._rings(made, now), list(reqs[i:])
                    raise
                made.append((r, ctx))
            return self._rings(made, now), []

    def _rings(self, made, now):
        """Field rings of (request, context) pairs, evaluated in groups of at
        most RING_GROUP_NODES nodes (a flow's values do not depend on its
        group), as Active records."""
        import torch
        out = []
        times = self.dt * np.arange(self.ring, dtype=np.float64)
        i = 0
        while i < len(made):
            j, nodes = i, 0
            while j < len(made) and (j == i or nodes + made[j][1].s["Nc"] <= self.RING_GROUP_NODES):
                nodes += made[j][1].s["Nc"]
                j += 1
            grp = made[i:j]
            ffs = [synth.FourierField(synth.CHANNEL_LX, synth.CHANNEL_LY, r["field_seed"]) for r, _ in grp]
            v, p, offs = synth.channel_rings_torch(
                ffs, [(r["nx"], r["ny"]) for r, _ in grp], times, synth.CHANNEL_LX, synth.CHANNEL_LY, 1.5,
                synth.CHANNEL_LY, "cuda", upload=lambda dst, src: self.arena.upload(dst, src, self.stream))
            v32, p32 = v.float(), p.float()       # ring x nodes (x 2), the group's flows in order
            for k, (r, ctx) in enumerate(grp):
                a, n = int(offs[k]), int(offs[k + 1] - offs[k])
                # views of the group's FP32 arrays: level l of the flow is a
                # contiguous run at vring[l], the row stride spans the group
                vring = v32[:, a:a + n].reshape(self.ring, 2 * n)
                pring = p32[:, a:a + n]
                b_out = torch.empty(2 * ctx.s["Nc"], dtype=torch.float64, device="cuda")
                out.append(Active(r, r.get("_idx", -1), ctx, vring, pring, b_out, admitted=now))
            i = j
        return out

    def admit(self, req, idx, now):
        """admit_group for one request; None if the arena has no block for it
        yet."""
        acts, rest = self.admit_group([dict(req, _idx=idx)], now)
        return acts[0] if acts else None

    def retire(self, a, results=None, steps=0):
        import torch
        if results is not None:
            h = torch.empty(a.ctx.s["P"] * self.H, dtype=torch.float32, device="cuda")
            u = torch.empty(2 * a.ctx.s["Fn"], dtype=torch.float32, device="cuda")
            with torch.cuda.stream(self.stream):
                a.ctx.get_state(h, u, stream=self.stream)
            self.stream.synchronize()
            results[a.req["id"]] = dict(h=h.cpu().numpy(), u=u.cpu().numpy(), bL=a.b_out.cpu().numpy(),
                                        steps=steps, queue_delay=a.req["admitted_at"] - a.req["queued_at"])
        a.ctx.close()

    def run(self, requests, time_scale=1.0, log_every=0.0, results=None, depth=2, admit_burst=4):
        """Serve `requests` (dicts with id, arrival [s], nx, ny, steps,
        field_seed).  Arrival times are divided by time_scale (10 = ten times
        the offered rate).  Up to `depth` ticks are in flight: the host admits
        requests and prepares tick n+1 while the GPU runs tick n (stream order
        keeps them apart); while ticks are in flight at most `admit_burst`
        requests are admitted between two ticks.  Returns pooled statistics; with a dict `results`,
        also each request's final state (h, corrected velocity) and last b_L."""
        import collections
        import torch
        self.warmup()
        pending = sorted((dict(r) for r in requests), key=lambda r: r["arrival"])
        nreq = len(pending)
        # per-request arrays (row = position in arrival order)
        nsteps = np.array([r["steps"] for r in pending], dtype=np.int64)
        npatch = np.array([r["nx"] * r["ny"] for r in pending], dtype=np.int64)
        issued = np.zeros(nreq, dtype=np.int64)
        completed = np.zeros(nreq, dtype=np.int64)
        eligible = np.zeros(nreq)
        for i, r in enumerate(pending):
            r["_idx"] = i
        sched = Scheduler(self.hbm_budget, self.max_flows, lambda r: self.flow_bytes(r["nx"], r["ny"]))
        active = []                      # flows still issuing steps, in table order
        by_idx = {}                      # request row -> Active, until retired
        table = None                     # (rows, handles, vbase, pbase, bptr, vstride, pstride) of `active`
        inflight = collections.deque()   # ticks on the GPU: (start event, end event, member rows)
        spare = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(depth + 1)]
        stats = dict(ticks=0, conc=0, patch_steps=0, busy=0.0, max_conc=0, done=0)
        latencies = []
        qdelay = []
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        last_log = 0.0

        def build_table():
            rows = np.array([a.idx for a in active], dtype=np.int64)
            u = np.uintp
            handles = np.array([a.ctx.handle.value for a in active], dtype=u)
            vbase = np.array([a.vring.data_ptr() for a in active], dtype=u)
            pbase = np.array([a.pring.data_ptr() for a in active], dtype=u)
            bptr = np.array([a.b_out.data_ptr() for a in active], dtype=u)
            vstride = np.array([a.vring.stride(0) * 4 for a in active], dtype=u)
            pstride = np.array([a.pring.stride(0) * 4 for a in active], dtype=u)
            return rows, handles, vbase, pbase, bptr, vstride, pstride

        def complete_oldest():
            e0, e1, rows = inflight.popleft()
            e1.synchronize()
            t_done = now()
            stats["busy"] += e0.elapsed_time(e1) / 1e3
            spare.append((e0, e1))
            latencies.append(t_done - eligible[rows])
            eligible[rows] = t_done
            completed[rows] += 1
            stats["patch_steps"] += int(npatch[rows].sum())
            for i in rows[completed[rows] >= nsteps[rows]]:
                a = by_idx.pop(int(i))
                a.req["finished_at"] = t_done
                qdelay.append(a.req["admitted_at"] - a.req["queued_at"])
                self.retire(a, results, steps=int(issued[i]))
                sched.release(a.req)
                stats["done"] += 1
            return t_done

        while pending or sched.queue or active or inflight:
            t = now()
            while pending and pending[0]["arrival"] / time_scale <= t:
                r = pending.pop(0)
                r["queued_at"] = r["arrival"] / time_scale
                sched.arrive(r)
            # admissions, a few at a time while ticks are in flight (each
            # costs host time: its set-up and field ring are enqueued), so
            # the active flows' next tick is not held back by a burst
            cap = admit_burst if inflight else len(sched.queue)
            acts, unplaced = self.admit_group(sched.admissible(limit=cap), now())
            for r in reversed(unplaced):      # the arena is fragmented: wait for a release
                sched.requeue(r)
            for a in acts:
                a.req["admitted_at"] = a.admitted
                eligible[a.idx] = a.admitted
                active.append(a)
                by_idx[a.idx] = a
            if acts:
                table = None
            stats["max_conc"] = max(stats["max_conc"], len(active))
            if active and len(inflight) < depth:
                # issue one tick: every active flow advances one step
                if table is None:
                    table = build_table()
                rows, handles, vbase, pbase, bptr, vstride, pstride = table
                lvl = (issued[rows] % self.ring).astype(np.uintp)
                vptr = vbase + lvl * vstride
                pptr = pbase + lvl * pstride
                e0, e1 = spare.pop()
                with torch.cuda.stream(self.stream):
                    self.batch.prepare_raw(len(rows), handles, vptr, pptr, bptr, stream=self.stream)
                    e0.record(self.stream)
                    self.batch.launch(graph=self.use_graph, stream=self.stream)
                    e1.record(self.stream)
                inflight.append((e0, e1, rows))
                stats["ticks"] += 1
                stats["conc"] += len(rows)
                issued[rows] += 1
                if np.any(issued[rows] >= nsteps[rows]):
                    active = [a for a in active if issued[a.idx] < nsteps[a.idx]]
                    table = None
                continue
            if inflight:
                t_done = complete_oldest()
                if log_every and t_done - last_log > log_every:
                    last_log = t_done
                    print("serve: t=%.1fs active=%d queued=%d done=%d" % (t_done, len(active), len(sched.queue),
                                                                           stats["done"]), flush=True)
            elif pending:
                time.sleep(max(0.0, min(pending[0]["arrival"] / time_scale - now(), 0.01)))
        wall = now()
        lat = np.concatenate(latencies) if latencies else np.zeros(0)
        qd = np.asarray(qdelay)
        ticks = stats["ticks"]
        return {
            "requests": stats["done"],
            "steps": int(lat.size),
            "ticks": ticks,
            "depth": depth,
            "wall_s": wall,
            "gpu_busy_s": stats["busy"],
            "gpu_busy_frac": stats["busy"] / wall if wall > 0 else 0.0,
            "patch_steps": stats["patch_steps"],
            "patch_steps_per_s": stats["patch_steps"] / wall if wall > 0 else 0.0,
            "mean_concurrency": stats["conc"] / ticks if ticks else 0.0,
            "max_concurrency": stats["max_conc"],
            "p50_step_latency_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_step_latency_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "max_step_latency_ms": float(lat.max() * 1e3) if lat.size else None,
            "p50_queue_delay_ms": float(np.percentile(qd, 50) * 1e3) if qd.size else None,
            "p99_queue_delay_ms": float(np.percentile(qd, 99) * 1e3) if qd.size else None,
            "graph": self.use_graph,
        }

    def close(self):
        self.batch.close()
        self.arena.close()
        self.model.close()
