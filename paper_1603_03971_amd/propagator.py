"""Time stepping of one subdomain: the per-step phase sequence of the paper's section II.

One step n (u^{n+1} from u^n and u^{n-1}) runs, in the default "overlap" schedule, on two HIP
streams like the paper's halo-first schedule with a communication thread:

    halo stream H:      wait(interior n-1) -> rtm_step_halo_pack (the halo update, which also writes
                        the faces) -> inject shell sources and re-copy those in faces -> [halo done]
                        -> exchange -> rtm_unpack_halo
    interior stream I:  rtm_step_interior -> inject interior sources -> wait(halo done)
                        -> rtm_record -> [level n+1 complete]

The exchange is where a multi-GPU run would send the packed faces; one subdomain uses its physical
boundary (NULL slots: zero ghosts) or a periodic self-exchange (slot f receives the opposite face,
a pointer swap with no copy).  Time levels rotate by pointer: by default u^{n+1} overwrites
u^{n-1} in place (two buffers), and a level that must outlive the rotation (an RTM snapshot) is
"pinned" so that the next write goes to a fresh buffer instead of copying it.

The "serial" schedule runs the same phases on one stream (the halo call that packs, shell sources,
interior call, interior sources, unpack, record); both give bitwise identical fields.

With ghosts="slots" (serial and overlap schedules, radius 4, nx % 4 == 0) the unpack pass goes away:
the ghosts of level n stay in the receive slots that the exchange filled, and step n's halo call reads
them there (rtm_step_halo_pack_slots); the interior call reads no ghost cell.  The level buffers'
ghost rings are then not kept (fill_ghosts() writes the newest level's from its slots), and the face
buffer alternates between two buffers, since step n + 1 packs while a periodic exchange still has
step n's faces in use as its receive slots.  Same bits as ghosts="ring".

With ghosts="slots" and halo="shell" the halo call only produces the faces: rtm_step_shell_pack
computes the owned cells within R of a face into the send buffer (reading the x faces of u^n, u^{n-1}
and kappa densely from the face buffers of the last two steps and a packed copy of kappa's faces),
and rtm_step_whole_slots then updates every owned cell in one launch of full-width tiles, the shell
again included (about 5% of the cells at 512^3), on the interior stream; the sources are injected
after it and those in face cells re-copied into the send buffer.  The face buffers rotate over three
(step n writes the faces of u^{n+1} while those of u^n and u^{n-1} are read).  Same bits.  The
"fused" schedule, for one subdomain with nothing to overlap, updates every owned cell in one launch
(rtm_step_whole) instead of the halo and interior calls, then injects, refreshes the ghosts and
records on one stream; it too is bitwise identical.  With no face received (the physical boundary),
the ghost ring of a level buffer holds zeros once written, and the refresh is skipped for buffers
known to be in that state.
"""
from __future__ import annotations

import weakref

import numpy as np
import torch

from . import _abi
from .grid import Grid

OPPOSITE = [1, 0, 3, 2, 5, 4]


class Sources:
    """Point sources (or receivers re-injecting data): cells, weights and an amplitude table.

    amp has shape (nsteps, n): row n is injected after step n.  On the device the sources are split
    into the cells the halo call updates and the rest, so that each source is added on the stream
    that wrote its cell, and halo-region sources before the pack."""

    def __init__(self, grid: Grid, ijk, weights, amp, reverse_time: bool = False):
        ijk = np.asarray(ijk, dtype=np.int64).reshape(-1, 3)
        w = np.asarray(weights, dtype=np.float32).reshape(-1)
        if isinstance(amp, torch.Tensor):
            amp_t = amp.to(device=grid.device, dtype=torch.float32)
        else:
            amp_t = torch.from_numpy(np.ascontiguousarray(amp, dtype=np.float32)).to(grid.device)
        amp_t = amp_t.reshape(-1, len(w))
        if reverse_time:
            amp_t = torch.flip(amp_t, dims=[0])
        self.nsteps = amp_t.shape[0]
        self._ijk, self._w = ijk, w
        self._order = np.arange(len(w))
        self.amp = amp_t.contiguous()
        self._split(grid)

    def _split(self, grid: Grid):
        """Order the sources as halo region first, then the rest, for the halo region of the current
        options (rtm_halo_region); self.amp's columns follow the order."""
        ijk, w = self._ijk, self._w
        self.widths = _abi.rtm_halo_region(grid.c)
        shell = grid.in_halo(ijk)
        # halo-region cells within R of a face: packed by the halo call before their injection, so
        # re-copied into the face buffer after it (rtm_pack_cells)
        R = grid.radius
        face = shell & ((ijk[:, 0] < R) | (ijk[:, 0] >= grid.nx - R) | (ijk[:, 1] < R) | (ijk[:, 1] >= grid.ny - R)
                        | (ijk[:, 2] < R) | (ijk[:, 2] >= grid.nz - R))
        self.face_idx = torch.from_numpy(grid.index(ijk[face])).to(grid.device) if face.any() else None
        # one table with the halo-region sources first: set 0 (halo region), set 1 (the rest) and set 2
        # (all, for a schedule that updates every cell in one launch) are column ranges of it
        order = np.concatenate([np.nonzero(shell)[0], np.nonzero(~shell)[0]])
        n0 = int(shell.sum())
        self.count = len(order)
        self.idx = torch.from_numpy(grid.index(ijk[order])).to(grid.device)
        self.w = torch.from_numpy(w[order]).to(grid.device)
        # the table's columns are in self._order; re-order them to `order`
        pos = np.empty(len(order), dtype=np.int64)
        pos[self._order] = np.arange(len(order))
        self.amp = self.amp[:, torch.from_numpy(pos[order]).to(grid.device)].contiguous()
        self._order = order
        self.ranges = [(0, n0), (n0, self.count - n0), (0, self.count)]

    def ensure_split(self, grid: Grid):
        """Re-split when the halo region changed since the split (an option set between steps), so
        every source is still added by the call that owns its cell.  Rare: it waits for the device,
        so that no kernel still reads the tables it replaces."""
        if _abi.rtm_halo_region(grid.c) != self.widths:
            torch.cuda.synchronize(grid.device)
            self._split(grid)

    def inject_args(self, n: int, which: int):
        """(index, weight and amplitude addresses, count) of row n at set `which` (0 = halo region,
        1 = the rest, 2 = all), or None when there is nothing to add."""
        off, cnt = self.ranges[which]
        if cnt == 0 or n >= self.nsteps:
            return None
        return (self.idx.data_ptr() + 8 * off, self.w.data_ptr() + 4 * off,
                self.amp.data_ptr() + 4 * (n * self.count + off), cnt)

    def inject(self, grid: Grid, u: torch.Tensor, n: int, which: int, stream):
        """Add row n of the amplitude table at set `which`: 0 = halo region, 1 = the rest, 2 = all."""
        a = self.inject_args(n, which)
        if a is not None:
            _abi.rtm_inject(grid.c, u, *a, stream)

    def repack(self, grid: Grid, u: torch.Tensor, n: int, faces: torch.Tensor, stream):
        """After the halo-region injection of row n: copy the injected face cells into `faces`."""
        if self.face_idx is None or n >= self.nsteps:
            return
        _abi.rtm_pack_cells(grid.c, u, self.face_idx, self.face_idx.numel(), faces, stream)


def tune_grid(grid: Grid, reps: int = 3):
    """Pick the fastest tile shape and workgroup order of the one-launch call for grids of this
    grid's shape on the current device (rtm_tune_step on scratch fields; the results of every call
    stay the same).  Waits for the device; returns the choice."""
    st = torch.cuda.current_stream()
    u_nxt, u_cur, u_prv, kap = grid.field(), grid.field(), grid.field(), grid.field(0.05)
    choice = _abi.rtm_tune_step(grid.c, u_nxt, u_cur, u_prv, kap, reps, st)
    st.synchronize()
    return choice


class Propagator:
    def __init__(self, grid: Grid, kappa: torch.Tensor, *, sources: Sources | list | None = None,
                 receivers=None, boundary: str = "zero", schedule: str = "overlap", debug: bool = False,
                 check_every: int = 0, unpack_aside: bool = False, ghosts: str = "ring", halo: str = "region"):
        """ghosts: "ring" (default) keeps every level's ghost ring current with an unpack pass after
        each step; "slots" (serial and overlap schedules, radius 4, nx % 4 == 0) leaves the ghosts of
        each level in the receive slots, where the next halo call reads them (rtm_step_halo_pack_slots),
        so a step has no unpack pass and the level buffers' rings are not kept (fill_ghosts() writes
        the newest level's).

        halo (ghosts="slots"): "region" (default) updates the halo region in the halo call and the
        rest in the interior call; "shell" computes only the faces in the halo call
        (rtm_step_shell_pack) and every owned cell in the second call (rtm_step_whole_slots).  The
        shell call reads kappa's faces from a copy packed here: after changing kappa in place, call
        refresh_kappa().

        unpack_aside (serial schedule): the unpack runs on a second stream as soon as the halo call
        and the shell sources are done, concurrently with the interior call (it writes ghost cells
        only, the interior call owned cells only); the next step waits for it.  Same bits.

        check_every = K > 0: health check of the production path.  After every K-th step the
        newest level's non-finite owned cells are counted on the device (rtm_count_nonfinite, 4 bytes
        per cell) and the host reads the count (one synchronisation per K steps); a run that went
        unstable (e.g. a time step past the stability limit) raises FloatingPointError within K
        steps of its first non-finite level.

        debug: NaN-poison mode.  Buffers taken fresh for a new time level (when a pinned level
        blocks the in-place rotation) start as NaN, ghost ring included, and after every step the
        owned cells of the new level must be finite; a kernel that read a cell nobody wrote (an unset
        ghost, an edge or corner of the ring, a stale buffer) would carry NaN into them.  The check
        synchronises every step, so it is for testing, not for timing."""
        self.grid = grid
        self.kappa = kappa
        if sources is None:
            sources = []
        self.sources = sources if isinstance(sources, list) else [sources]
        self.rec_idx = None
        if receivers is not None and len(np.asarray(receivers).reshape(-1, 3)):
            self.rec_idx = torch.from_numpy(grid.index(receivers)).to(grid.device)
        self.nrec = 0 if self.rec_idx is None else self.rec_idx.numel()
        if boundary not in ("zero", "zero_faces", "periodic"):
            raise ValueError(boundary)
        self.boundary = boundary
        if schedule not in ("overlap", "serial", "fused"):
            raise ValueError(schedule)
        self.schedule = schedule
        self.u_prv = grid.field()
        self.u_cur = grid.field()
        # level buffers whose ghost ring is known to hold zeros (the physical boundary's ghosts), by
        # buffer identity: the fused schedule skips the ghost refresh for them when no face is received
        self._zero_ghosts: dict[int, weakref.ref] = {}
        self._mark_zero_ghosts(self.u_prv)
        self._mark_zero_ghosts(self.u_cur)
        self.pinned: set[int] = set()
        self.pool: list[torch.Tensor] = []
        if ghosts not in ("ring", "slots"):
            raise ValueError(ghosts)
        if halo not in ("region", "shell"):
            raise ValueError(halo)
        if halo == "shell" and ghosts != "slots":
            raise ValueError("halo='shell' reads the ghosts from the receive slots (ghosts='slots')")
        self.ghosts = ghosts
        self.halo = halo
        if ghosts == "slots":
            if schedule == "fused" or unpack_aside:
                raise ValueError("ghosts='slots' is for the serial and overlap schedules (no unpack pass)")
            if grid.radius != 4 or grid.nx % 4:
                raise ValueError("ghosts='slots' needs radius 4 and nx % 4 == 0")
        self.send = grid.faces()
        # ghosts="slots": step n packs into send_bufs[n % len(send_bufs)]: two buffers, three with
        # halo="shell" (whose shell call reads the faces of u^n and u^{n-1} from the last two)
        nbuf = 1 if ghosts != "slots" else (3 if halo == "shell" else 2)
        self.send_bufs = [self.send] + [grid.faces() for _ in range(nbuf - 1)]
        self.kappa_faces = None
        if halo == "shell":
            self.kappa_faces = grid.faces()
            _abi.rtm_pack_halo(grid.c, kappa, self.kappa_faces, torch.cuda.current_stream())
        slots = grid.face_slots(self.send)
        # what face f of each new level receives: NULL slots for the physical boundary (the unpack
        # writes zero ghosts and reads nothing); "zero_faces": the same zeros received through six
        # real slots of a zero-filled receive buffer, as a subdomain whose neighbours all sent zero
        # faces (the unpack reads them); "periodic": the opposite face's send slot (a pointer swap)
        self.recv_buf = None
        if boundary == "zero" and ghosts == "slots":
            self.recv_buf = grid.faces()        # the physical boundary's zeros, read by the halo call
            self.recv = grid.face_slots(self.recv_buf)
        elif boundary == "zero":
            self.recv = [None] * 6
        elif boundary == "zero_faces":
            self.recv_buf = grid.faces()
            self.recv = grid.face_slots(self.recv_buf)
        else:
            self.recv = [slots[OPPOSITE[f]] for f in range(6)]
        # ghosts="slots", periodic: the receive slots of a level made by a step that packed into
        # send_bufs[b] (a pointer swap, as above), for level m in buffer (m - 1) % len(send_bufs)
        self._recv_periodic = [[self.grid.face_slots(b)[OPPOSITE[f]].data_ptr() for f in range(6)]
                               for b in self.send_bufs]
        self.n = 0
        self.sH = torch.cuda.Stream(device=grid.device)
        self.sI = torch.cuda.Stream(device=grid.device)
        self._ev_int = None
        # list of (start, end) timing events around the dominant call (rtm_step_interior; with
        # halo="shell", rtm_step_whole_slots), or None
        self.interior_events = None
        # time the interior call on every k-th step only: an event pair costs the step it brackets
        # about 11 us at 512^3 (each event waits for the kernel before it and writes back the caches)
        self.interior_event_every = 1
        self.interior_event_start = 0       # timed steps: n - start a multiple of interior_event_every
        self.debug = bool(debug)
        if check_every < 0:
            raise ValueError("check_every must be >= 0")
        self.check_every = int(check_every)
        self.unpack_aside = bool(unpack_aside)
        self._ev_unpack = None
        self._bad = torch.zeros(1, dtype=torch.int32, device=grid.device) if self.check_every else None

    # ------------------------------------------------------------------------------------------
    def set_state(self, u_cur_host=None, u_prv_host=None, n: int = 0):
        """Load (u^n, u^{n-1}) from host arrays (None = zero) and fill the ghosts of u^n."""
        g = self.grid
        self.u_cur.zero_()
        self.u_prv.zero_()
        if u_cur_host is not None:
            g.upload(u_cur_host, self.u_cur)
        if u_prv_host is not None:
            g.upload(u_prv_host, self.u_prv)
        self.n = n
        self.exchange_ghosts(self.u_cur)

    def exchange_ghosts(self, u: torch.Tensor, stream=None):
        """Pack, exchange and unpack the faces of an existing level (used to prime u^0).  With
        ghosts="slots", u must be the newest level: its faces are packed where the next step's halo
        call reads them, and its ghost ring is written from there too."""
        st = stream if stream is not None else torch.cuda.current_stream()
        if self.ghosts == "slots":
            nb = len(self.send_bufs)
            _abi.rtm_pack_halo(self.grid.c, u, self.send_bufs[(self.n - 1) % nb], st)
            if self.halo == "shell":        # the shell call reads u^{n-1}'s faces too
                _abi.rtm_pack_halo(self.grid.c, self.u_prv, self.send_bufs[(self.n - 2) % nb], st)
            _abi.rtm_unpack_halo(self.grid.c, u, self._recv_for(self.n), st)
            return
        _abi.rtm_pack_halo(self.grid.c, u, self.send, st)
        _abi.rtm_unpack_halo(self.grid.c, u, self.recv, st)
        if all(r is None for r in self.recv):
            self._mark_zero_ghosts(u)

    def _recv_for(self, m: int):
        """ghosts="slots": the six receive slots that hold level m's ghost faces (the faces packed by
        the step that made level m, or by exchange_ghosts)."""
        if self.boundary != "periodic":
            return self.recv
        return self._recv_periodic[(m - 1) % len(self.send_bufs)]

    def fill_ghosts(self, stream=None):
        """Write the newest level's ghost ring (kept in the receive slots with ghosts="slots", for code
        that reads the ring: rtm_step_whole, the adjoint and gradient calls); a no-op otherwise."""
        if self.ghosts != "slots":
            return
        self.sync()
        st = stream if stream is not None else torch.cuda.current_stream()
        _abi.rtm_unpack_halo(self.grid.c, self.u_cur, self._recv_for(self.n), st)

    def refresh_kappa(self):
        """halo="shell": re-pack kappa's faces after kappa was changed in place (the shell call reads
        the x strips' kappa from that copy); a no-op otherwise."""
        if self.kappa_faces is not None:
            self.sync()
            _abi.rtm_pack_halo(self.grid.c, self.kappa, self.kappa_faces, torch.cuda.current_stream())

    def _mark_zero_ghosts(self, u: torch.Tensor):
        self._zero_ghosts[u.data_ptr()] = weakref.ref(u)

    def _ghosts_known_zero(self, u: torch.Tensor) -> bool:
        r = self._zero_ghosts.get(u.data_ptr())
        return r is not None and r() is u

    def pin_current(self):
        """Keep the buffer of the newest level: later steps will not write into it."""
        self.pinned.add(self.u_cur.data_ptr())
        return self.u_cur

    def pin_previous(self):
        """Keep the buffer of the level before the newest one."""
        self.pinned.add(self.u_prv.data_ptr())
        return self.u_prv

    def set_levels(self, u_cur: torch.Tensor, u_prv: torch.Tensor, n: int):
        """Continue from existing device levels (u^n, u^{n-1}) without copying them; u_prv may be
        overwritten by the next step unless it is pinned.  u_cur's ghosts must be current."""
        self.sync()
        self._zero_ghosts.pop(u_prv.data_ptr(), None)     # its ghosts are the caller's: refreshed on reuse
        self.u_cur, self.u_prv, self.n = u_cur, u_prv, n
        nb, st = len(self.send_bufs), torch.cuda.current_stream()
        if self.ghosts == "slots" and (self.boundary == "periodic" or self.halo == "shell"):
            # the next halo call reads u^n's ghosts from the slots (periodic: the faces they are copies
            # of) and, with halo="shell", the faces of u^n and u^{n-1}
            _abi.rtm_pack_halo(self.grid.c, u_cur, self.send_bufs[(n - 1) % nb], st)
        if self.halo == "shell":
            _abi.rtm_pack_halo(self.grid.c, u_prv, self.send_bufs[(n - 2) % nb], st)

    def unpin(self, t: torch.Tensor, recycle: bool = True):
        self.pinned.discard(t.data_ptr())
        # the caller may have written anything into it meanwhile: its ghosts are refreshed on reuse
        self._zero_ghosts.pop(t.data_ptr(), None)
        if recycle:
            self.pool.append(t)

    def _next_buffer(self) -> torch.Tensor:
        if self.u_prv.data_ptr() not in self.pinned:
            return self.u_prv                       # in-place over u^{n-1}
        buf = self.pool.pop() if self.pool else self.grid.field(fill=None)
        if self.debug:
            # after everything queued so far (a recycled buffer may still be read), on the current
            # stream, which both step streams then wait for
            self.sync()
            buf.fill_(float("nan"))
        return buf

    def _check_finite(self, u: torch.Tensor):
        self.sync()
        if not bool(torch.isfinite(self.grid.owned(u)).all()):
            raise RuntimeError(f"NaN-poison check: level {self.n} has non-finite owned cells")

    # ------------------------------------------------------------------------------------------
    def step(self, traces: torch.Tensor | None = None):
        """Advance one step; record into row n of `traces` (device, shape (nsteps, nrec)) if given."""
        g, c = self.grid, self.grid.c
        u_nxt = self._next_buffer()
        u_cur, u_prv, kap = self.u_cur, self.u_prv, self.kappa
        n = self.n
        slots = self.ghosts == "slots"
        shell = self.halo == "shell"
        dense = None
        if slots:
            nb = len(self.send_bufs)
            self.send = self.send_bufs[n % nb]
            # halo="shell": the face buffers of u^n and u^{n-1}, and kappa's
            dense = (self.send_bufs[(n - 1) % nb], self.send_bufs[(n - 2) % nb], self.kappa_faces) if shell else None
        tr_ptr = None if traces is None or self.nrec == 0 else traces.data_ptr() + 4 * n * self.nrec
        if self.schedule == "fused":
            st = torch.cuda.current_stream()
            _abi.rtm_step_whole(c, u_nxt, u_cur, u_prv, kap, st)
            for s in self.sources:
                s.inject(g, u_nxt, n, 2, st)
            if any(r is not None for r in self.recv):
                _abi.rtm_pack_halo(c, u_nxt, self.send, st)
                _abi.rtm_unpack_halo(c, u_nxt, self.recv, st)
            elif not self._ghosts_known_zero(u_nxt):
                # no face is received: the ghosts are the boundary's zeros, written once per buffer
                # (the updates write owned cells only)
                _abi.rtm_unpack_halo(c, u_nxt, self.recv, st)
                self._mark_zero_ghosts(u_nxt)
            if tr_ptr is not None:
                _abi.rtm_record(c, u_nxt, self.rec_idx, tr_ptr, self.nrec, st)
        elif self.schedule == "serial" and shell:
            for s in self.sources:
                s.ensure_split(g)
            st = torch.cuda.current_stream()
            self._shell_step(u_nxt, u_cur, u_prv, n, dense, tr_ptr, st, st)
        elif self.schedule == "serial":
            for s in self.sources:
                s.ensure_split(g)
            # one stream, in the paper's phase order: the halo call that also writes the faces, the
            # shell sources (re-copied into the faces they sit in), the interior call, the interior
            # sources, the unpack (at 512^3: 0.525 ms per step against 0.546 ms with the pack after
            # the interior call, once each row's owned cells start a cache line)
            st = torch.cuda.current_stream()
            if self._ev_unpack is not None:
                st.wait_event(self._ev_unpack)          # the ghosts of u^n are complete
                self._ev_unpack = None
            if slots:
                _abi.rtm_step_halo_pack_slots(c, u_nxt, u_cur, u_prv, kap, self._recv_for(n), self.send, st)
            else:
                _abi.rtm_step_halo_pack(c, u_nxt, u_cur, u_prv, kap, self.send, st)
            for s in self.sources:
                s.inject(g, u_nxt, n, 0, st)
                s.repack(g, u_nxt, n, self.send, st)
            if self.unpack_aside:
                ev = torch.cuda.Event()
                ev.record(st)
                self.sH.wait_event(ev)
                _abi.rtm_unpack_halo(c, u_nxt, self.recv, self.sH)
                self._ev_unpack = torch.cuda.Event()
                self._ev_unpack.record(self.sH)
            self._interior(u_nxt, u_cur, u_prv, n, st)
            if slots:
                self._inject_and_record(u_nxt, n, 1, tr_ptr, st)
            else:
                for s in self.sources:
                    s.inject(g, u_nxt, n, 1, st)
                if not self.unpack_aside:
                    _abi.rtm_unpack_halo(c, u_nxt, self.recv, st)
                if tr_ptr is not None:
                    _abi.rtm_record(c, u_nxt, self.rec_idx, tr_ptr, self.nrec, st)
        else:
            for s in self.sources:
                s.ensure_split(g)
            sH, sI = self.sH, self.sI
            if self._ev_int is not None:
                sH.wait_event(self._ev_int)
            else:
                sH.wait_stream(torch.cuda.current_stream())
                sI.wait_stream(torch.cuda.current_stream())
            if shell:
                self._shell_step(u_nxt, u_cur, u_prv, n, dense, tr_ptr, sH, sI)
            else:
                if slots:
                    _abi.rtm_step_halo_pack_slots(c, u_nxt, u_cur, u_prv, kap, self._recv_for(n), self.send, sH)
                else:
                    _abi.rtm_step_halo_pack(c, u_nxt, u_cur, u_prv, kap, self.send, sH)
                for s in self.sources:
                    s.inject(g, u_nxt, n, 0, sH)
                    s.repack(g, u_nxt, n, self.send, sH)
                ev_halo = torch.cuda.Event()
                ev_halo.record(sH)
                if not slots:
                    _abi.rtm_unpack_halo(c, u_nxt, self.recv, sH)
                self._interior(u_nxt, u_cur, u_prv, n, sI)
                for s in self.sources:
                    s.inject(g, u_nxt, n, 1, sI)
                sI.wait_event(ev_halo)
                if tr_ptr is not None:
                    _abi.rtm_record(c, u_nxt, self.rec_idx, tr_ptr, self.nrec, sI)
            ev_int = torch.cuda.Event()
            ev_int.record(sI)
            self._ev_int = ev_int
        self.u_prv, self.u_cur = self.u_cur, u_nxt
        self.n = n + 1
        if self.debug:
            self._check_finite(u_nxt)
        if self.check_every and self.n % self.check_every == 0:
            self._health_check(u_nxt)

    def _interior(self, u_nxt, u_cur, u_prv, n, st):
        """The interior call, bracketed by timing events on every interior_event_every-th step when
        interior_events is a list."""
        c = self.grid.c
        if self.interior_events is not None and \
                (n - self.interior_event_start) % self.interior_event_every == 0:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            _abi.rtm_step_interior(c, u_nxt, u_cur, u_prv, self.kappa, st)
            e1.record(st)
            self.interior_events.append((e0, e1))
        else:
            _abi.rtm_step_interior(c, u_nxt, u_cur, u_prv, self.kappa, st)

    def _shell_step(self, u_nxt, u_cur, u_prv, n, dense, tr_ptr, sH, sI):
        """halo="shell": the shell call on sH (faces of u^{n+1} into the send buffer), then on sI,
        once it is done (u_nxt may be u_prv, which the shell call reads), the call over every owned
        cell (timed like the interior call), the sources, the re-copy of those in face cells into the
        send buffer, and the record.  The exchange of a multi-GPU run would start on sH after the
        shell call, and wait for the re-copy when a source sits in a face cell."""
        g, c, kap = self.grid, self.grid.c, self.kappa
        recv = self._recv_for(n)
        _abi.rtm_step_shell_pack(c, u_cur, u_prv, kap, recv, self.send, sH, dense=dense)
        if sI is not sH:
            ev = torch.cuda.Event()
            ev.record(sH)
            sI.wait_event(ev)
        if self.interior_events is not None and \
                (n - self.interior_event_start) % self.interior_event_every == 0:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(sI)
            _abi.rtm_step_whole_slots(c, u_nxt, u_cur, u_prv, kap, recv, sI)
            e1.record(sI)
            self.interior_events.append((e0, e1))
        else:
            _abi.rtm_step_whole_slots(c, u_nxt, u_cur, u_prv, kap, recv, sI)
        self._inject_and_record(u_nxt, n, 2, tr_ptr, sI)

    def _inject_and_record(self, u_nxt, n, which, tr_ptr, st):
        """Sources of set `which`, their face cells re-copied into the send buffer, then the record; one
        launch for both when a single source table has no face cell (rtm_inject_record)."""
        g, c = self.grid, self.grid.c
        if len(self.sources) == 1 and self.sources[0].face_idx is None:
            a = self.sources[0].inject_args(n, which)
            if a is not None or tr_ptr is not None:
                a = a if a is not None else (None, None, None, 0)
                _abi.rtm_inject_record(c, u_nxt, *a, self.rec_idx, tr_ptr, self.nrec if tr_ptr is not None else 0, st)
            return
        for s in self.sources:
            s.inject(g, u_nxt, n, which, st)
            if which != 1:
                s.repack(g, u_nxt, n, self.send, st)
        if tr_ptr is not None:
            _abi.rtm_record(c, u_nxt, self.rec_idx, tr_ptr, self.nrec, st)

    def _health_check(self, u: torch.Tensor):
        st = self.level_stream
        with torch.cuda.stream(st):
            self._bad.zero_()
        _abi.rtm_count_nonfinite(self.grid.c, u, self._bad, st)
        st.synchronize()
        bad = int(self._bad.item())
        if bad:
            raise FloatingPointError(f"level {self.n}: {bad} owned cells are not finite (unstable run?)")

    @property
    def level_stream(self):
        """Stream on which the newest level is complete (for work that reads it)."""
        return self.sI if self.schedule == "overlap" else torch.cuda.current_stream()

    def sync(self):
        """Make the caller's current stream wait for everything enqueued so far."""
        if self._ev_unpack is not None:
            torch.cuda.current_stream().wait_event(self._ev_unpack)
            self._ev_unpack = None
        if self.schedule == "overlap":
            cur = torch.cuda.current_stream()
            cur.wait_stream(self.sH)
            cur.wait_stream(self.sI)
            self._ev_int = None

    def run(self, nsteps: int, traces: torch.Tensor | None = None, on_level=None):
        """Run nsteps steps.  on_level(k, prop) is called after the step that produced level k, with
        prop.level_stream ready for work that reads u^k (prop.u_cur)."""
        for _ in range(nsteps):
            self.step(traces)
            if on_level is not None:
                on_level(self.n, self)
        self.sync()
        return traces

    def new_traces(self, nsteps: int) -> torch.Tensor:
        return torch.zeros((nsteps, max(self.nrec, 1)), dtype=torch.float32, device=self.grid.device)
