"""Shared set-up for the GPU parity tests: a library context and, per array, the
GPU geometry/operator next to the oracle's independent discretisation."""
from __future__ import annotations

import numpy as np

import workloads as W
from oracle import discretise, greens, grouping

_CTX = None
_CACHE = {}


def ctx():
    global _CTX
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    if _CTX is None:
        import paper_2603_10586_amd as q
        _CTX = q.Context(0)
    return _CTX


ARRAYS = {
    "tiny": lambda: W.tiny(),
    "rand5x3": lambda: W.random_lattice(5, 3, seed=11),
    "rand8x8": lambda: W.random_lattice(8, 8, seed=2),
    "rand6x7": lambda: W.random_lattice(6, 7, seed=5),
    "rand16x16": lambda: W.random_lattice(16, 16, seed=7),
    # a 33 x 33 request of the seeded serving stream: a ragged quadtree whose edge nodes hold
    # one particle, so it has tall far blocks of one particle's columns (2304 x 144)
    "serving33": lambda: W.serving_requests(n=8, seed=0, rate_per_s=1.0, side_lo=8, side_hi=48)[7].array,
}


class Case:
    def __init__(self, name: str, eps: float = 1e-6, max_block_rows: int = 0, far_prec: int = 0,
                 compression: str = "aca"):
        import paper_2603_10586_amd as q
        print(f"[gpu case] building {name} eps={eps} cap={max_block_rows} far_prec={far_prec} {compression}",
              flush=True)
        self.name = name
        self.eps = eps
        self.array = ARRAYS[name]()
        self.disc = discretise.Discretisation(self.array)
        self.ctx = ctx()
        self.geom = q.Geometry(self.ctx, self.array)
        self.op = q.Operator(self.ctx, self.geom, eps=eps, max_block_rows=max_block_rows, far_prec=far_prec,
                             compression=compression)
        self.order = self.geom.order()
        self._Z = None
        self._factors = None

    @property
    def Z(self):
        if self._Z is None:
            self._Z = greens.assemble_dense(self.disc)
        return self._Z

    def factors(self):
        """Exported GPU factors as (caller rows, caller cols, Q, R, info)."""
        if self._factors is None:
            out = []
            for b in range(self.op.num_blocks()):
                info, Q, R = self.op.export_block(b)
                rows = self.order[info["row_first"]:info["row_first"] + info["row_count"]]
                cols = self.order[info["col_first"]:info["col_first"] + info["col_count"]]
                if Q is None:
                    Q = np.zeros((info["m"], 0), complex)
                    R = np.zeros((0, info["n"]), complex)
                out.append((rows, cols, Q, R, info))
            self._factors = out
        return self._factors

    def oracle_blocks(self):
        return grouping.build_blocks(self.array.lattice_ij, self.array.nx, self.array.ny)


def case(name: str, eps: float = 1e-6, max_block_rows: int = 0, far_prec: int = 0, compression: str = "aca") -> Case:
    key = (name, eps, max_block_rows, far_prec, compression)
    if key not in _CACHE:
        _CACHE[key] = Case(name, eps, max_block_rows, far_prec, compression)
    return _CACHE[key]


def to_dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


_MID = {}


def mid(compression: str = "aca"):
    """The mid-size workload (32 x 32 disks, 147,456 unknowns, eps = 1e-6) on the GPU, with the
    oracle's discretisation, the internal order and every block's export record; one operator
    per compression, on one geometry."""
    import paper_2603_10586_amd as q
    if not _MID:
        print("[gpu case] mid 32x32 geometry", flush=True)
        arr = W.mid(0)
        geom = q.Geometry(ctx(), arr)
        _MID[None] = dict(arr=arr, disc=discretise.Discretisation(arr), geom=geom, order=geom.order())
        _MID[None]["internal"] = np.argsort(_MID[None]["order"])
    if compression not in _MID:
        print(f"[gpu case] building mid 32x32 eps=1e-6 {compression}", flush=True)
        base = _MID[None]
        op = q.Operator(ctx(), base["geom"], eps=1e-6, compression=compression)
        infos = [op.export_block(b, factors=False)[0] for b in range(op.num_blocks())]
        _MID[compression] = dict(base, op=op, infos=infos)
    return _MID[compression]


def block_particles(order, info):
    """Caller particle lists (rows, cols) of an exported block, in the block's DoF order."""
    rows = order[info["row_first"]:info["row_first"] + info["row_count"]]
    cols = order[info["col_first"]:info["col_first"] + info["col_count"]]
    return rows, cols
