"""The FP64 oracle projector pair run over a pool of worker processes, one
slice of the views per worker.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``).  Alg. 1 and Alg. 2
treat every view on its own and the back projection sums the views'
contributions, so splitting the views between processes changes nothing but
the order of that final sum: each worker runs ``projector.forward`` or
``projector.back`` on its own views, unchanged, and the parent adds the
workers' volumes in worker order (a fixed order, so results do not depend
on scheduling).

Workers are started with the "spawn" method: they are fresh interpreters
that never touch a GPU, whatever the parent process has initialised.  Each
worker receives mu, the PSFs and the geometry once, at start-up.
"""
from __future__ import annotations

import concurrent.futures as cf
import multiprocessing as mp
import os

import numpy as np

from . import convolution, projector

_W = {}


def _init(mu, psf, geom):
    _W["mu"], _W["psf"], _W["geom"] = mu, psf, geom
    convolution.FFT_WORKERS = 1


def _fwd(args):
    x, views, conv = args
    v = projector.forward(x, _W["mu"], _W["psf"], _W["geom"], views=views, conv=conv)
    return views, v[views]


def _back(args):
    v, views, conv = args
    return projector.back(v, _W["mu"], _W["psf"], _W["geom"], views=views, conv=conv)


def host_cores(cap=16):
    """Cores this process may run on, at most ``cap``."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, cap))


class OraclePool:
    """forward(x) / back(v) of the FP64 oracle over ``workers`` processes.

    x, mu: [nz][ny][nx]; psf: [nview][ny][pz][px]; v: [nview][nz][nx].
    ``conv`` is "direct" (the defining sum) or "fft" (its FFT form)."""

    def __init__(self, mu, psf, geom, workers=None, conv="fft"):
        self.geom = geom
        self.conv = conv
        self.workers = host_cores() if workers is None else max(1, int(workers))
        self.workers = min(self.workers, geom.nview)
        n = geom.nview
        self.slices = [list(range(n * w // self.workers, n * (w + 1) // self.workers))
                       for w in range(self.workers)]
        # a worker that dies raises BrokenProcessPool here instead of hanging
        self._pool = cf.ProcessPoolExecutor(self.workers, mp_context=mp.get_context("spawn"),
                                            initializer=_init,
                                            initargs=(np.asarray(mu), np.asarray(psf), geom))

    def forward(self, x):
        x = np.asarray(x, dtype=np.float64)
        g = self.geom
        out = np.zeros((g.nview, g.nz, g.nx))
        for views, rows in self._pool.map(_fwd, [(x, s, self.conv) for s in self.slices]):
            out[views] = rows
        return out

    def back(self, v):
        v = np.asarray(v, dtype=np.float64)
        parts = list(self._pool.map(_back, [(v, s, self.conv) for s in self.slices]))
        out = parts[0]
        for p in parts[1:]:
            out = out + p
        return out

    def close(self):
        if self._pool is not None:
            self._pool.shutdown(wait=True)
            self._pool = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
