"""The process entry points (condensation, breakup, sedimentation) captured
together in one graph and replayed: every replay must equal the same calls
made eagerly, bit for bit, with eager work and synchronisations between the
replays.  The calls launch kernels only (their counters are cleared by a
kernel, not a memset) once the first calls of a shape have allocated the
workspaces and uploaded the breakup shares, which happens before the
capture here."""

import numpy as np
import pytest

from paper_2409_07232_amd import workloads as wl

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def test_condense_breakup_sediment_graph_replays():
    from paper_2409_07232_amd import _lib as L
    w = wl.config2(nx=16, ny=16, nz=50)
    ssat, g = wl.condensation_inputs(w)
    rate, Q = wl.breakup_tables(w.nbins, w.s, w.x1_g)
    geo = wl.sediment_geometry(w)
    h = L.FsbmCoal.from_workload(w, precision=0)
    h.set_breakup(rate, Q)
    sd, gd = _dev(ssat), _dev(g)
    dz, v, vf = _dev(geo["dz_cm"]), _dev(geo["v_cm_s"]), _dev(geo["vfac"])
    dt, n = 2.0, 4

    def calls(N, ev, pr, stream):
        h.condense(N, sd, gd, dt, n, ev, stream=stream)
        h.breakup(N, dt, n, stream=stream)
        h.sediment(N, geo["ncols"], geo["nlev"], geo["col_stride"],
                   geo["lev_stride"], dz, v, vf, dt, n, pr, stream=stream)

    def buffers():
        return (_dev(w.N), torch.zeros(w.npoints, dtype=torch.float64,
                                       device="cuda"),
                torch.zeros((geo["ncols"], 1, w.nbins), dtype=torch.float64,
                            device="cuda"))

    # eager copy; its first call also allocates and uploads
    Ne, ee, pe = buffers()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        calls(Ne, ee, pe, side)
    torch.cuda.synchronize()
    Ng, eg, pg = buffers()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        calls(Ng, eg, pg, torch.cuda.current_stream())
    torch.cuda.synchronize()
    try:
        for rep in range(3):
            graph.replay()
            torch.cuda.synchronize()
            if rep:
                calls(Ne, ee, pe, torch.cuda.current_stream())
                torch.cuda.synchronize()
            # eager work of the program between replays
            junk = torch.randn(1 << 16, device="cuda").cumsum(0)
            torch.cuda.synchronize()
            assert torch.isfinite(junk).all()
            assert torch.equal(Ng, Ne), rep
            assert torch.equal(eg, ee), rep
            assert torch.equal(pg, pe), rep
    finally:
        h.close()
