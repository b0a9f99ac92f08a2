"""Small acquisition geometries used across the test-suite."""
import numpy as np

import oracle
import tt_inputs as synth


def tilted_angles(n_rot, tilts_deg, span_deg=180.0, phase_deg=7.0):
    rot = phase_deg + np.arange(n_rot) * span_deg / n_rot
    inner = np.deg2rad(np.tile(rot, len(tilts_deg)))
    outer = np.deg2rad(np.repeat(np.asarray(tilts_deg, float), n_rot))
    return inner, outer


def tiny(ell_max=2, n=(6, 7, 8), nj=9, nk=10, n_seg=8, step=1.0, offsets=False):
    inner, outer = tilted_angles(3, (0.0, 33.0))
    kw = {}
    if offsets:
        kw = dict(joff=np.linspace(-0.4, 0.3, len(inner)), koff=np.linspace(0.25, -0.35, len(inner)))
    return oracle.Geometry(n, ell_max, inner, outer, nj, nk, n_seg, synth.lab_frame(), step=step, **kw)


def small(ell_max=4, n=(20, 24, 17), nj=23, nk=29, n_seg=8, n_rot=4, tilts=(0.0, 20.0, 45.0)):
    inner, outer = tilted_angles(n_rot, tilts, span_deg=360.0)
    return oracle.Geometry(n, ell_max, inner, outer, nj, nk, n_seg, synth.lab_frame())


def workload(name, **kw):
    return oracle.Geometry.from_workload(synth.WORKLOADS[name], **kw)


def steep(ell_max=4, n=(12, 10, 9), nj=13, nk=11, n_seg=8, model="trilinear"):
    """Tilts of 60-90 degrees: rays with |d_x|, |d_y| < 1/4 (gathered straight from
    global memory by the forward march) beside slab-staged ones, and at 90 degrees
    rays parallel to two voxel faces."""
    inner, outer = tilted_angles(3, (60.0, 72.0, 80.0, 90.0), span_deg=360.0)
    return oracle.Geometry(n, ell_max, inner, outer, nj, nk, n_seg, synth.lab_frame(), model=model)


def degenerate(model="trilinear"):
    """A volume one voxel thick along x, a single detector row and two segments."""
    inner, outer = tilted_angles(3, (0.0, 40.0), span_deg=180.0)
    return oracle.Geometry((1, 5, 4), 2, inner, outer, 1, 7, 2, synth.lab_frame(), model=model)
