import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


# Map parameters of the workloads (Appendix-A readings: obstacle band 0.4-2.0 m,
# density threshold 1/2, 5x5 fit, 0.5 m negative threshold, 5 m search).
def params(nx, ny, nz, res, szv=None, **kw):
    p = dict(nx=nx, ny=ny, nz=nz, res_m=res, sensor_z_voxel=nz // 2 if szv is None else szv,
             obs_min_m=0.4, obs_max_m=2.0, dens_num=1, dens_den=2, fit_n=5,
             neg_thresh_m=0.5, neg_search_m=5.0)
    p.update(kw)
    return p


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    return oracle
