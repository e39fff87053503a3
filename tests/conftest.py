import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (MI355X) and the built libadc.so")


@pytest.fixture(scope="session")
def ctx():
    import torch
    from paper_1510_04591_amd import adc
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    c = adc.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def cuda(x):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")
