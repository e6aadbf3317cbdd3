import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def _describe_device_tensors():
    """Failure reports print the values in a failed assertion; printing a
    device tensor launches GPU work from inside the report.  Describe such
    tensors by shape, dtype and device instead."""
    try:
        import torch
    except ImportError:
        return
    orig = torch.Tensor.__repr__

    def safe_repr(self, *args, **kwargs):
        if self.device.type != "cpu":
            return f"<tensor shape={tuple(self.shape)} dtype={self.dtype} device={self.device}>"
        return orig(self, *args, **kwargs)

    torch.Tensor.__repr__ = safe_repr


_describe_device_tensors()
