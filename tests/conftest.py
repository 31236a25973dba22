import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import oracle as O

    O.lib()
    return O


def generate_on_device(make, *args, **kw):
    """Runs a device-side graph generator for a module fixture.  If it raises,
    the exception's traceback (whose frames hold the generator's tensors, tens
    of GB for the largest shapes) is dropped and the torch caching allocator
    emptied before a plain error is raised, so that a failed setup does not
    leave that memory held for the rest of the session and its teardown."""
    import gc

    try:
        return make(*args, **kw)
    except Exception as exc:  # noqa: BLE001 (re-raised without its frames)
        msg = f"{type(exc).__name__}: {exc}"
        exc.__traceback__ = None
        del exc
        gc.collect()
        try:
            import torch

            if torch.cuda.is_available():
                torch.cuda.synchronize()
                torch.cuda.empty_cache()
        except Exception:  # noqa: BLE001
            pass
        raise RuntimeError(f"device graph generation failed: {msg}") from None
