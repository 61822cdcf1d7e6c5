import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (MI355X) and the built library")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def synth_mod():
    import synth
    synth._load()
    return synth


@pytest.fixture(scope="session")
def lp():
    """The GPU library binding; fails loudly if it is not built or no device."""
    import paper_2410_19119_amd as m
    m._load()
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return m


@pytest.fixture(scope="session")
def rmat24(synth_mod):
    """The benchmark graph: R-MAT scale 24, edge factor 16, seed 1 (generated once per session)."""
    return synth_mod.rmat_scale(24, 16, seed=1)


@pytest.fixture(scope="session")
def progress(request):
    """Prints a line past pytest's output capture: the full-size tests report
    each finished step (generation, GPU run, oracle round) as it ends."""
    capman = request.config.pluginmanager.getplugin("capturemanager")

    def say(msg: str) -> None:
        if capman is None:
            print(f"[progress] {msg}", flush=True)
            return
        with capman.global_and_fixture_disabled():
            print(f"[progress] {msg}", flush=True)
    return say
