"""The grid barrier protocol of the persistent ensemble launch, modelled on
the CPU with threads and C++ atomics (tests/barrier_model.cpp; the device
code uses the same words and memory orders at agent scope): data written
before a barrier is seen by every participant after it, over many reuses of
the same words; and when one participant never arrives, every wait gives up
within its poll bound and reports through the status word instead of
hanging, and later barriers return at once.  The ordering check also runs
under ThreadSanitizer (host code), which reports the data slots as a race
unless the barrier's atomics order every write before it against every read
after it under the C++ memory model."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("barrier") / "barrier_model")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-pthread", os.path.join(HERE, "barrier_model.cpp"),
                           "-o", exe])
    return exe


def test_barrier_orders_writes_over_many_rounds(model):
    r = subprocess.run([model, "ok", "16", "2000"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr


def test_barrier_orders_writes_under_thread_sanitizer(tmp_path):
    exe = str(tmp_path / "barrier_model_tsan")
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-pthread", "-fsanitize=thread",
                           os.path.join(HERE, "barrier_model.cpp"), "-o", exe])
    r = subprocess.run([exe, "ok", "8", "200"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "ThreadSanitizer" not in r.stderr, r.stdout + r.stderr


def test_absent_participant_makes_every_wait_give_up(model):
    r = subprocess.run([model, "absent", "12", "200000"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "status=1" in r.stdout
