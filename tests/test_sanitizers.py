"""The C ABI's host code under AddressSanitizer + UndefinedBehaviorSanitizer
and under ThreadSanitizer, on the CPU.

`paper_1702_00817_amd/build.py --sanitize {address,thread}` builds the
library's sources (host pass instrumented, device code untouched) with
tests/sanitize/fake_device_driver.cpp into one executable. The driver runs
the fake-device server from several threads at once (submit, wait, poll,
release, statistics), injected failures at completion and partway through a
launch, admission under a tight budget, replay and shutdown with work in
flight, the resident queue protocol with relaunches, failed creation, and
the argument checks of the plain and batch calls. A sanitizer report fails
the run (halt_on_error) as does any failed check."""
import importlib.util
import os
import subprocess

import pytest

from conftest import ROOT


def _build_module():
    spec = importlib.util.spec_from_file_location(
        "tdct_build", os.path.join(ROOT, "paper_1702_00817_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


# a 4 EiB arena is the failed-creation case: the sanitizer's allocator must
# return null for it as the plain one does
OPTIONS = {
    "address": {"ASAN_OPTIONS": "allocator_may_return_null=1:halt_on_error=1:detect_leaks=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"},
    "thread": {"TSAN_OPTIONS": "allocator_may_return_null=1:halt_on_error=1:second_deadlock_stack=1"},
}


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_fake_device_driver_is_clean_under_sanitizer(kind, tmp_path):
    exe = _build_module().build_sanitized(kind)
    env = dict(os.environ)
    env.update(OPTIONS[kind])
    r = subprocess.run([exe], cwd=str(tmp_path), env=env, stdin=subprocess.DEVNULL,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300)
    out = r.stdout
    assert r.returncode == 0, out[-4000:]
    assert "fake-device driver: ok (0 failed checks)" in out, out[-4000:]
    for marker in ("ERROR: AddressSanitizer", "WARNING: ThreadSanitizer", "runtime error:",
                   "ERROR: LeakSanitizer"):
        assert marker not in out, out[-4000:]
