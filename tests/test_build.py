"""The build's scratch-memory check (host logic, no GPU)."""

import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build_module():
    spec = importlib.util.spec_from_file_location("xl_build", os.path.join(ROOT, "paper_2303_00689_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_scratch_report_parsing():
    b = _build_module()
    report = "\n".join([
        "a.hip:1:1: remark: Function Name: k_one [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     VGPRs: 40 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark: Function Name: k_two [-Rpass-analysis=kernel-resource-usage]",
        "a.hip:9:1: remark:     ScratchSize [bytes/lane]: 8720 [-Rpass-analysis=kernel-resource-usage]",
    ])
    assert b.scratch_kernels(report) == [("k_two", 8720)]
    assert b.scratch_kernels("") == []


def test_build_asks_for_the_resource_report():
    b = _build_module()
    assert "-Rpass-analysis=kernel-resource-usage" in b.FLAGS
