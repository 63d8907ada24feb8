"""Host-side checks of the measurement tooling: the kernel-source hash that
keeps counter-based traffic figures tied to the code they were taken on, and
the kernel-name parsing of the rocprofv3 summaries (CPU only)."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import rocprof_summary  # noqa: E402


def _hash_of(tmp_path, src_text, kernel):
    d = tmp_path / "repo"
    (d / os.path.dirname(bench.KERNEL_SRC)).mkdir(parents=True, exist_ok=True)
    (d / bench.KERNEL_SRC).write_text(src_text)
    old = bench.ROOT
    try:
        bench.ROOT = str(d)
        return bench.kernel_hash(kernel)
    finally:
        bench.ROOT = old


def _src():
    with open(os.path.join(ROOT, bench.KERNEL_SRC)) as f:
        return f.read()


def test_kernel_hash_tracks_only_its_kernel(tmp_path):
    """Comments and other kernels' bodies leave a kernel's hash unchanged; a
    change to its own body changes it."""
    src = _src()
    h0 = _hash_of(tmp_path, src, "k_forward_p")
    assert h0 == bench.kernel_hash("k_forward_p")
    # a comment line inside the kernel and an edit of another kernel
    key = "void k_forward_p("
    i = src.index(key)
    body = src.index("{", i) + 1
    commented = src[:body] + "\n    // a remark\n" + src[body:]
    assert _hash_of(tmp_path, commented, "k_forward_p") == h0
    j = src.index("void k_adjoint_h16s(")
    jb = src.index("{", j) + 1
    other = src[:jb] + "\n    (void)0;\n" + src[jb:]
    assert _hash_of(tmp_path, other, "k_forward_p") == h0
    assert _hash_of(tmp_path, other, "k_adjoint_h16s") != bench.kernel_hash("k_adjoint_h16s")
    own = src[:body] + "\n    (void)0;\n" + src[body:]
    assert _hash_of(tmp_path, own, "k_forward_p") != h0


def test_unknown_kernel_is_an_error():
    with pytest.raises(ValueError):
        bench.kernel_hash("k_no_such_kernel")


def test_committed_traffic_matches_the_kernel_sources():
    """Every traffic figure in profiles/traffic.json was taken on the kernel
    source in the tree (the benchmark reports null for one that was not)."""
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        rec = json.load(f)
    assert rec
    for workload, kernels in rec.items():
        for k, ent in kernels.items():
            assert ent["kernel_hash"] == bench.kernel_hash(k), (workload, k)
            assert bench.traffic_from_profiles(k, workload) == ent["bytes_per_launch"]


def test_traffic_lookup_misses_return_null():
    assert bench.traffic_from_profiles("k_forward_p", "no-such-workload") is None


@pytest.mark.parametrize("name,fn,short", [
    ("void uvm::(anonymous namespace)::k_forward_p<float, 128, 256>(uvm::FwdPItem const*, double const*)",
     "k_forward_p", "void uvm::k_forward_p<float, 128, 256>"),
    ("_ZN3uvm12_GLOBAL__N_114k_adjoint_h16sIDF16bEEvPKNS_7AdjItemEPKdS6_PK15HIP_vector_typeIdLj2EEPKfS6_PKiPfii",
     "k_adjoint_h16s", "uvm::k_adjoint_h16s<__bf16>"),
    ("_ZN3uvm12_GLOBAL__N_114k_forward_h16mIDF16_Li128ELi256EEEvPKNS_8FwdPItemEPKdS6_PKfP15HIP_vector_typeIdLj2EEiix",
     "k_forward_h16m", "uvm::k_forward_h16m<_Float16, 128, 256>"),
    ("__amd_rocclr_copyBuffer", "__amd_rocclr_copyBuffer", "__amd_rocclr_copyBuffer"),
])
def test_kernel_name_parsing(name, fn, short):
    assert rocprof_summary._fname(name) == fn
    assert rocprof_summary._short(name) == short
