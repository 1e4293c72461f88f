"""sfhk_propagate_static (the propagation without a workspace argument, on
the library's static device array) against sfhk_propagate with a caller
workspace, through the C ABI: two calls in a row, the second with a smaller
input, in both precisions; and its size limits, checked on the host."""
import ctypes as C

import numpy as np
import pytest

import workloads


def _static(L, arr, n_prob, ens, precision, acc, fs, stream):
    return L.sfhk_propagate_static(arr, n_prob, C.byref(ens.struct()), precision,
                                   C.c_void_p(acc.data_ptr()),
                                   C.c_void_p(fs.data_ptr() if fs is not None else 0),
                                   None, 0, 1, stream)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_static_entry_equals_workspace_entry(precision):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2608_13686_amd as sf
    from paper_2608_13686_amd import _abi
    L = _abi.lib()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    cases = [([workloads.n2(0.0), workloads.n2(90.0)], [20000, 20000], [1002, 1002]),
             ([workloads.h2_softcore(30.0)], [3000], [1001])]
    for probs, n, seeds in cases:  # the second call is smaller than the first
        print(f"{precision}: {[p['name'] for p in probs]} x {n}", flush=True)
        ens, ws = sf.sample_initial(probs, n, seeds)
        acc_ref, fs_ref = sf.propagate(probs, ens, precision, final_state=True, workspace=ws)
        acc = torch.zeros_like(acc_ref)
        fs = torch.zeros_like(fs_ref)
        arr = _abi.make_problems(probs)
        _abi.check(_static(L, arr, len(probs), ens, sf.PRECISION[precision], acc, fs, stream),
                   "sfhk_propagate_static")
        torch.cuda.synchronize()
        a, b = acc.cpu().numpy(), acc_ref.cpu().numpy()
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        live = np.nonzero(ens.w.cpu().numpy() > 0)[0]
        same = np.array_equal(fs.cpu().numpy()[:, live], fs_ref.cpu().numpy()[:, live])
        print(f"  accum rel L2 {err:.2e}; final records of {live.size} live slots equal: {same}",
              flush=True)
        assert err < 1e-12  # only the order of the dipole atomics differs
        assert same


def test_static_entry_rejects_sizes_beyond_its_array():
    """Beyond 32 MiB of workspace or 1024 problems: SFHK_E_NOMEM and a message,
    before any device work (no device is touched here)."""
    from paper_2608_13686_amd import _abi
    L = _abi.lib()
    fake = 64  # never dereferenced: the calls fail first
    ens = _abi.Ensemble()
    for f in ("k0", "prob", "qx", "qy", "qz", "px", "py", "pz", "w", "nx", "ny", "nz", "dph",
              "order", "live_start", "live_count", "pack_start"):
        setattr(ens, f, fake)
    arr = _abi.make_problems([workloads.n2(0.0)])
    ens.capacity = 5 << 20  # 8 B per slot of mixed hand-over arrays: 40 MiB
    assert L.sfhk_propagate_static(arr, 1, C.byref(ens), _abi.MIXED, C.c_void_p(fake), None,
                                   None, 0, 1, None) == 2
    assert b"static workspace holds" in L.sfhk_last_error()
    arr = _abi.make_problems([workloads.h2_softcore()] * 1025)
    ens.capacity = 1000
    assert L.sfhk_propagate_static(arr, 1025, C.byref(ens), _abi.FP64, C.c_void_p(fake), None,
                                   None, 0, 1, None) == 2
    assert b"at most 1024 problems" in L.sfhk_last_error()
    # argument errors as for sfhk_propagate
    assert L.sfhk_propagate_static(arr, 1, C.byref(ens), 9, C.c_void_p(fake), None, None, 0, 1,
                                   None) == 1
