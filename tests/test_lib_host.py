"""Host-side tests of the native library (no GPU needed): the C ABI loads and
exports every declared entry point; the C++ symbolic analysis agrees bit for
bit with the oracle; malformed inputs are rejected."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1410_2697_amd as mfh
from mfinputs import q1_grid, p1_kuhn_cube, q1_elasticity
from oracle import symbolic

INCLUDE = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include")


def declared_functions():
    names = set()
    for h in os.listdir(INCLUDE):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(INCLUDE, h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(?:mf_status|void|const char\s*\*)\s*(\w+)\s*\(", src))
    return sorted(names)


def test_exports_every_declared_symbol():
    lib = mfh.load()
    names = declared_functions()
    assert "mf_analyze" in names and "gmres_solve" in names and "mf_apply" in names and "mf_factor" in names
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares them all
    assert set(names) == {s[0] for s in mfh.SIGNATURES}


def test_scratch_size_constant_matches_header():
    src = open(os.path.join(INCLUDE, "mfh.h")).read()
    m = re.search(r"#define MF_APPLY_SCRATCH_BYTES \((\d+)ull << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == mfh.MF_APPLY_SCRATCH_BYTES


CASES = [
    ("q1_2d_64_leaf64", lambda: q1_grid(64, 2), 64),
    ("q1_2d_20_leaf8", lambda: q1_grid(20, 2), 8),
    ("q1_3d_16_leaf128", lambda: q1_grid(16, 3), 128),
    ("q1_3d_11_leaf24", lambda: q1_grid(11, 3), 24),
    ("p1kuhn_9_leaf40", lambda: p1_kuhn_cube(9, 0.2, 7), 40),
    ("elasticity_7_leaf60", lambda: q1_elasticity(7), 60),
]


@pytest.mark.parametrize("name,maker,leaf", CASES)
def test_symbolic_bit_exact(name, maker, leaf):
    p = maker()
    _assert_symbolic_equal(p, leaf)


def _assert_symbolic_equal(p, leaf):
    """Every exported array of mf_analyze equals the oracle's analysis."""
    ref = symbolic.analyze(p.A, p.coords, leaf)
    s = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    assert np.array_equal(s.export(mfh.MF_EXP_PERM), ref.perm)
    fr = s.export(mfh.MF_EXP_FRONT).reshape(-1, 6)
    assert fr.shape[0] == ref.nfronts
    want = np.array([[f.start, f.npiv, f.nf, f.parent, f.height, len(f.children)] for f in ref.fronts])
    assert np.array_equal(fr, want)
    upd = s.export(mfh.MF_EXP_UPD)
    assert np.array_equal(upd, np.concatenate([f.upd for f in ref.fronts]))
    rm = s.export(mfh.MF_EXP_RELMAP)
    ref_rm = np.concatenate([f.relmap if f.relmap is not None else -np.ones(f.nf, dtype=np.int64)
                             for f in ref.fronts])
    assert np.array_equal(rm, ref_rm)
    asm = s.export(mfh.MF_EXP_ASM).reshape(-1, 4)
    assert np.array_equal(asm, np.stack([ref.asm_front, ref.asm_row, ref.asm_col, ref.asm_src], axis=1))
    blk = s.export(mfh.MF_EXP_BLOCKS).reshape(-1, 7)
    kinds = {"top": 0, "pp": 1, "ff": 2}
    want_b = np.array([[q, kinds[b.kind], b.r0, b.nr, b.c0, b.nc, b.level]
                       for q, f in enumerate(ref.fronts) for b in f.blocks])
    assert np.array_equal(blk, want_b)
    info = s.info()
    assert info["nfronts"] == ref.nfronts and info["nlevels"] == len(ref.levels)


@pytest.mark.parametrize("name,maker,leaf", CASES[1:])
@pytest.mark.parametrize("depth,cap", [(1, 1000), (3, 17), (-1, 40)])
def test_bdlr_sets_bit_exact(name, maker, leaf, depth, cap):
    p = maker()
    ref = symbolic.analyze(p.A, p.coords, leaf)
    s = mfh.Symbolic.from_csr(p.A, p.coords, leaf)
    s.bdlr(depth, cap)
    I, Ip = s.export(mfh.MF_EXP_BDLR_I), s.export(mfh.MF_EXP_BDLR_IPTR)
    J, Jp = s.export(mfh.MF_EXP_BDLR_J), s.export(mfh.MF_EXP_BDLR_JPTR)
    g = 0
    for f in ref.fronts:
        for b in f.blocks:
            ri, rj = symbolic.bdlr_sets(ref, f, b, depth, cap)
            assert np.array_equal(I[Ip[g]:Ip[g + 1]], ri)
            assert np.array_equal(J[Jp[g]:Jp[g + 1]], rj)
            g += 1
    assert g == Ip.shape[0] - 1


@pytest.mark.parametrize("name", ["q1_3d_64_leaf128", "p1kuhn_48_leaf128"])
def test_symbolic_bit_exact_full_size(name):
    """The analyses of the largest workloads, in full: the 64^3 Q1 grid (the
    pattern and coordinates of the 64^3 diffusion workload; its coefficient
    field changes only values) and the jittered Kuhn-P1 mesh of 48^3 cells
    with the generator's own seed."""
    if name.startswith("q1"):
        p = q1_grid(64, 3)
    else:
        from mfinputs import make_workload
        p = make_workload("p1kuhn_48").problem
    _assert_symbolic_equal(p, 128)


def test_symbolic_full_size_3d_32():
    p = q1_grid(32, 3)
    ref = symbolic.analyze(p.A, p.coords, 128)
    s = mfh.Symbolic.from_csr(p.A, p.coords, 128)
    assert np.array_equal(s.export(mfh.MF_EXP_PERM), ref.perm)
    assert np.array_equal(s.export(mfh.MF_EXP_UPD), np.concatenate([f.upd for f in ref.fronts]))


def test_malformed_csr_rejected():
    p = q1_grid(4, 2)
    rp, ci = p.A.rowptr.copy(), p.A.colind.copy()
    bad = ci.copy()
    bad[0], bad[1] = bad[1], bad[0]                    # unsorted row
    with pytest.raises(mfh.MfError) as e:
        mfh.Symbolic(p.A.n, rp, bad, p.coords, 4)
    assert e.value.status == mfh.MF_EINVAL
    bad = ci.copy()
    bad[3] = 99                                        # out of range
    with pytest.raises(mfh.MfError):
        mfh.Symbolic(p.A.n, rp, bad, p.coords, 4)
    # asymmetric pattern: drop one off-diagonal entry of row 0
    k = int(np.flatnonzero(ci[rp[0]:rp[1]] == 1)[0])
    ci2 = np.delete(ci, k)
    rp2 = rp.copy()
    rp2[1:] -= 1
    with pytest.raises(mfh.MfError):
        mfh.Symbolic(p.A.n, rp2, ci2, p.coords, 4)
    with pytest.raises(mfh.MfError):
        mfh.Symbolic(p.A.n, rp, ci, p.coords, 0)       # leaf 0


def test_factor_without_gpu_is_a_clean_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    p = q1_grid(6, 2)
    s = mfh.Symbolic.from_csr(p.A, p.coords, 8)
    lib = mfh.load()
    o = mfh.default_opts()
    h = ctypes.c_void_p()
    st = lib.mf_factor(s.h, mfh._ptr(p.A.vals), 1e-4, 0, ctypes.byref(o), ctypes.byref(h))
    assert st == mfh.MF_ESTATE
    assert b"no HIP device" in lib.mf_last_error()


def test_option_validation():
    p = q1_grid(6, 2)
    s = mfh.Symbolic.from_csr(p.A, p.coords, 8)
    lib = mfh.load()
    h = ctypes.c_void_p()
    for kw, eps in [({"precision": 7}, 1e-4), ({"method": 9}, 1e-4), ({}, -1.0), ({"bdlr_cap": -1}, 1e-4),
                    ({"bdlr_cap": 500}, 1e-4), ({"apply_split_chunk": 100}, 1e-4),
                    ({"apply_split_chunk": 8192}, 1e-4), ({"apply_split_target": -1}, 1e-4)]:
        o = mfh.default_opts(**kw)
        st = lib.mf_factor(s.h, mfh._ptr(p.A.vals), eps, 0, ctypes.byref(o), ctypes.byref(h))
        assert st == mfh.MF_EINVAL, (kw, eps)
    o = mfh.default_opts()
    assert lib.mf_factor(s.h, mfh._ptr(p.A.vals), 1e-4, 5, ctypes.byref(o), ctypes.byref(h)) == mfh.MF_EINVAL


def test_prof_start_stop_without_launches():
    """Kernel timing starts and stops on the host; with no launches nothing is reported."""
    import paper_1410_2697_amd as mfh
    mfh.prof_start(["gemm_kernel<float>", "no_such_kernel"])
    assert mfh.prof_stop() == []
    mfh.prof_start()
    assert mfh.prof_stop() == []


def test_estimate_bytes_dense_part_is_exact():
    """The estimator's dense-front factor bytes equal the sum over fronts of
    npiv^2 + nf*npiv entries (explicit inverse of L_pp plus L_fp), and the
    peak covers at least the front workspace of the largest level."""
    import paper_1410_2697_amd as mfh
    from mfinputs import q1_grid
    p = q1_grid(12, 3)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 32)
    e1 = mfh.estimate_bytes(sym, nrhs=1, restart=30, method="dense", precision="fp64")
    e2 = mfh.estimate_bytes(sym, nrhs=2, restart=30, method="dense", precision="fp64")
    ref = symbolic.analyze(p.A, p.coords, 32)
    dense = sum(f.npiv * f.npiv + f.nf * f.npiv for f in ref.fronts) * 8
    biggest_level = max(sum(ref.fronts[q].n * ref.fronts[q].n for q in lv) for lv in ref.levels) * 8
    assert e1["persistent_bytes"] > dense and e1["peak_bytes"] > dense + biggest_level
    # one more right-hand side adds apply and GMRES(30) workspaces only
    delta = e2["persistent_bytes"] - e1["persistent_bytes"]
    n = p.A.n
    assert delta >= 8 * n * 63 and delta < 8 * n * 63 + 8 * sum(f.n + f.npiv for f in ref.fronts) + 1
    eh = mfh.estimate_bytes(sym, nrhs=1, restart=30, method="hodlr", precision="fp32", n_c=64)
    assert 0 < eh["persistent_bytes"] and 0 < eh["peak_bytes"]


def test_estimate_bytes_sampled_drops_compressed_fronts():
    """Sampled extend-add: the compressed fronts leave the front workspace, so
    the estimated peak falls, while the persistent factor is the same."""
    import paper_1410_2697_amd as mfh
    from mfinputs import q1_grid
    p = q1_grid(24, 3)
    sym = mfh.Symbolic.from_csr(p.A, p.coords, 64)
    kw = dict(nrhs=1, restart=30, method="hodlr", precision="fp32", n_c=0, adaptive=0)
    ea = mfh.estimate_bytes(sym, sampled=0, **kw)
    es = mfh.estimate_bytes(sym, sampled=1, **kw)
    assert es["persistent_bytes"] == ea["persistent_bytes"]
    assert es["peak_bytes"] < ea["peak_bytes"]
    ref = symbolic.analyze(p.A, p.coords, 64)
    largest_front = max(f.n * f.n for f in ref.fronts) * 4
    assert ea["peak_bytes"] - es["peak_bytes"] > largest_front / 2


def test_symbolic_merge_is_the_shifted_union():
    """mf_symbolic_merge: the analysis of diag(A_1, A_2, A_3) is each part's
    own analysis with rows, fronts, blocks and CSR entries shifted by the
    parts before it; the levels are by height across parts."""
    parts_in = [(q1_grid(10, 3), 32), (p1_kuhn_cube(5, 0.2, 3), 32), (q1_grid(12, 3), 32)]
    parts = [mfh.Symbolic.from_csr(p.A, p.coords, leaf) for p, leaf in parts_in]
    for s in parts:
        s.bdlr(3, 48)
    m = mfh.Symbolic.merge(parts)
    m.bdlr(3, 48)
    infos = [s.info() for s in parts]
    mi = m.info()
    assert mi["n"] == sum(i["n"] for i in infos) and mi["nnz"] == sum(i["nnz"] for i in infos)
    assert mi["nfronts"] == sum(i["nfronts"] for i in infos)
    assert mi["nlevels"] == max(i["nlevels"] for i in infos)
    no = [0]; fo = [0]; eo = [0]; bo = [0]
    for s, i in zip(parts, infos):
        no.append(no[-1] + i["n"]); fo.append(fo[-1] + i["nfronts"]); eo.append(eo[-1] + i["nnz"])
        bo.append(bo[-1] + s.export(mfh.MF_EXP_BLOCKS).size // 7)

    def shifted(what, fn):
        return np.concatenate([fn(s.export(what), k) for k, s in enumerate(parts)])

    assert np.array_equal(m.export(mfh.MF_EXP_PERM), shifted(mfh.MF_EXP_PERM, lambda a, k: a + no[k]))

    def fr(a, k):
        a = a.reshape(-1, 6).copy()
        a[:, 0] += no[k]
        a[:, 3] = np.where(a[:, 3] >= 0, a[:, 3] + fo[k], -1)
        return a.ravel()
    assert np.array_equal(m.export(mfh.MF_EXP_FRONT), shifted(mfh.MF_EXP_FRONT, fr))
    assert np.array_equal(m.export(mfh.MF_EXP_UPD), shifted(mfh.MF_EXP_UPD, lambda a, k: a + no[k]))
    assert np.array_equal(m.export(mfh.MF_EXP_RELMAP), shifted(mfh.MF_EXP_RELMAP, lambda a, k: a))

    def blk(a, k):
        a = a.reshape(-1, 7).copy()
        a[:, 0] += fo[k]
        return a.ravel()
    assert np.array_equal(m.export(mfh.MF_EXP_BLOCKS), shifted(mfh.MF_EXP_BLOCKS, blk))

    def asm(a, k):
        a = a.reshape(-1, 4).copy()
        a[:, 0] += fo[k]
        a[:, 3] += eo[k]
        return a.ravel()
    assert np.array_equal(m.export(mfh.MF_EXP_ASM), shifted(mfh.MF_EXP_ASM, asm))
    for what in (mfh.MF_EXP_BDLR_I, mfh.MF_EXP_BDLR_J):   # front positions: unchanged
        assert np.array_equal(m.export(what), shifted(what, lambda a, k: a))
    # the fronts of one level come from every part whose tree reaches that height
    fm = m.export(mfh.MF_EXP_FRONT).reshape(-1, 6)
    for k in range(len(parts)):
        assert fm[fo[k]:fo[k + 1], 4].max() == infos[k]["nlevels"] - 1
        assert (fm[fo[k]:fo[k + 1], 3] == -1).sum() == 1          # one root per part


def test_symbolic_merge_rejects_bad_parts():
    a = mfh.Symbolic.from_csr(q1_grid(6, 3).A, q1_grid(6, 3).coords, 16)
    b = mfh.Symbolic.from_csr(q1_grid(6, 3).A, q1_grid(6, 3).coords, 24)
    c = mfh.Symbolic.from_csr(q1_grid(8, 2).A, q1_grid(8, 2).coords, 16)
    for bad in ([a, b], [a, c]):
        with pytest.raises(mfh.MfError) as e:
            mfh.Symbolic.merge(bad)
        assert e.value.status == mfh.MF_EINVAL
    lib = mfh.load()
    h = ctypes.c_void_p()
    assert lib.mf_symbolic_merge(None, 0, ctypes.byref(h)) == mfh.MF_EINVAL
    arr = (ctypes.c_void_p * 2)(a.h.value, None)
    assert lib.mf_symbolic_merge(arr, 2, ctypes.byref(h)) == mfh.MF_EINVAL
    m = mfh.Symbolic.merge([a])
    assert np.array_equal(m.export(mfh.MF_EXP_ASM), a.export(mfh.MF_EXP_ASM))


def test_no_kernel_spills_to_scratch():
    """Every device function of the library keeps its working set in
    registers and LDS: the compiler reports no scratch (private memory) for
    any of them.  The register-resident skeleton and Cholesky kernels slow
    down many times over when a change pushes their rows out to scratch."""
    import json
    path = os.path.join(os.path.dirname(os.path.dirname(__file__)), "_build", "kernel_resources.json")
    if not os.path.exists(path):
        pytest.skip("library not built here")
    res = json.load(open(path))
    assert any("skreg_kernel" in k for k in res) and any("gemm_narrow_kernel" in k for k in res)
    spills = {k: v for k, v in res.items() if v.get("ScratchSize", 0) > 0}
    assert not spills, spills


def test_tuned_options_reads_the_table(tmp_path):
    """autotune.tuned_options: nearest size bucket, the goal's eps/n_c/d, and
    for the settings that keep compressed fronts the tuned launch shape of
    the apply's GEMMs."""
    import json
    from paper_1410_2697_amd import autotune
    t = {"poisson3d": {"32768": {"solve": {"eps": 1e-3, "n_c": 4096, "depth": 3, "solve_ms": 1.0},
                                 "solve_hodlr": {"eps": 1e-4, "n_c": 1024, "depth": 3, "solve_ms": 2.0},
                                 "tiles": {"best": {"apply_split_chunk": 256, "apply_split_target": 2048,
                                                    "solve_ms": 1.9}}},
                       "262144": {"solve": {"eps": 1e-5, "n_c": 4096, "depth": -1, "solve_ms": 5.0}}}}
    path = tmp_path / "t.json"
    path.write_text(json.dumps(t))
    assert autotune.tuned_options("poisson3d", 30000, "solve", str(path)) == {"eps": 1e-3, "n_c": 4096, "depth": 3}
    assert autotune.tuned_options("poisson3d", 40000, "solve_hodlr", str(path)) == {
        "eps": 1e-4, "n_c": 1024, "depth": 3, "apply_split_chunk": 256, "apply_split_target": 2048}
    assert autotune.tuned_options("poisson3d", 250000, "solve", str(path))["eps"] == 1e-5
    assert autotune.tuned_options("poisson3d", 250000, "solve_hodlr", str(path)) is None
    assert autotune.tuned_options("p1kuhn", 1000, "solve", str(path)) is None
    for cls in ("poisson3d", "p1kuhn", "elasticity3d"):      # the committed table
        assert autotune.tuned_options(cls, 32768) is not None
