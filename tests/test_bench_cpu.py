"""Host-side checks of bench.py that need no GPU: every module-level name
the script uses is defined (a missing helper would only surface at the end of
a long GPU run), and a request for more than one GPU exits with a message."""
import ast
import builtins
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _bound_names(tree):
    names = set(dir(builtins))
    for node in ast.walk(tree):
        if isinstance(node, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            names.add(node.name)
            a = node.args if not isinstance(node, ast.ClassDef) else None
            if a is not None:
                for arg in a.posonlyargs + a.args + a.kwonlyargs:
                    names.add(arg.arg)
                for arg in (a.vararg, a.kwarg):
                    if arg is not None:
                        names.add(arg.arg)
        elif isinstance(node, ast.Lambda):
            for arg in node.args.args + node.args.kwonlyargs:
                names.add(arg.arg)
        elif isinstance(node, (ast.Import, ast.ImportFrom)):
            for al in node.names:
                names.add((al.asname or al.name).split(".")[0])
        elif isinstance(node, ast.Name) and isinstance(node.ctx, (ast.Store, ast.Del)):
            names.add(node.id)
        elif isinstance(node, ast.ExceptHandler) and node.name:
            names.add(node.name)
        elif isinstance(node, (ast.Global, ast.Nonlocal)):
            names.update(node.names)
    return names


def test_bench_names_are_defined():
    tree = ast.parse(open(BENCH).read())
    bound = _bound_names(tree) | {"__file__", "__name__"}
    used = {n.id for n in ast.walk(tree) if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load)}
    assert not sorted(used - bound), f"bench.py uses undefined names: {sorted(used - bound)}"


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_oracle_rows_on_samples():
    # the per-line oracle timing of the bench runs on the host alone: every
    # line it knows gets a positive rate and a stated sample
    sys.path.insert(0, ROOT)
    import bench
    from paper_1604_04815_amd import workloads

    keys = ["int64_add_2p27", "int32_max_2p28", "float32_add_2p27", "float32_add_2p27_compensated",
            "bf16_add_2p27", "bf16_add_2p27_compensated", "segmented_4096_int32_add", "compact_int32_2p28_half",
            "argmax_int32_2p28", "radix_offsets_int32_2p28_8bit", "custom_affine_2p27", "bfs_rmat22"]
    configs = {k: {} for k in keys}
    configs["serving"] = {}
    bench.cpu_oracle_rows(workloads, configs)
    for k in keys:
        row = configs[k]["oracle_cpu"]
        assert row["gelem_s"] > 0 and row["cores"] == 1 and row["sample"], k
    assert "oracle_cpu" not in configs["serving"]


def test_float_error_ratio_by_hand():
    # bench.float_error on host tensors: y = [1, 3, 2.5] against exact
    # prefixes [1, 2, 2.5] of x = [1, 1, 0.5] -> errors [0, 1, 0] over
    # A = [1, 2, 2.5]: ratio 0.5 at j = 1; segmented with offsets [0, 1, 3]:
    # second segment prefixes [1, 1.5], y[1:] = [1, 2] -> ratio 0.5/1.5 at 2
    import torch

    sys.path.insert(0, ROOT)
    import bench

    x = torch.tensor([1.0, 1.0, 0.5], dtype=torch.float32)
    r = bench.float_error(x, torch.tensor([1.0, 3.0, 2.5]))
    assert r["argmax"] == 1 and abs(r["max_error_ratio"] - 0.5) < 1e-12
    r = bench.float_error(x, torch.tensor([1.0, 1.0, 2.0]), torch.tensor([0, 1, 3]))
    assert r["argmax"] == 2 and abs(r["max_error_ratio"] - 0.5 / 1.5) < 1e-12
    r = bench.float_error(x, torch.tensor([1.0, 2.0, 2.5]))
    assert r["max_error_ratio"] == 0.0
    # a zero prefix sum of magnitudes admits only an exact zero
    z = torch.tensor([0.0, 0.0], dtype=torch.float32)
    assert bench.float_error(z, torch.tensor([0.0, 1e-30]))["max_error_ratio"] == float("inf")
