"""bench.py's calls into the Python binding name only arguments that the
binding's methods take (a renamed keyword would otherwise surface only when
that benchmark mode runs on a GPU).  Host-only: reads the source and the
binding's signatures, launches nothing."""
import ast
import inspect
import os

from paper_2004_13887_amd import dsw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _tree():
    return ast.parse(open(os.path.join(ROOT, "bench.py")).read())


def _receivers(tree):
    """names bench.py binds to a Grid or an Ensemble of the binding"""
    out = {}
    for node in ast.walk(tree):
        if isinstance(node, ast.Assign) and isinstance(node.value, ast.Call):
            f = ast.unparse(node.value.func)
            cls = dsw.Grid if f.startswith("dsw.Grid") else dsw.Ensemble if f.startswith("dsw.Ensemble") else None
            if cls is not None:
                for t in node.targets:
                    if isinstance(t, ast.Name):
                        out[t.id] = cls
    return out


def _calls(tree):
    """method calls on those names: (call node, class)"""
    rec = _receivers(tree)
    for node in ast.walk(tree):
        if (isinstance(node, ast.Call) and isinstance(node.func, ast.Attribute)
                and isinstance(node.func.value, ast.Name) and node.func.value.id in rec):
            yield node, rec[node.func.value.id]


def test_bench_keywords_match_binding():
    tree = _tree()
    assert set(_receivers(tree).values()) == {dsw.Grid, dsw.Ensemble}
    checked, bad = 0, []
    for node, cls in _calls(tree):
        meth = getattr(cls, node.func.attr, None)
        assert meth is not None, f"bench.py:{node.lineno} {cls.__name__} has no {node.func.attr}"
        params = inspect.signature(meth).parameters
        has_var_kw = any(p.kind is p.VAR_KEYWORD for p in params.values())
        for kw in node.keywords:
            if kw.arg is None or has_var_kw:
                continue
            checked += 1
            if kw.arg not in params:
                bad.append(f"bench.py:{node.lineno} {cls.__name__}.{node.func.attr}({kw.arg}=...)")
    assert checked > 0
    assert not bad, bad


def test_bench_forced_passes_both_wall_levels():
    # the forced step takes the wall velocities at t^n and at t^{n+1}
    params = inspect.signature(dsw.Grid.split_step_forced).parameters
    assert "wall0" in params and "wall1" in params
    kws = set()
    for node, _ in _calls(_tree()):
        if node.func.attr == "split_step_forced":
            kws |= {kw.arg for kw in node.keywords}
    assert {"wall0", "wall1", "src", "bnd"} <= kws
