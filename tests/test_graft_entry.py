"""__graft_entry__.build() reaches every compile step (generators, oracle, library)
and imports the package; the compilers themselves are replaced by recorders here."""
import importlib
import types

import __graft_entry__ as entry


def test_build_calls_every_compile_step(monkeypatch):
    import oracle
    import synth

    calls = []
    monkeypatch.setattr(synth, "build_lib", lambda force=True: calls.append("synth"))
    monkeypatch.setattr(oracle, "build_lib", lambda force=True: calls.append("oracle"))
    libbuild = importlib.import_module("paper_2201_12523_amd.buildlib")
    monkeypatch.setattr(libbuild, "build", lambda verbose=True: calls.append("library"))
    import paper_2201_12523_amd as pkg

    monkeypatch.setattr(pkg, "lib", lambda: calls.append("load"))
    entry.build()
    assert calls == ["synth", "oracle", "library", "load"]
    # importing the compile step leaves the package's tensor builder in place
    assert not isinstance(pkg.build, types.ModuleType) and pkg.build.__name__ == "build"
