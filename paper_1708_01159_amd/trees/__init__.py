"""Decision trees shipped with the library (JSON, flat CART arrays).

``mi355x.json`` is trained on per-level kernel times measured on MI355X;
``seed.json`` is a hand-written starting point used until one is trained.
"""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def path(name: str) -> str:
    return os.path.join(HERE, name if name.endswith(".json") else name + ".json")


def default_path() -> str:
    p = path("mi355x")
    return p if os.path.exists(p) else path("seed")


def load_default():
    from ..gsw import Tree

    return Tree.load(default_path())
