"""Graph operations on the undirected graphical model.

* fixing a vertex's value removes the vertex and its edges (Section
  "Parallelization by fixing the values of variables", Fig. 5);
* eliminating a vertex connects every pair of its neighbours and then
  removes it (Section "Variable elimination", step 4; Fig. 6); the tensor it
  produces has rank deg(v), so its size is 2^deg(v), the per-step cost
  estimate of the same section.
"""
from __future__ import annotations


class Graph:
    def __init__(self, vertices=(), edges=()):
        self.adj = {v: set() for v in vertices}
        for a, b in edges:
            self.add_edge(a, b)

    def copy(self) -> "Graph":
        g = Graph()
        g.adj = {v: set(n) for v, n in self.adj.items()}
        return g

    def add_edge(self, a, b):
        if a == b:
            return
        self.adj.setdefault(a, set()).add(b)
        self.adj.setdefault(b, set()).add(a)

    @property
    def vertices(self):
        return set(self.adj)

    @property
    def edges(self):
        return {(a, b) if a < b else (b, a) for a in self.adj for b in self.adj[a]}

    def degree(self, v) -> int:
        return len(self.adj[v])

    def fix(self, v) -> None:
        for u in self.adj.pop(v):
            self.adj[u].discard(v)

    def eliminate(self, v) -> int:
        """Eliminate v; returns the rank deg(v) of the tensor it creates."""
        nb = sorted(self.adj[v])
        for i in range(len(nb)):
            for j in range(i + 1, len(nb)):
                self.add_edge(nb[i], nb[j])
        self.fix(v)
        return len(nb)

    def fill_in(self, v) -> int:
        nb = sorted(self.adj[v])
        missing = 0
        for i in range(len(nb)):
            for j in range(i + 1, len(nb)):
                if nb[j] not in self.adj[nb[i]]:
                    missing += 1
        return missing
