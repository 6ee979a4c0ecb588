"""Host logic of the binding's allocators, without a GPU: torch's caching
allocator is replaced by a counter, so only the bookkeeping runs."""
import random
import threading
import time

import torch


def _fake_torch_pool(monkeypatch):
    nxt = [1 << 20]
    lock = threading.Lock()

    def alloc(nbytes, device, stream):
        time.sleep(0)   # give up the GIL inside the allocation, as a real one may
        with lock:
            nxt[0] += 1 << 12
            return nxt[0]

    monkeypatch.setattr(torch.cuda, "current_device", lambda: 0)
    monkeypatch.setattr(torch.cuda, "caching_allocator_alloc", alloc)
    monkeypatch.setattr(torch.cuda, "caching_allocator_delete", lambda ptr: None)


def test_budget_allocator_holds_its_budget_across_threads(monkeypatch):
    # the service's query threads allocate snapshots while the update thread
    # allocates batch scratch: the budget check, the allocation and the count
    # must be one step, or two requests can both pass the check
    from paper_1709_05061_amd.service import BudgetAllocator
    _fake_torch_pool(monkeypatch)
    budget = 20000
    a = BudgetAllocator(budget)
    refused = [0]

    def worker(seed):
        rng = random.Random(seed)
        held = []
        for _ in range(400):
            n = rng.randrange(500, 4000)
            p = a.struct.alloc(n, None, None)   # through the C callback, as the library calls it
            if p:
                held.append((p, n))
            else:
                refused[0] += 1
            if held and rng.random() < 0.5:
                q, m = held.pop(rng.randrange(len(held)))
                a.struct.free(q, m, None, None)
        for q, m in held:
            a.struct.free(q, m, None, None)

    threads = [threading.Thread(target=worker, args=(s,)) for s in range(16)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert a.peak_bytes <= budget
    assert a.held_bytes == 0
    assert refused[0] > 0   # the budget was reached
