"""Command line: tune, train and score the schedule cost model on this GPU,
and write the model next to the package (``cost_model.json``).

    python -m paper_2206_07896_amd.train [--train-count 500] [--heldout 2000]
    python -m paper_2206_07896_amd.train --contention   # skewed-key histogram schedules only
"""

from .learned import main

if __name__ == "__main__":
    main()
